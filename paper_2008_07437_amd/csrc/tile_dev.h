// Device access to the tile storage of a matrix (lower tiles, column-major
// inside a tile, per-tile byte offsets and kinds).
#pragma once

#include "mvgeo_internal.h"

namespace mvg {

__device__ __forceinline__ double *tile_ptr(TileMap M, int I, int J) {
  return reinterpret_cast<double *>(M.base + M.off[tidx(I, J, M.T)]);
}
__device__ __forceinline__ float *tile_ptr_f32(TileMap M, int I, int J) {
  return reinterpret_cast<float *>(M.base + M.off[tidx(I, J, M.T)]);
}
__device__ __forceinline__ bool tile_is_f32(TileMap M, int I, int J) {
  return M.kind && M.kind[tidx(I, J, M.T)] == TK_F32;
}

}  // namespace mvg
