// Mixed-precision tiled Cholesky and FP64 iterative refinement on gfx950.
//
// Not in the paper: the paper's factorisation is FP64 throughout (Section 5).
// Here tiles within `band` tile-diagonals of the diagonal stay FP64 (including
// every diagonal-tile factorisation, the log-determinant and the solve's
// refinement), while off-band tiles are stored in FP32 and updated on FP32
// MFMA (v_mfma_f32_16x16x4_f32), or on BF16 operands with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16).  Per step k:
//   panel TRSM: band tiles as the FP64 GEMM against W_k, off-band tiles as an
//   FP32 GEMM against W_k rounded to FP32;
//   the solved panel is staged once as FP64 (exact upcast), FP32 and, for
//   BF16, as row-major BF16 (round to nearest even from the FP32 value);
//   trailing update: band targets on FP64 MFMA, off-band targets on FP32 /
//   BF16 MFMA;
//   the look-ahead stream factors the next diagonal tile in FP64.
// FP32X keeps every tile in FP64 and solves every panel in FP64; only the
// off-band trailing GEMMs run on FP32 MFMA (operands rounded from the FP64
// panel, 16-product stage sums added to the FP64 tile).  BF16X3 is FP32X
// with each off-band operand split into two BF16 terms and each product
// formed from three BF16 MFMAs (FP32 accumulation, added to the FP64 tile).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "mvgeo_internal.h"

namespace mvg {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int LB = 128;   // output block
constexpr int LK32 = 16;  // K slice per stage, FP32 operands (8 KB per operand)
constexpr int LK16 = 32;  // K slice per stage, BF16 operands (8 KB per operand)
constexpr int LS = 4;     // pipeline stages

#define MVG_LDSP(p) ((__attribute__((address_space(3))) void *)(p))

__device__ __forceinline__ void lp_wait_vmcnt_8() { __builtin_amdgcn_s_waitcnt(0x0F78); }
__device__ __forceinline__ void lp_wait_vmcnt_0() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ char *tile_bytes(TileMap M, int I, int J) {
  return M.base + M.off[tidx(I, J, M.T)];
}

__device__ __forceinline__ int64_t lp_xcd_remap(int64_t bid, int64_t pad) {
  const int64_t per = pad >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// UPDATE: FP32 target tile; TRSM: off-band panel solve into an FP32 tile;
// UPDATE64: FP64 target tile (FP32 operands, FP64 storage).
enum { LP_UPDATE = 0, LP_TRSM = 1, LP_UPDATE64 = 2 };

// Off-band target tiles of step k, enumerated column by column: (i, j) with
// j > k and i >= j + band.
__device__ __forceinline__ void lp_offband(const TileMap &M, int k, int band, int64_t q, int &i,
                                           int &j) {
  j = k + 1;
  while (q >= (int64_t)max(0, M.T - j - band)) {
    q -= max(0, M.T - j - band);
    ++j;
  }
  i = j + band + (int)q;
}

// ------------------------------------------------------------ FP32 GEMM
//
// 128 x 128 output block of a tile; 4 waves in a 2 x 2 grid of 64 x 64.
// UPDATE (FP32 tile) and UPDATE64 (FP64 tile): C -= A B^T with A, B the
// staged FP32 panel; TRSM: C = A W^T with A
// the pre-TRSM copy of the tile and W = W_k in FP32 (lower triangular, only
// the first (sc+1)*128 columns of K contribute).  Accumulator layout of
// v_mfma_f32_16x16x4_f32: lane l, element e <-> D[4(l/16) + e][l%16].
template <int NB, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_lowp_f32(
    TileMap M, int k, int band, int64_t nwg, int64_t pad, const float *__restrict__ P32,
    const float *__restrict__ W32) {
  __shared__ float sA0[LK32 * LB], sA1[LK32 * LB], sA2[LK32 * LB], sA3[LK32 * LB];
  __shared__ float sB0[LK32 * LB], sB1[LK32 * LB], sB2[LK32 * LB], sB3[LK32 * LB];
#define LP_STA(u) ((u) == 0 ? sA0 : (u) == 1 ? sA1 : (u) == 2 ? sA2 : sA3)
#define LP_STB(u) ((u) == 0 ? sB0 : (u) == 1 ? sB1 : (u) == 2 ? sB2 : sB3)
  const int64_t lid = lp_xcd_remap(blockIdx.x, pad);
  if (lid >= nwg) return;
  constexpr int s = NB / LB, ss = s * s;
  const int64_t q = lid / ss;
  const int sub = (int)(lid % ss), sr = sub % s, sc = sub / s;
  typedef typename std::conditional<MODE == LP_UPDATE64, double, float>::type CT;
  constexpr bool upd = MODE != LP_TRSM;
  const float *A, *B;
  CT *C;
  int nk;
  if (upd) {
    int i, j;
    lp_offband(M, k, band, q, i, j);
    A = P32 + (int64_t)(i - k - 1) * NB * NB + sr * LB;
    B = P32 + (int64_t)(j - k - 1) * NB * NB + sc * LB;
    C = reinterpret_cast<CT *>(tile_bytes(M, i, j)) + (int64_t)sc * LB * NB + sr * LB;
    nk = NB / LK32;
  } else {
    const int i = k + band + (int)q;
    A = P32 + (int64_t)(i - k - 1) * NB * NB + sr * LB;
    B = W32 + sc * LB;
    C = reinterpret_cast<CT *>(tile_bytes(M, i, k)) + (int64_t)sc * LB * NB + sr * LB;
    nk = (sc + 1) * (LB / LK32);
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 1, wc = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
  // a direct load moves 1 KB = two 128-float columns: lanes 0-31 the first,
  // lanes 32-63 the second; per stage 8 such loads for A and 8 for B, wave w
  // issues the loads w, w + 4, w + 8, w + 12.
  const int64_t lsrc = (int64_t)(lane >> 5) * NB + (lane & 31) * 4;
#define LP_ISSUE(kb, st)                                                                        \
  do {                                                                                          \
    _Pragma("unroll") for (int i_ = 0; i_ < 4; ++i_) {                                          \
      const int q_ = wave + 4 * i_;                                                             \
      const int pr_ = q_ & 7;                                                                   \
      const float *src_ = ((q_ < 8) ? A : B) + (int64_t)((kb) * LK32 + 2 * pr_) * NB + lsrc;    \
      float *dst_ = ((q_ < 8) ? LP_STA(st) : LP_STB(st)) + 2 * pr_ * LB;                        \
      __builtin_amdgcn_global_load_lds((const void *)src_, MVG_LDSP(dst_), 16, 0, 0);           \
    }                                                                                           \
  } while (0)
#pragma unroll
  for (int p = 0; p < LS - 1; ++p) LP_ISSUE(p, p);
  // Each stage's 16 products per entry are summed on the FP32 MFMA from zero;
  // the stage sums are added in FP64 and the tile is rounded to FP32 once
  // (a K-long FP32 accumulation chain would add about sqrt(K) times the
  // rounding noise of the stored result).
  dbl4 acc[4][4];
  const int64_t coff = (int64_t)(wc * 64 + l16) * NB + wr * 64 + 4 * lk;
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      if (MODE == LP_UPDATE64) {
        acc[ti][tj] = *reinterpret_cast<const dbl4 *>(C + coff + (int64_t)tj * 16 * NB + ti * 16);
      } else if (MODE == LP_UPDATE) {
        const flt4 c = *reinterpret_cast<const flt4 *>(C + coff + (int64_t)tj * 16 * NB + ti * 16);
        acc[ti][tj] = dbl4{(double)c[0], (double)c[1], (double)c[2], (double)c[3]};
      } else {
        acc[ti][tj] = dbl4{0.0, 0.0, 0.0, 0.0};
      }
    }
  for (int kb0 = 0; kb0 < nk; kb0 += LS) {
#pragma unroll
    for (int u = 0; u < LS; ++u) {
      const int kb = kb0 + u;
      lp_wait_vmcnt_8();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("" ::: "memory");
      const int p = kb + LS - 1;
      // as in the FP64 update: the first k-step's fragments are read, then
      // the refill issued, at raised priority
      __builtin_amdgcn_s_setprio(1);
      const float *a = LP_STA(u) + wr * 64 + l16;
      const float *bb = LP_STB(u) + wc * 64 + l16;
      float af0[4], bf0[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        af0[t] = upd ? -a[lk * LB + t * 16] : a[lk * LB + t * 16];
        bf0[t] = bb[lk * LB + t * 16];
      }
      LP_ISSUE(p < nk ? p : nk - 1, (u + LS - 1) % LS);
      __builtin_amdgcn_s_setprio(0);
      flt4 part[4][4];
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) part[ti][tj] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < LK32; ks += 4) {
        float af[4], bf[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          af[t] = ks == 0 ? af0[t]
                          : (upd ? -a[(ks + lk) * LB + t * 16] : a[(ks + lk) * LB + t * 16]);
          bf[t] = ks == 0 ? bf0[t] : bb[(ks + lk) * LB + t * 16];
        }
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
          for (int tj = 0; tj < 4; ++tj)
            part[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[ti], bf[tj], part[ti][tj], 0, 0, 0);
      }
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[ti][tj][e] += (double)part[ti][tj][e];
    }
  }
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      const dbl4 v = acc[ti][tj];
      if (MODE == LP_UPDATE64)
        *reinterpret_cast<dbl4 *>(C + coff + (int64_t)tj * 16 * NB + ti * 16) = v;
      else
        *reinterpret_cast<flt4 *>(C + coff + (int64_t)tj * 16 * NB + ti * 16) =
            flt4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    }
  lp_wait_vmcnt_0();
#undef LP_ISSUE
#undef LP_STA
#undef LP_STB
}

// ------------------------------------------------------------ BF16 GEMM
//
// Off-band update C (FP32) -= A B^T with A, B the panel staged as row-major
// BF16 (row r of a tile holds its nb values contiguously).  K slices of 32;
// each lane's MFMA operand is 8 consecutive K values of one row, one 16-byte
// LDS read.  FP32 accumulation in the same layout as the FP32 kernel.
template <int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_lowp_bf16(
    TileMap M, int k, int band, int64_t nwg, int64_t pad, const uint16_t *__restrict__ P16) {
  __shared__ uint16_t sA0[LK16 * LB], sA1[LK16 * LB], sA2[LK16 * LB], sA3[LK16 * LB];
  __shared__ uint16_t sB0[LK16 * LB], sB1[LK16 * LB], sB2[LK16 * LB], sB3[LK16 * LB];
#define LP_STA(u) ((u) == 0 ? sA0 : (u) == 1 ? sA1 : (u) == 2 ? sA2 : sA3)
#define LP_STB(u) ((u) == 0 ? sB0 : (u) == 1 ? sB1 : (u) == 2 ? sB2 : sB3)
  const int64_t lid = lp_xcd_remap(blockIdx.x, pad);
  if (lid >= nwg) return;
  constexpr int s = NB / LB, ss = s * s;
  const int64_t q = lid / ss;
  const int sub = (int)(lid % ss), sr = sub % s, sc = sub / s;
  int i, j;
  lp_offband(M, k, band, q, i, j);
  const uint16_t *A = P16 + (int64_t)(i - k - 1) * NB * NB + (int64_t)sr * LB * NB;
  const uint16_t *B = P16 + (int64_t)(j - k - 1) * NB * NB + (int64_t)sc * LB * NB;
  float *C = reinterpret_cast<float *>(tile_bytes(M, i, j)) + (int64_t)sc * LB * NB + sr * LB;
  constexpr int nk = NB / LK16;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 1, wc = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
  // a direct load moves 16 rows x 64 bytes (32 BF16 of K): lane l row l/4,
  // 16-byte chunk l%4; 8 loads per operand per stage.
  const int64_t lsrc = (int64_t)(lane >> 2) * NB + (lane & 3) * 8;
#define LP_ISSUE(kb, st)                                                                       \
  do {                                                                                         \
    _Pragma("unroll") for (int i_ = 0; i_ < 4; ++i_) {                                         \
      const int q_ = wave + 4 * i_;                                                            \
      const int pr_ = q_ & 7;                                                                  \
      const uint16_t *src_ = ((q_ < 8) ? A : B) + (int64_t)(16 * pr_) * NB + (kb) * LK16 + lsrc; \
      uint16_t *dst_ = ((q_ < 8) ? LP_STA(st) : LP_STB(st)) + 16 * pr_ * LK16;                 \
      __builtin_amdgcn_global_load_lds((const void *)src_, MVG_LDSP(dst_), 16, 0, 0);          \
    }                                                                                          \
  } while (0)
#pragma unroll
  for (int p = 0; p < LS - 1; ++p) LP_ISSUE(p, p);
  flt4 acc[4][4];
  const int64_t coff = (int64_t)(wc * 64 + l16) * NB + wr * 64 + 4 * lk;
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
      acc[ti][tj] = *reinterpret_cast<const flt4 *>(C + coff + (int64_t)tj * 16 * NB + ti * 16);
  for (int kb0 = 0; kb0 < nk; kb0 += LS) {
#pragma unroll
    for (int u = 0; u < LS; ++u) {
      const int kb = kb0 + u;
      lp_wait_vmcnt_8();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("" ::: "memory");
      const int p = kb + LS - 1;
      // the fragments are read, then the refill issued, at raised priority
      __builtin_amdgcn_s_setprio(1);
      bf16x8 af[4], bf[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        uint4 va = *reinterpret_cast<const uint4 *>(LP_STA(u) + (wr * 64 + t * 16 + l16) * LK16 + lk * 8);
        va.x ^= 0x80008000u;  // -A: flip the eight sign bits
        va.y ^= 0x80008000u;
        va.z ^= 0x80008000u;
        va.w ^= 0x80008000u;
        const uint4 vb = *reinterpret_cast<const uint4 *>(LP_STB(u) + (wc * 64 + t * 16 + l16) * LK16 + lk * 8);
        af[t] = __builtin_bit_cast(bf16x8, va);
        bf[t] = __builtin_bit_cast(bf16x8, vb);
      }
      LP_ISSUE(p < nk ? p : nk - 1, (u + LS - 1) % LS);
      __builtin_amdgcn_s_setprio(0);
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ti], bf[tj], acc[ti][tj], 0, 0, 0);
    }
  }
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
      *reinterpret_cast<flt4 *>(C + coff + (int64_t)tj * 16 * NB + ti * 16) = acc[ti][tj];
  lp_wait_vmcnt_0();
#undef LP_ISSUE
#undef LP_STA
#undef LP_STB
}

// ------------------------------------------------------ split-BF16 GEMM
//
// Off-band update of an FP64 target tile, C -= A B^T, with every operand
// value a split into two BF16 terms, a = a_hi + a_lo with |a - a_hi - a_lo|
// <= 2^-17 |a| (a_hi the BF16 rounding of the FP32 value, a_lo that of the
// remainder, which is exact in FP32; both staged row-major like the BF16
// panel).  Each product is formed from three BF16 MFMAs, a_hi b_hi +
// a_hi b_lo + a_lo b_hi (the dropped a_lo b_lo is at most 2^-16 of the
// product), accumulated in FP32 over the whole K and added to the FP64 tile
// once: a product error of at most about 2^-15 relative, against FP32
// operands' 2^-23 and BF16 operands' 2^-7, at three BF16 MFMAs per product.
// NS stages of 32 K values (four 8 KB planes each): two stages take 64 KB
// of LDS (two workgroups per CU), three 96 KB (one).  Measured at n = 50,000
// (tile 1024): two stages 262 TFLOP/s of useful flops, three 192.
constexpr int X3_STAGES = 2;

template <int NB, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NS == 2 ? 2 : 1, NS == 2 ? 2 : 1))) void k_lowp_bf16x3(
    TileMap M, int k, int band, int64_t nwg, int64_t pad, const uint16_t *__restrict__ Phi,
    const uint16_t *__restrict__ Plo) {
  static_assert(NS == 2 || NS == 3, "two or three stages");
  __shared__ uint16_t sbuf[NS][4][LK16 * LB];  // stage, plane (A_hi, A_lo, B_hi, B_lo)
  const int64_t lid = lp_xcd_remap(blockIdx.x, pad);
  if (lid >= nwg) return;
  constexpr int s = NB / LB, ss = s * s;
  const int64_t q = lid / ss;
  const int sub = (int)(lid % ss), sr = sub % s, sc = sub / s;
  int i, j;
  lp_offband(M, k, band, q, i, j);
  const int64_t ao = (int64_t)(i - k - 1) * NB * NB + (int64_t)sr * LB * NB;
  const int64_t bo = (int64_t)(j - k - 1) * NB * NB + (int64_t)sc * LB * NB;
  double *C = reinterpret_cast<double *>(tile_bytes(M, i, j)) + (int64_t)sc * LB * NB + sr * LB;
  constexpr int nk = NB / LK16;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 1, wc = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
  // a direct load moves 16 rows x 64 bytes (32 BF16 of K): lane l row l/4,
  // 16-byte chunk l%4; per stage 8 loads per plane, wave w issues the loads
  // w + 4 i of the 32 (planes A_hi, A_lo, B_hi, B_lo in that order).  Every
  // stage issues its 8 loads per wave (a slice past the end reloads the last
  // one into the stage that is free), so the count in flight is the same at
  // every wait.
  const int64_t lsrc = (int64_t)(lane >> 2) * NB + (lane & 3) * 8;
  auto issue = [&](int kb, int st) {
#pragma unroll
    for (int i_ = 0; i_ < 8; ++i_) {
      const int q_ = wave + 4 * i_;
      const int pl_ = q_ >> 3, pr_ = q_ & 7;  // plane, 16-row group
      const uint16_t *src_ = (pl_ & 1 ? Plo : Phi) + (pl_ < 2 ? ao : bo) +
                             (int64_t)(16 * pr_) * NB + kb * LK16 + lsrc;
      __builtin_amdgcn_global_load_lds((const void *)src_,
                                       MVG_LDSP(&sbuf[st][pl_][16 * pr_ * LK16]), 16, 0, 0);
    }
  };
#pragma unroll
  for (int p = 0; p < NS - 1; ++p) issue(p < nk ? p : nk - 1, p);
  flt4 acc[4][4];
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = flt4{0.f, 0.f, 0.f, 0.f};
  for (int kb = 0; kb < nk; ++kb) {
    const int u = kb % NS;
    // slice kb has landed (the later stage's 8 loads may still be in flight)
    if (NS == 2)
      lp_wait_vmcnt_0();
    else
      lp_wait_vmcnt_8();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
    const uint16_t *sAh = sbuf[u][0], *sAl = sbuf[u][1], *sBh = sbuf[u][2], *sBl = sbuf[u][3];
    // the fragments are read, then the refill issued, at raised priority
    __builtin_amdgcn_s_setprio(1);
    bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ar = (wr * 64 + t * 16 + l16) * LK16 + lk * 8;
      const int br = (wc * 64 + t * 16 + l16) * LK16 + lk * 8;
      uint4 vh = *reinterpret_cast<const uint4 *>(sAh + ar);
      uint4 vl = *reinterpret_cast<const uint4 *>(sAl + ar);
      vh.x ^= 0x80008000u;  // -A: flip the eight sign bits of each term
      vh.y ^= 0x80008000u;
      vh.z ^= 0x80008000u;
      vh.w ^= 0x80008000u;
      vl.x ^= 0x80008000u;
      vl.y ^= 0x80008000u;
      vl.z ^= 0x80008000u;
      vl.w ^= 0x80008000u;
      ah[t] = __builtin_bit_cast(bf16x8, vh);
      al[t] = __builtin_bit_cast(bf16x8, vl);
      bh[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(sBh + br));
      bl[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(sBl + br));
    }
    {
      const int nxt = kb + NS - 1;  // into the stage every wave finished before this barrier
      issue(nxt < nk ? nxt : nk - 1, nxt % NS);
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ti], bh[tj], acc[ti][tj], 0, 0, 0);
        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ti], bl[tj], acc[ti][tj], 0, 0, 0);
        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ti], bh[tj], acc[ti][tj], 0, 0, 0);
      }
  }
  lp_wait_vmcnt_0();  // no direct LDS load outlives the workgroup
  const int64_t coff = (int64_t)(wc * 64 + l16) * NB + wr * 64 + 4 * lk;
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      dbl4 *c = reinterpret_cast<dbl4 *>(C + coff + (int64_t)tj * 16 * NB + ti * 16);
      const dbl4 v = *c;
      *c = dbl4{v[0] + (double)acc[ti][tj][0], v[1] + (double)acc[ti][tj][1],
                v[2] + (double)acc[ti][tj][2], v[3] + (double)acc[ti][tj][3]};
    }
}

// ------------------------------------------------------------ panel staging

// Before the TRSM: the panel tiles (i, k), i > k, copied as stored: FP64
// tiles into P64 slot i-k-1, FP32 tiles into P32 slot i-k-1.
__global__ void k_panel_stage_pre(TileMap M, int k, double *__restrict__ P64,
                                  float *__restrict__ P32) {
  const int nb = M.nb;
  const int i = k + 1 + blockIdx.y;
  const int64_t t = tidx(i, k, M.T);
  const int64_t per = (int64_t)nb * nb;
  const char *src = M.base + M.off[t];
  if (M.kind[t] == TK_F32) {
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    float4 *d4 = reinterpret_cast<float4 *>(P32 + (int64_t)blockIdx.y * per);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per / 4;
         e += (int64_t)gridDim.x * blockDim.x)
      d4[e] = s4[e];
  } else {
    const double2 *s2 = reinterpret_cast<const double2 *>(src);
    double2 *d2 = reinterpret_cast<double2 *>(P64 + (int64_t)blockIdx.y * per);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per / 2;
         e += (int64_t)gridDim.x * blockDim.x)
      d2[e] = s2[e];
  }
}

__global__ void k_to_f32(const double *__restrict__ src, float *__restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// After the TRSM: every panel tile as FP64 (P64, column-major), FP32 (P32,
// column-major) and, if P16, BF16 row-major (rounded from the FP32 value);
// if P16lo, P16 holds the high BF16 term of the split and P16lo the BF16
// rounding of the remainder (exact in FP32).  One workgroup per 64 x 64
// block, transposed through LDS for P16.
__global__ __launch_bounds__(256) void k_panel_stage_post(TileMap M, int k, double *__restrict__ P64,
                                                          float *__restrict__ P32,
                                                          uint16_t *__restrict__ P16,
                                                          uint16_t *__restrict__ P16lo) {
  __shared__ float blk[64][65];
  const int nb = M.nb, s = nb / 64;
  const int i = k + 1 + blockIdx.y;
  const int br = blockIdx.x % s, bc = blockIdx.x / s;
  const int64_t t = tidx(i, k, M.T);
  const bool f32 = M.kind[t] == TK_F32;
  const char *src = M.base + M.off[t];
  const int64_t slot = (int64_t)blockIdx.y * nb * nb;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    const int64_t o = (int64_t)(bc * 64 + c) * nb + br * 64 + r;
    const double v = f32 ? (double)reinterpret_cast<const float *>(src)[o]
                         : reinterpret_cast<const double *>(src)[o];
    P64[slot + o] = v;
    const float fv = (float)v;
    P32[slot + o] = fv;
    blk[c][r] = fv;
  }
  if (!P16) return;
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int c = e & 63, r = e >> 6;  // row-major: consecutive threads along a row
    const float fv = blk[c][r];
    const uint16_t hi = bf16_rne(fv);
    const int64_t o = slot + (int64_t)(br * 64 + r) * nb + bc * 64 + c;
    P16[o] = hi;
    if (P16lo) P16lo[o] = bf16_rne(fv - __uint_as_float((uint32_t)hi << 16));
  }
}

// ------------------------------------------------------------ driver

// Off-band operand form of the trailing update.
enum { LOWP_F32 = 0, LOWP_BF16 = 1, LOWP_BF16X3 = 2 };

template <int NB>
static int launch_lowp_update(const TileMap &M, int k, int band, int64_t nwg, const float *P32,
                              const uint16_t *P16, const uint16_t *P16lo, int form, bool c64,
                              hipStream_t st) {
  const int64_t pad = (nwg + 7) / 8 * 8;
  if (form == LOWP_BF16X3)
    hipLaunchKernelGGL((k_lowp_bf16x3<NB, X3_STAGES>), dim3((unsigned)pad), dim3(256), 0, st, M, k,
                       band, nwg, pad, P16, P16lo);
  else if (form == LOWP_BF16)
    hipLaunchKernelGGL(k_lowp_bf16<NB>, dim3((unsigned)pad), dim3(256), 0, st, M, k, band, nwg, pad,
                       P16);
  else if (c64)
    hipLaunchKernelGGL((k_lowp_f32<NB, LP_UPDATE64>), dim3((unsigned)pad), dim3(256), 0, st, M, k,
                       band, nwg, pad, P32, (const float *)nullptr);
  else
    hipLaunchKernelGGL((k_lowp_f32<NB, LP_UPDATE>), dim3((unsigned)pad), dim3(256), 0, st, M, k,
                       band, nwg, pad, P32, (const float *)nullptr);
  return check_launch("lowp_update");
}

template <int NB>
static int launch_lowp_trsm(const TileMap &M, int k, int band, int64_t nwg, const float *P32,
                            const float *W32, hipStream_t st) {
  const int64_t pad = (nwg + 7) / 8 * 8;
  hipLaunchKernelGGL((k_lowp_f32<NB, LP_TRSM>), dim3((unsigned)pad), dim3(256), 0, st, M, k, band,
                     nwg, pad, P32, W32);
  return check_launch("lowp_trsm");
}

static int lowp_update(const TileMap &M, int k, int band, int64_t nwg, const float *P32,
                       const uint16_t *P16, const uint16_t *P16lo, int form, bool c64,
                       hipStream_t st) {
  switch (M.nb) {
    case 128: return launch_lowp_update<128>(M, k, band, nwg, P32, P16, P16lo, form, c64, st);
    case 256: return launch_lowp_update<256>(M, k, band, nwg, P32, P16, P16lo, form, c64, st);
    case 512: return launch_lowp_update<512>(M, k, band, nwg, P32, P16, P16lo, form, c64, st);
    case 768: return launch_lowp_update<768>(M, k, band, nwg, P32, P16, P16lo, form, c64, st);
    case 1024: return launch_lowp_update<1024>(M, k, band, nwg, P32, P16, P16lo, form, c64, st);
  }
  set_error("mixed precision: unsupported tile size %d", M.nb);
  return MVG_ERR_STATE;
}

static int lowp_trsm(const TileMap &M, int k, int band, int64_t nwg, const float *P32,
                     const float *W32, hipStream_t st) {
  switch (M.nb) {
    case 128: return launch_lowp_trsm<128>(M, k, band, nwg, P32, W32, st);
    case 256: return launch_lowp_trsm<256>(M, k, band, nwg, P32, W32, st);
    case 512: return launch_lowp_trsm<512>(M, k, band, nwg, P32, W32, st);
    case 768: return launch_lowp_trsm<768>(M, k, band, nwg, P32, W32, st);
    case 1024: return launch_lowp_trsm<1024>(M, k, band, nwg, P32, W32, st);
  }
  set_error("mixed precision: unsupported tile size %d", M.nb);
  return MVG_ERR_STATE;
}

// Useful flops of the trailing update of step k split by target precision.
static void mixed_flops(int64_t N, int nb, int T, int k, int band, double *f64, double *flow) {
  auto len = [&](int t) { return (double)std::min<int64_t>(nb, N - (int64_t)t * nb); };
  const double K = len(k);
  *f64 = 0.0;
  *flow = 0.0;
  for (int j = k + 1; j < T; ++j)
    for (int i = j; i < T; ++i) {
      const double f = (i == j) ? len(j) * (len(j) + 1.0) * K : 2.0 * len(i) * len(j) * K;
      if (i - j < band) {
        if (!(i == k + 1 && j == k + 1)) *f64 += f;
      } else {
        *flow += f;
      }
    }
}

int mixed_potrf(mvg_mat *A, int64_t *d_info, hipStream_t st) {
  const TileMap M = A->map();
  const int T = M.T, nb = M.nb, band = A->band;
  const bool bf16 = A->precision == MVG_MIXED_BF16;
  // BF16X3: as FP32X, with the off-band operands split into two BF16 terms
  const bool x3 = A->precision == MVG_MIXED_BF16X3;
  // FP32X: every tile FP64 and every panel solved in FP64; only the off-band
  // trailing GEMMs take FP32 operands (FP32 MFMA, FP64 target tiles)
  const bool x64 = A->precision == MVG_MIXED_FP32X || x3;
  const int form = x3 ? LOWP_BF16X3 : bf16 ? LOWP_BF16 : LOWP_F32;
  const int s = nb / LB;
  const int64_t ss = (int64_t)s * s;
  const int64_t per = (int64_t)nb * nb;
  const int nslot = std::max(1, T - 1);
  // workspaces: P64 | P32 | P16 (BF16: one plane; BF16X3: high, low) | W32
  const int p16b = bf16 ? 2 : x3 ? 4 : 0;
  const size_t bytes = (size_t)nslot * per * (8 + 4 + p16b) + (size_t)per * 4;
  char *ws = nullptr;
  if (malloc_async((void **)&ws, bytes, st) != hipSuccess) {
    hipGetLastError();
    set_error("mixed_potrf: workspace allocation of %.2f GB failed", bytes / 1e9);
    return MVG_ERR_ALLOC;
  }
  double *P64 = reinterpret_cast<double *>(ws);
  float *P32 = reinterpret_cast<float *>(ws + (size_t)nslot * per * 8);
  uint16_t *P16 = p16b ? reinterpret_cast<uint16_t *>(ws + (size_t)nslot * per * 12) : nullptr;
  uint16_t *P16lo = x3 ? P16 + (size_t)nslot * per : nullptr;
  float *W32 = reinterpret_cast<float *>(ws + (size_t)nslot * per * (12 + p16b));
  hipStream_t side = side_stream();
  hipEvent_t evD, evS, ev0;
  hipEventCreateWithFlags(&evD, hipEventDisableTiming);
  hipEventCreateWithFlags(&evS, hipEventDisableTiming);
  hipEventCreateWithFlags(&ev0, hipEventDisableTiming);
  const PivotTol pt = pivot_tol(A);
  int rc = 0;
  hipEventRecord(ev0, st);
  hipStreamWaitEvent(side, ev0, 0);
  rc = diag_factor(M, 0, A->d_winv, d_info, pt, side);
  hipEventRecord(evD, side);
  for (int k = 0; k < T && !rc; ++k) {
    hipStreamWaitEvent(st, evD, 0);
    const int nbelow = T - k - 1;
    if (nbelow > 0) {
      const int nband = x64 ? nbelow : std::min(band - 1, nbelow);  // FP64 panel tiles
      const int noff = nbelow - nband;                               // FP32 panel tiles
      hipLaunchKernelGGL(k_panel_stage_pre, dim3(64, nbelow), dim3(256), 0, st, M, k, P64, P32);
      rc = check_launch("panel_stage_pre");
      if (!rc && nband > 0)
        rc = launch_trail<TRAIL_TRSM>(M, k, 0, 0, (int64_t)nband * ss, P64,
                                      A->d_winv + (int64_t)k * per, st);
      if (!rc && noff > 0) {
        hipLaunchKernelGGL(k_to_f32, dim3(256), dim3(256), 0, st, A->d_winv + (int64_t)k * per,
                           W32, per);
        rc = check_launch("to_f32");
        if (!rc) rc = lowp_trsm(M, k, band, (int64_t)noff * ss, P32, W32, st);
      }
    }
    hipEventRecord(evS, st);
    if (rc || k + 1 >= T) continue;
    hipStreamWaitEvent(side, evS, 0);
    rc = launch_syrk_next(A, k, side);
    if (!rc) rc = diag_factor(M, k + 1, A->d_winv, d_info, pt, side);
    hipEventRecord(evD, side);
    if (rc) break;
    hipLaunchKernelGGL(k_panel_stage_post, dim3((nb / 64) * (nb / 64), nbelow), dim3(256), 0, st,
                       M, k, P64, P32, P16, P16lo);
    rc = check_launch("panel_stage_post");
    double f64 = 0.0, flow = 0.0;
    mixed_flops(A->N, nb, T, k, band, &f64, &flow);
    if (!rc) {
      int64_t nband_t = 0;
      for (int j = k + 1; j < T; ++j) nband_t += std::min(band, T - j);
      int h = prof_begin(MVG_PROF_TRAILING, st, f64, 0.0);
      rc = launch_trail<TRAIL_BAND>(M, k, band, ss, nband_t * ss, P64, nullptr, st);
      prof_end(h, st);
    }
    if (!rc) {
      int64_t noff_t = 0;
      for (int j = k + 1; j < T; ++j) noff_t += std::max(0, T - j - band);
      if (noff_t > 0) {
        int h = prof_begin(MVG_PROF_LOWP, st, flow, 0.0);
        rc = lowp_update(M, k, band, noff_t * ss, P32, P16, P16lo, form, x64, st);
        prof_end(h, st);
      }
    }
  }
  hipEventRecord(evD, side);
  hipStreamWaitEvent(st, evD, 0);
  hipFreeAsync(ws, st);
  hipEventDestroy(evD);
  hipEventDestroy(evS);
  hipEventDestroy(ev0);
  return rc;
}

// ------------------------------------------------ FP64 symmetric product
//
// y = Sigma x from the lower tiles of an FP64 (unfactored) matrix, every tile
// read once: tile (I, J) contributes T_IJ x_J to y_I and, off the diagonal,
// T_IJ^T x_I to y_J.  The two partial vectors of every tile are written out
// and added per row in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_symv_tile(TileMap M, const double *__restrict__ x,
                                                   double *__restrict__ prow,
                                                   double *__restrict__ pcol) {
  __shared__ double xi[1024], xj[1024];
  __shared__ double red[4][1024];
  const int nb = M.nb, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int J = 0;
  int64_t t = blockIdx.x;
  while (t >= M.T - J) {
    t -= M.T - J;
    ++J;
  }
  const int I = J + (int)t;
  const int64_t tile = blockIdx.x;
  for (int r = tid; r < nb; r += 256) {
    xi[r] = x[(int64_t)I * nb + r];
    xj[r] = x[(int64_t)J * nb + r];
  }
  __syncthreads();
  const double *Tl = reinterpret_cast<const double *>(M.base + M.off[tile]);
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  const int nq = nb / 64;
  for (int c = wave; c < nb; c += 4) {
    const double *col = Tl + (int64_t)c * nb;
    const double xc = xj[c];
    double dot = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (q < nq) {
        const double v = col[lane + 64 * q];
        acc[q] += v * xc;
        dot += v * xi[lane + 64 * q];
      }
    }
    if (I != J) {
      for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
      if (lane == 0) pcol[tile * nb + c] = dot;
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (q < nq) red[wave][lane + 64 * q] = acc[q];
  __syncthreads();
  for (int r = tid; r < nb; r += 256)
    prow[tile * nb + r] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
}

__global__ void k_symv_reduce(TileMap M, const double *__restrict__ prow,
                              const double *__restrict__ pcol, double *__restrict__ y) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = M.nb;
  if (g >= (int64_t)M.T * nb) return;
  const int I = (int)(g / nb), r = (int)(g % nb);
  double s = 0.0;
  for (int J = 0; J <= I; ++J) s += prow[tidx(I, J, M.T) * nb + r];
  for (int J = I + 1; J < M.T; ++J) s += pcol[tidx(J, I, M.T) * nb + r];
  y[g] = s;
}

int launch_symv(const mvg_mat *A, const double *d_x, double *d_y, double *d_part, hipStream_t st) {
  const TileMap M = A->map();
  if (M.nb > 1024) {
    set_error("symv: tile size above 1024");
    return MVG_ERR_STATE;
  }
  const int64_t nt = (int64_t)M.T * (M.T + 1) / 2;
  double *prow = d_part, *pcol = d_part + nt * M.nb;
  hipLaunchKernelGGL(k_symv_tile, dim3((unsigned)nt), dim3(256), 0, st, M, d_x, prow, pcol);
  if (int rc = check_launch("symv_tile")) return rc;
  hipLaunchKernelGGL(k_symv_reduce, dim3((unsigned)((A->Np + 255) / 256)), dim3(256), 0, st, M,
                     (const double *)prow, (const double *)pcol, d_y);
  return check_launch("symv_reduce");
}

// Fixed-order reductions over vectors of length n: one workgroup per chunk
// of AX_CHUNK entries, then one thread adds the chunk sums in order.
constexpr int AX_CHUNK = 4096;

__device__ __forceinline__ double block_sum(double a, double *red) {
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
    __syncthreads();
  }
  return red[0];
}

// r = z - sx, part[chunk] = sum r^2
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ z,
                                                  const double *__restrict__ sx,
                                                  double *__restrict__ r, int64_t n,
                                                  double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t base = (int64_t)blockIdx.x * AX_CHUNK;
  double a = 0.0;
  for (int t = threadIdx.x; t < AX_CHUNK; t += 256) {
    const int64_t g = base + t;
    if (g >= n) break;
    const double v = z[g] - sx[g];
    r[g] = v;
    a += v * v;
  }
  const double tot = block_sum(a, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// part[chunk] = sum a b
__global__ __launch_bounds__(256) void k_dot_part(const double *__restrict__ a,
                                                  const double *__restrict__ b, int64_t n,
                                                  double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t base = (int64_t)blockIdx.x * AX_CHUNK;
  double acc = 0.0;
  for (int t = threadIdx.x; t < AX_CHUNK; t += 256) {
    const int64_t g = base + t;
    if (g >= n) break;
    acc += a[g] * b[g];
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void k_sum_parts(const double *__restrict__ part, int n, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += part[i];
    out[0] = s2;
  }
}

__global__ void k_axpy(double *__restrict__ x, const double *__restrict__ d, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) x[g] += d[g];
}

int reduce_chunks(int64_t n) { return (int)((n + AX_CHUNK - 1) / AX_CHUNK); }

int launch_axpy_norm(const double *d_z, const double *d_sx, double *d_r, int64_t n, double *d_part,
                     double *d_out, hipStream_t st) {
  const int nblk = reduce_chunks(n);
  hipLaunchKernelGGL(k_residual, dim3(nblk), dim3(256), 0, st, d_z, d_sx, d_r, n, d_part);
  if (int rc = check_launch("residual")) return rc;
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, (const double *)d_part, nblk, d_out);
  return check_launch("sum_parts");
}

int launch_dot(const double *d_a, const double *d_b, int64_t n, double *d_part, double *d_out,
               hipStream_t st) {
  const int nblk = reduce_chunks(n);
  hipLaunchKernelGGL(k_dot_part, dim3(nblk), dim3(256), 0, st, d_a, d_b, n, d_part);
  if (int rc = check_launch("dot_part")) return rc;
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, (const double *)d_part, nblk, d_out);
  return check_launch("sum_parts");
}

int launch_axpy(double *d_x, const double *d_d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d_x, d_d, n);
  return check_launch("axpy");
}

// Copy an FP64 matrix into a mixed-layout matrix of the same shape: FP64
// tiles verbatim, FP32 tiles rounded to nearest.
__global__ __launch_bounds__(256) void k_mat_convert(TileMap S, TileMap D) {
  const int64_t t = blockIdx.y;
  const int64_t per = (int64_t)S.nb * S.nb;
  const double *src = reinterpret_cast<const double *>(S.base + S.off[t]);
  char *dst = D.base + D.off[t];
  const bool f32 = D.kind[t] == TK_F32;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; e < per;
       e += (int64_t)gridDim.x * blockDim.x * 2) {
    const double2 v = *reinterpret_cast<const double2 *>(src + e);
    if (f32)
      *reinterpret_cast<float2 *>(reinterpret_cast<float *>(dst) + e) =
          make_float2((float)v.x, (float)v.y);
    else
      *reinterpret_cast<double2 *>(reinterpret_cast<double *>(dst) + e) = v;
  }
}

int launch_mat_convert(const mvg_mat *S, mvg_mat *D, hipStream_t st) {
  if (S->T != D->T || S->nb != D->nb) {
    set_error("mat_convert: shapes differ");
    return MVG_ERR_STATE;
  }
  const int64_t nt = (int64_t)S->T * (S->T + 1) / 2;
  const TileMap Ms = S->map(), Md = D->map();
  for (int64_t t0 = 0; t0 < nt; t0 += 65535) {
    const int64_t cnt = std::min<int64_t>(65535, nt - t0);
    TileMap a = Ms, b = Md;
    a.off += t0;
    b.off += t0;
    b.kind += t0;
    hipLaunchKernelGGL(k_mat_convert, dim3(16, (unsigned)cnt), dim3(256), 0, st, a, b);
    if (int rc = check_launch("mat_convert")) return rc;
  }
  return 0;
}

}  // namespace mvg
