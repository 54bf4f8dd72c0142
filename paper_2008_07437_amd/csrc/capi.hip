// C ABI entry points (declared in include/mvgeo.h): argument checking, the
// library-owned matrices and factors, and the orchestration of the kernels.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <string>
#include <tuple>
#include <vector>

#include "mvgeo_internal.h"
#include "tlr.h"

namespace mvg {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch %s failed: %s", what, hipGetErrorString(e));
    return MVG_ERR_LAUNCH;
  }
  return 0;
}

// The look-ahead stream of the calling thread (default priority), destroyed
// when the thread exits.
namespace {
struct ThreadStream {
  hipStream_t s = nullptr;
  int dev = -1;
  ~ThreadStream() {
    if (s) hipStreamDestroy(s);
  }
};
thread_local ThreadStream g_side;
}  // namespace

hipStream_t side_stream() {
  int cur = 0;
  hipGetDevice(&cur);
  if (!g_side.s || g_side.dev != cur) {
    if (g_side.s) hipStreamDestroy(g_side.s);
    hipStreamCreateWithFlags(&g_side.s, hipStreamNonBlocking);  // default priority
    g_side.dev = cur;
  }
  return g_side.s;
}

// Device memory of the library that outlives a call (tile arenas, per-matrix
// buffers, factors) is allocated stream-ordered on a per-device release
// stream, which is then synchronised (it is idle: the allocation is usable on
// any stream at once), and freed stream-ordered on that stream once idle.
// hipFree would wait for the whole device, i.e. for every other stream's
// work, which serialises concurrent requests.
constexpr uint64_t POOL_KEEP = (uint64_t)48 << 30;

static hipStream_t release_stream() {
  static std::mutex mu;
  static hipStream_t s[64] = {};
  int dev = 0;
  hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (!s[dev]) {
    hipStreamCreateWithFlags(&s[dev], hipStreamNonBlocking);  // default priority
    // keep up to POOL_KEEP bytes of freed stream-ordered memory mapped in the
    // device's default pool: the per-evaluation workspaces and TLR stores
    // (GBs) are then reused instead of mapped anew (~0.1 s per GB-sized
    // allocation otherwise); dev_alloc trims the pool before giving up
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) {
      uint64_t keep = POOL_KEEP;
      hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    hipGetLastError();
  }
  return s[dev];
}

void *dev_alloc(size_t bytes) {
  void *p = nullptr;
  hipStream_t r = release_stream();
  if (hipMallocAsync(&p, bytes ? bytes : 8, r) != hipSuccess) {
    hipGetLastError();
    // memory kept by the pool after frees: return it and try once more
    int dev = 0;
    hipGetDevice(&dev);
    hipMemPool_t pool = nullptr;
    hipStreamSynchronize(r);
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) hipMemPoolTrimTo(pool, 0);
    if (hipMallocAsync(&p, bytes ? bytes : 8, r) != hipSuccess) {
      hipGetLastError();
      return nullptr;
    }
  }
  if (hipStreamSynchronize(r) != hipSuccess) {
    hipGetLastError();
    return nullptr;
  }
  return p;
}

// p idle (no work that uses it is pending)
void dev_free(void *p) {
  if (p) hipFreeAsync(p, release_stream());
}

// Records that the library's work on A so far is on stream st (for the
// entry points that return before it completes), so that destroying A waits
// for that work only.
static int mark_done(const mvg_mat *A, hipStream_t st) {
  if (!A->done && hipEventCreateWithFlags(&A->done, hipEventDisableTiming) != hipSuccess) {
    A->done = nullptr;
    hipGetLastError();
    set_error("event creation failed");
    return MVG_ERR_LAUNCH;
  }
  if (hipEventRecord(A->done, st) != hipSuccess) {
    hipGetLastError();
    set_error("event record failed");
    return MVG_ERR_LAUNCH;
  }
  return 0;
}

// ------------------------------------------------------------ profiling

struct ProfRec {
  int kind;
  hipEvent_t a, b;
  double flops, bytes;
};
static std::mutex g_prof_mu;
static std::vector<ProfRec> g_prof;
static bool g_prof_on = false;

// Events are created once and reused across recording sessions (creating two
// per record would cost more host time than the launches being timed).
static std::vector<hipEvent_t> g_prof_events;

int prof_begin(int kind, hipStream_t st, double flops, double bytes) {
  if (!g_prof_on) return -1;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  const size_t need = 2 * (g_prof.size() + 1);
  while (g_prof_events.size() < need) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      hipGetLastError();
      return -1;
    }
    g_prof_events.push_back(e);
  }
  ProfRec r{kind, g_prof_events[need - 2], g_prof_events[need - 1], flops, bytes};
  hipEventRecord(r.a, st);
  g_prof.push_back(r);
  return (int)g_prof.size() - 1;
}

void prof_end(int h, hipStream_t st) {
  if (h < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (h < (int)g_prof.size()) hipEventRecord(g_prof[h].b, st);
}

static void prof_clear() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.clear();  // the events stay for the next session
}

// ------------------------------------------------------------ arena pool
//
// Tile arenas are large (GBs) and reused across evaluations of the same size;
// a small pool avoids a hipMalloc / hipFree pair per likelihood call.
struct PoolEntry {
  void *p;
  size_t bytes;
  int dev;
};
static std::mutex g_pool_mu;
static std::vector<PoolEntry> g_pool;
constexpr size_t POOL_MAX = 4;

static void release_cached(hipStream_t st);

static void *arena_acquire(size_t bytes) {
  int dev = 0;
  hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (size_t i = 0; i < g_pool.size(); ++i)
      if (g_pool[i].dev == dev && g_pool[i].bytes >= bytes && g_pool[i].bytes <= bytes + bytes / 4) {
        void *p = g_pool[i].p;
        g_pool.erase(g_pool.begin() + i);
        return p;
      }
  }
  void *p = dev_alloc(bytes);
  if (!p) {  // free the pooled arenas and retry once
    release_cached(nullptr);
    p = dev_alloc(bytes);
  }
  return p;
}

// every pooled arena back to the device pool, then the device pool's cached
// memory back to the device
static void release_cached(hipStream_t st) {
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto &e : g_pool) dev_free(e.p);
    g_pool.clear();
  }
  hipStreamSynchronize(release_stream());
  if (st) hipStreamSynchronize(st);
  int dev = 0;
  hipGetDevice(&dev);
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) hipMemPoolTrimTo(pool, 0);
  hipGetLastError();
}

hipError_t malloc_async(void **p, size_t bytes, hipStream_t st) {
  if (hipMallocAsync(p, bytes ? bytes : 8, st) == hipSuccess) return hipSuccess;
  hipGetLastError();
  release_cached(st);
  const hipError_t e = hipMallocAsync(p, bytes ? bytes : 8, st);
  if (e != hipSuccess) hipGetLastError();
  return e;
}

static void arena_release(void *p, size_t bytes) {
  if (!p) return;
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool.size() >= POOL_MAX) {
    dev_free(g_pool.front().p);
    g_pool.erase(g_pool.begin());
  }
  g_pool.push_back({p, bytes, dev});
}

// ------------------------------------------------------------- small kernels

__global__ void k_reduce_chunks(const double *__restrict__ part, int64_t m, int nchunk,
                                double *__restrict__ zhat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // i = 2t + j
  if (i >= 2 * m) return;
  const int64_t t = i / 2;
  const int j = (int)(i % 2);
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(t * nchunk + c) * 2 + j];
  zhat[i] = s;
}

__global__ void k_mse_final(const double *__restrict__ ss, int64_t m, double trc0,
                            double *__restrict__ mse) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  mse[t] = trc0 - (ss[2 * t] + ss[2 * t + 1]);
}

__global__ void k_add_pair(const double *__restrict__ s, double *__restrict__ out) {
  if (threadIdx.x == 0) out[0] = s[0] + s[1];
}

__global__ void k_stride_copy(const double *__restrict__ z, int p, int i, int64_t n,
                              double *__restrict__ out) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n) out[l] = z[(int64_t)p * l + i];
}

__global__ void k_loe_mom(const double *__restrict__ sT, const double *__restrict__ sA,
                          const double *__restrict__ dT, const double *__restrict__ sQ, int64_t m,
                          double trt, double tra, double *__restrict__ loe,
                          double *__restrict__ mom) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= m) return;
  const double et = trt - (sT[2 * l] + sT[2 * l + 1]);
  const double ea = tra - (sA[2 * l] + sA[2 * l + 1]);
  const double eta = trt - 2.0 * (dT[2 * l] + dT[2 * l + 1]) + (sQ[2 * l] + sQ[2 * l + 1]);
  loe[l] = eta / et - 1.0;
  mom[l] = ea / eta - 1.0;
}

__global__ void k_copy_pad(const double *__restrict__ src, int64_t n, double *__restrict__ dst,
                           int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) dst[i] = i < n ? src[i] : 0.0;
}

SmallTask small_task(const double *x, const double *y, const double *z, int64_t n,
                     const mvg_theta &th) {
  SmallTask t{};
  t.x = x;
  t.y = y;
  t.z = z;
  t.n = n;
  matern_setup(&th, &t.P);
  t.t0 = 0x1p-40 * th.sigma11_sq;
  t.t1 = 0x1p-40 * th.sigma22_sq;
  return t;
}

}  // namespace mvg

using namespace mvg;

// ------------------------------------------------------------ matrices

static bool is_mixed(int precision) {
  return precision == MVG_MIXED_FP32 || precision == MVG_MIXED_BF16 ||
         precision == MVG_MIXED_FP32X || precision == MVG_MIXED_BF16X3;
}

static int normalize_opts(const mvg_opts *o, mvg_opts *out) {
  mvg_opts d{};
  if (o) d = *o;
  if (d.precision < MVG_FP64 || d.precision > MVG_MIXED_BF16X3) return -1;
  if (d.nb == 0) d.nb = (d.precision == MVG_TLR) ? 1200 : 512;
  if (d.precision == MVG_TLR) {
    if (d.nb < 64 || d.nb % 2 || d.nb > QR_MAXM) return -2;
  } else {
    if (d.nb != 128 && d.nb != 256 && d.nb != 512 && d.nb != 768 && d.nb != 1024) return -2;
  }
  if (d.band_tiles <= 0) d.band_tiles = 2;
  if (is_mixed(d.precision) && d.band_tiles < 2) return -3;
  if (d.tlr_acc <= 0.0) d.tlr_acc = 1e-7;
  if (d.tlr_max_rank <= 0) d.tlr_max_rank = 300;
  if (d.tlr_max_rank > QR_MAXN - 16) return -4;
  if (d.ir_max_iter <= 0) d.ir_max_iter = 20;
  if (d.ir_tol <= 0.0) d.ir_tol = 1e-14;
  *out = d;
  return 0;
}

PivotTol mvg::pivot_tol(const mvg_mat *A) {
  PivotTol t{};
  t.p = A->p;
  if (A->p == 2) {
    t.tol[0] = 0x1p-40 * A->theta.sigma11_sq;
    t.tol[1] = 0x1p-40 * A->theta.sigma22_sq;
  } else {
    for (int i = 0; i < A->p; ++i) t.tol[i] = 0x1p-40 * A->theta_p.sigma_sq[i];
  }
  t.N = A->N;
  return t;
}

static void mat_free(mvg_mat *A) {
  if (!A) return;
  tlr_state_free(A->tlr);
  arena_release(A->arena, A->arena_bytes);
  dev_free(A->d_off);
  dev_free(A->d_kind);
  dev_free(A->d_x);
  dev_free(A->d_y);
  dev_free(A->d_qtab);
  dev_free(A->d_winv);
  if (A->done) hipEventDestroy(A->done);
  delete[] A->h_off;
  delete[] A->h_kind;
  delete A;
}

// Tile layout: band tiles (|I - J| < band) FP64; the rest FP32 (mixed), FP64,
// or (DST) all mapped to one shared zero tile stored after the others.
// zero_off receives that tile's offset (-1: none).
static int tile_layout(int T, int nb, int precision, int band, int64_t *off, int *kind,
                       size_t *total, int64_t *zero_off) {
  size_t pos = 0;
  bool any_zero = false;
  for (int J = 0; J < T; ++J)
    for (int I = J; I < T; ++I) {
      const int64_t t = tidx(I, J, T);
      const bool far = (I - J) >= band;
      const bool lowp = (precision == MVG_MIXED_FP32 || precision == MVG_MIXED_BF16) && far;
      if (precision == MVG_DST && far) {
        kind[t] = TK_ZERO;
        any_zero = true;
        continue;
      }
      kind[t] = lowp ? TK_F32 : TK_F64;
      off[t] = (int64_t)pos;
      pos += (size_t)nb * nb * (lowp ? 4 : 8);
      pos = (pos + 255) / 256 * 256;
    }
  *zero_off = -1;
  if (any_zero) {
    *zero_off = (int64_t)pos;
    for (int64_t t = 0; t < (int64_t)T * (T + 1) / 2; ++t)
      if (kind[t] == TK_ZERO) off[t] = (int64_t)pos;
    pos += ((size_t)nb * nb * 8 + 255) / 256 * 256;
  }
  *total = pos;
  return 0;
}

static size_t layout_bytes(int64_t n_loc, const mvg_opts &o) {
  const int64_t N = 2 * n_loc;
  const int T = (int)((N + o.nb - 1) / o.nb);
  size_t total = 0;
  bool any_zero = false;
  for (int J = 0; J < T; ++J)
    for (int I = J; I < T; ++I) {
      const bool far = (I - J) >= o.band_tiles;
      const bool lowp = (o.precision == MVG_MIXED_FP32 || o.precision == MVG_MIXED_BF16) && far;
      if (o.precision == MVG_DST && far) {
        any_zero = true;
        continue;
      }
      total += ((size_t)o.nb * o.nb * (lowp ? 4 : 8) + 255) / 256 * 256;
    }
  if (any_zero) total += ((size_t)o.nb * o.nb * 8 + 255) / 256 * 256;
  return total;
}

// Tile storage for p variables (N = p n_loc); the caller sets theta.
static int mat_alloc(int64_t n_loc, int p, const mvg_opts &o, const double *d_x, const double *d_y,
                     hipStream_t st, mvg_mat **out);

static int mat_create(int64_t n_loc, const mvg_opts &o, const mvg_theta *th, const double *d_x,
                      const double *d_y, hipStream_t st, mvg_mat **out) {
  MaternArgs margs;
  if (int rc = matern_setup(th, &margs)) return rc;
  mvg_mat *A = nullptr;
  if (int rc = mat_alloc(n_loc, 2, o, d_x, d_y, st, &A)) return rc;
  A->theta = *th;
  A->margs = margs;
  *out = A;
  return 0;
}

// p-variate matrix; p = 2 keeps the bivariate kernels (theta converted).
static mvg_theta theta_from_p(const mvg_theta_p &t) {
  return mvg_theta{t.sigma_sq[0], t.sigma_sq[1], t.a, t.nu[0], t.nu[1], t.beta[1]};
}

static int mat_create_p(int64_t n_loc, const mvg_opts &o, const mvg_theta_p *th,
                        const double *d_x, const double *d_y, hipStream_t st, mvg_mat **out) {
  MaternArgsP mp;
  if (int rc = matern_setup_p(th, &mp)) return rc;
  if (th->p == 2) {
    const mvg_theta t2 = theta_from_p(*th);
    return mat_create(n_loc, o, &t2, d_x, d_y, st, out);
  }
  mvg_mat *A = nullptr;
  if (int rc = mat_alloc(n_loc, th->p, o, d_x, d_y, st, &A)) return rc;
  A->theta_p = *th;
  A->margs_p = mp;
  *out = A;
  return 0;
}

static int mat_alloc(int64_t n_loc, int p, const mvg_opts &o, const double *d_x, const double *d_y,
                     hipStream_t st, mvg_mat **out) {
  mvg_mat *A = new mvg_mat();
  A->n_loc = n_loc;
  A->p = p;
  A->N = (int64_t)p * n_loc;
  A->nb = o.nb;
  A->T = (int)((A->N + o.nb - 1) / o.nb);
  A->Np = (int64_t)A->T * o.nb;
  A->precision = o.precision;
  A->band = o.band_tiles;
  A->opts = o;
  const int64_t nt = (int64_t)A->T * (A->T + 1) / 2;
  A->h_off = new int64_t[nt];
  A->h_kind = new int[nt];
  int64_t zero_off = -1;
  tile_layout(A->T, A->nb, A->precision == MVG_TLR ? MVG_FP64 : A->precision, A->band, A->h_off,
              A->h_kind, &A->arena_bytes, &zero_off);
  A->arena = (char *)arena_acquire(A->arena_bytes);
  bool ok = A->arena != nullptr;
  ok = ok && (A->d_off = (int64_t *)dev_alloc(sizeof(int64_t) * nt)) != nullptr;
  ok = ok && (A->d_kind = (int *)dev_alloc(sizeof(int) * nt)) != nullptr;
  ok = ok && (A->d_x = (double *)dev_alloc(sizeof(double) * n_loc)) != nullptr;
  ok = ok && (A->d_y = (double *)dev_alloc(sizeof(double) * n_loc)) != nullptr;
  ok = ok && (A->d_qtab = (double *)dev_alloc(sizeof(double) * (1 + PORD) * QN)) != nullptr;
  ok = ok && (A->d_winv = (double *)dev_alloc(sizeof(double) * (size_t)A->Np * A->nb)) != nullptr;
  if (!ok) {
    hipGetLastError();
    set_error("device allocation of %.3f GB for a %lld-location matrix failed",
              A->arena_bytes / 1e9, (long long)n_loc);
    mat_free(A);
    return MVG_ERR_ALLOC;
  }
  hipMemcpyAsync(A->d_off, A->h_off, sizeof(int64_t) * nt, hipMemcpyHostToDevice, st);
  hipMemcpyAsync(A->d_kind, A->h_kind, sizeof(int) * nt, hipMemcpyHostToDevice, st);
  hipMemcpyAsync(A->d_x, d_x, sizeof(double) * n_loc, hipMemcpyDeviceToDevice, st);
  hipMemcpyAsync(A->d_y, d_y, sizeof(double) * n_loc, hipMemcpyDeviceToDevice, st);
  // the host offset tables are read by the copies above; keep them alive with A
  if (zero_off >= 0) {  // the shared tile of the annihilated DST tiles
    if (int rc = launch_fill_f64(reinterpret_cast<double *>(A->arena + zero_off), 0.0,
                                 (int64_t)A->nb * A->nb, st)) {
      mat_free(A);
      return rc;
    }
  }
  *out = A;
  return 0;
}

// A TLR matrix: locations, theta constants, quadrature table; the tiles are
// built by tlr_build.
static int tlr_mat_create(int64_t n_loc, const mvg_opts &o, const mvg_theta *th, const double *d_x,
                          const double *d_y, hipStream_t st, mvg_mat **out) {
  mvg_mat *A = new mvg_mat();
  A->n_loc = n_loc;
  A->N = 2 * n_loc;
  A->nb = o.nb;
  A->T = (int)((A->N + o.nb - 1) / o.nb);
  A->Np = (int64_t)A->T * o.nb;
  A->precision = MVG_TLR;
  A->theta = *th;
  A->opts = o;
  if (int rc = matern_setup(th, &A->margs)) {
    delete A;
    return rc;
  }
  A->tlr = new TlrState();
  bool ok = (A->d_x = (double *)dev_alloc(sizeof(double) * n_loc)) != nullptr;
  ok = ok && (A->d_y = (double *)dev_alloc(sizeof(double) * n_loc)) != nullptr;
  ok = ok && (A->d_qtab = (double *)dev_alloc(sizeof(double) * 4 * QN)) != nullptr;
  if (!ok) {
    hipGetLastError();
    set_error("device allocation for a %lld-location TLR matrix failed", (long long)n_loc);
    mat_free(A);
    return MVG_ERR_ALLOC;
  }
  hipMemcpyAsync(A->d_x, d_x, sizeof(double) * n_loc, hipMemcpyDeviceToDevice, st);
  hipMemcpyAsync(A->d_y, d_y, sizeof(double) * n_loc, hipMemcpyDeviceToDevice, st);
  *out = A;
  return 0;
}

// Regenerate and compress Sigma(theta) into a TLR matrix.
static int tlr_generate(mvg_mat *A, hipStream_t st) {
  if (int rc = launch_quad_table(A->margs, A->d_qtab, st)) return rc;
  A->factored = 0;
  store_free(A->tlr->S);
  store_free(A->tlr->L);
  return tlr_build(A, A->opts, st);
}

// Regenerate Sigma(theta) into an existing matrix of the same shape.
static int mat_generate(mvg_mat *A, hipStream_t st) {
  A->factored = 0;
  if (A->p != 2) {
    if (int rc = launch_quad_table_p(A->margs_p, A->d_qtab, st)) return rc;
    return launch_cov_tiles_p(A->margs_p, A->d_qtab, A->d_x, A->d_y, A->n_loc, A->map(), st);
  }
  if (int rc = launch_quad_table(A->margs, A->d_qtab, st)) return rc;
  const int64_t nt = (int64_t)A->T * (A->T + 1) / 2;
  return launch_cov_tiles(A->margs, A->d_qtab, A->d_x, A->d_y, A->n_loc, A->map(), 0, (int)nt, st);
}

extern "C" {

const char *mvg_last_error(void) { return g_err; }

int mvg_prof_enable(int on) {
  hipDeviceSynchronize();
  if (on) prof_clear();
  g_prof_on = on != 0;
  return 0;
}

int mvg_prof_read(int kind, int64_t *launches, double *total_ms, double *flops, double *bytes) {
  if (kind < 0 || kind >= MVG_PROF_NKINDS) return -1;
  hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int64_t n = 0;
  double ms = 0.0, f = 0.0, b = 0.0;
  for (auto &r : g_prof) {
    if (r.kind != kind) continue;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      hipGetLastError();
      continue;
    }
    ++n;
    ms += t;
    f += r.flops;
    b += r.bytes;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (flops) *flops = f;
  if (bytes) *bytes = b;
  return 0;
}

size_t mvg_footprint(int64_t n_loc, const mvg_opts *o) {
  mvg_opts d;
  if (n_loc < 1 || normalize_opts(o, &d)) return 0;
  const int64_t N = 2 * n_loc;
  const int T = (int)((N + d.nb - 1) / d.nb);
  const int64_t Np = (int64_t)T * d.nb;
  if (d.precision == MVG_TLR) {
    // estimate: dense diagonal tiles of Sigma and L plus W (3 T nbp^2), the
    // dense tile-column buffer (T nb^2), low-rank pairs at an assumed mean
    // rank of 64 for Sigma and L, the update workspace of the widest column
    const size_t nbp = (d.nb + 63) / 64 * 64;
    const size_t nt = (size_t)T * (T - 1) / 2;
    size_t b = sizeof(double) * (3 * (size_t)T * nbp * nbp + (size_t)T * d.nb * d.nb);
    b += sizeof(double) * 2 * nt * 2 * (size_t)d.nb * 64;
    b += sizeof(double) * (size_t)(T + 1) * d.nb * ((size_t)T / 2 * 64 + d.nb);
    b += sizeof(double) * (size_t)(2 * n_loc + 3 * Np + 4 * QN);
    return b;
  }
  size_t b = layout_bytes(n_loc, d);
  // matrix + inverse diagonal tiles + panel workspace + vectors
  b += sizeof(double) * (size_t)(2 * n_loc + 3 * Np + 4 * QN + 2 * Np * d.nb);
  b += (sizeof(int64_t) + sizeof(int)) * (size_t)T * (T + 1) / 2;
  if (is_mixed(d.precision)) {
    mvg_opts f = d;
    f.precision = MVG_FP64;
    b += layout_bytes(n_loc, f);  // FP64 Sigma kept for the refinement
    b += sizeof(double) * (size_t)T * (T + 1) * d.nb;  // symmetric-product partials
    b += sizeof(double) * (size_t)4 * Np;              // refinement vectors
    const int p16b = d.precision == MVG_MIXED_BF16 ? 2 : d.precision == MVG_MIXED_BF16X3 ? 4 : 0;
    b += (size_t)(T > 1 ? T - 1 : 1) * d.nb * d.nb * (4 + p16b);
  }
  return b;
}

int mvg_dst_band(int64_t n_loc, int nb, double keep_fraction) {
  if (n_loc < 1 || nb < 1 || !(keep_fraction > 0.0) || keep_fraction > 1.0) return -1;
  const int64_t T = (2 * n_loc + nb - 1) / nb;
  const double need = keep_fraction * (double)T * (double)T;
  for (int64_t w = 1; w < T; ++w)
    if ((double)(T + (w - 1) * (2 * T - w)) >= need) return (int)w;
  return (int)T;
}

int cov_generate(const double *d_x, const double *d_y, int64_t n_loc, const mvg_theta *th,
                 const mvg_opts *o, mvg_mat **out, void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (n_loc < 1) return -3;
  if (!th) return -4;
  mvg_opts d;
  if (normalize_opts(o, &d)) return -5;
  if (!out) return -6;
  MaternArgs tmp;
  if (matern_setup(th, &tmp)) return -4;
  hipStream_t st = (hipStream_t)hip_stream;
  mvg_mat *A = nullptr;
  if (int rc = mat_create(n_loc, d, th, d_x, d_y, st, &A)) return rc < 0 && rc > -100 ? -4 : rc;
  if (int rc = mat_generate(A, st)) {
    mat_free(A);
    return rc;
  }
  if (int rc = mark_done(A, st)) {
    hipStreamSynchronize(st);
    mat_free(A);
    return rc;
  }
  *out = A;
  return 0;
}

int potrf_tiled(mvg_mat *A, const mvg_opts *o, int64_t *h_info, void *hip_stream) {
  (void)o;
  if (!A) return -1;
  if (!h_info) return -3;
  if (A->factored) {
    set_error("potrf_tiled: matrix already factored");
    return -1;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  int64_t *d_info = nullptr;
  if (malloc_async((void **)&d_info, sizeof(int64_t), st) != hipSuccess) {
    set_error("hipMallocAsync failed");
    return MVG_ERR_ALLOC;
  }
  int rc = launch_fill_i64(d_info, INT64_MAX, 1, st);
  const bool mixed = is_mixed(A->precision);
  if (!rc)
    rc = A->precision == MVG_TLR ? tlr_potrf(A, A->opts, d_info, st)
                                 : mixed ? mixed_potrf(A, d_info, st) : dense_potrf(A, d_info, st);
  int64_t info = 0;
  hipMemcpyAsync(&info, d_info, sizeof(int64_t), hipMemcpyDeviceToHost, st);
  hipFreeAsync(d_info, st);
  hipStreamSynchronize(st);
  if (rc) return rc;
  *h_info = info == INT64_MAX ? 0 : info;
  A->factored = 1;
  return 0;
}

// One likelihood evaluation on a generated matrix; optionally leaves L^-1 Z in d_yv.
static int eval_one(mvg_mat *A, const double *d_z, double *d_yv, double *d_part, double *d_out2,
                    int64_t *d_info, hipStream_t st) {
  int rc = launch_fill_i64(d_info, INT64_MAX, 1, st);
  const double Nd = (double)A->N;
  int hp = prof_begin(MVG_PROF_POTRF, st, Nd * Nd * Nd / 3.0 + Nd * Nd / 2.0, 0.0);
  if (!rc) rc = A->tlr ? tlr_potrf(A, A->opts, d_info, st) : dense_potrf(A, d_info, st);
  prof_end(hp, st);
  int hs = prof_begin(MVG_PROF_SOLVE, st, Nd * Nd, 8.0 * Nd * (Nd + 1) / 2);
  if (!rc) {
    hipLaunchKernelGGL(k_copy_pad, dim3((unsigned)((A->Np + 255) / 256)), dim3(256), 0, st, d_z,
                       A->N, d_yv, A->Np);
    rc = check_launch("copy_pad");
  }
  if (!rc) rc = trsv_forward(A, d_yv, st);
  if (!rc) rc = logdet_quad(A, d_yv, d_part, d_out2, st);
  prof_end(hs, st);
  A->factored = 1;
  return rc;
}

// The refinement also stops once |x^T r| <= IR_QUAD_TOL |Z^T x|: the
// quadratic form is then known to ~IR_QUAD_TOL^2 relative.
constexpr double IR_QUAD_TOL = 1e-10;


struct IrStat {
  int iters, converged;
  double relres;
};
static thread_local std::vector<IrStat> g_ir;

int mvg_ir_stats(int i, int *iters, double *relres, int *converged) {
  if (i < 0 || i >= (int)g_ir.size()) return -1;
  if (iters) *iters = g_ir[i].iters;
  if (relres) *relres = g_ir[i].relres;
  if (converged) *converged = g_ir[i].converged;
  return 0;
}

// Workspace of one mixed-precision evaluation (device, one allocation).
struct MixedWs {
  double *zp, *x, *sx, *r, *yv, *part, *sym, *scal;  // scal: 8 doubles
};

// Mixed-precision evaluation: Sigma in FP64 (S) converted into the mixed
// matrix A, mixed factorisation, log|Sigma| from the mixed factor, then x =
// Sigma^-1 Z refined in FP64 against S, q = Z^T x.  out2 = {logdet, q}
// (device), info (device), stat (host).
static int eval_mixed(mvg_mat *S, mvg_mat *A, const double *d_z, const mvg_opts &o,
                      const MixedWs &w, double *d_out2, int64_t *d_info, IrStat *stat,
                      bool need_x, hipStream_t st) {
  const double Nd = (double)A->N;
  const int64_t Np = A->Np;
  int rc = launch_fill_i64(d_info, INT64_MAX, 1, st);
  if (!rc) rc = launch_mat_convert(S, A, st);
  int hp = prof_begin(MVG_PROF_POTRF, st, Nd * Nd * Nd / 3.0 + Nd * Nd / 2.0, 0.0);
  if (!rc) rc = mixed_potrf(A, d_info, st);
  prof_end(hp, st);
  A->factored = 1;
  if (rc) return rc;
  int64_t info = 0;
  hipMemcpyAsync(&info, d_info, sizeof(int64_t), hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return MVG_ERR_LAUNCH;
  stat->iters = 0;
  stat->converged = 0;
  stat->relres = NAN;
  if (info != INT64_MAX) return 0;  // not positive definite in mixed arithmetic
  int hs = prof_begin(MVG_PROF_SOLVE, st, Nd * Nd, 8.0 * Nd * (Nd + 1) / 2);
  hipLaunchKernelGGL(k_copy_pad, dim3((unsigned)((Np + 255) / 256)), dim3(256), 0, st, d_z, A->N,
                     w.zp, Np);
  rc = check_launch("copy_pad");
  if (!rc) rc = hipMemcpyAsync(w.yv, w.zp, sizeof(double) * Np, hipMemcpyDeviceToDevice, st)
                    ? MVG_ERR_LAUNCH : 0;
  if (!rc) rc = trsv_forward(A, w.yv, st);
  if (!rc) rc = logdet_quad(A, w.yv, w.part, d_out2, st);  // {logdet, y^T y}
  if (!rc) rc = hipMemcpyAsync(w.x, w.yv, sizeof(double) * Np, hipMemcpyDeviceToDevice, st)
                    ? MVG_ERR_LAUNCH : 0;
  if (!rc) rc = trsv_backward(A, w.x, st);
  if (!rc) rc = launch_dot(w.zp, w.zp, Np, w.part, w.scal, st);  // ||Z||^2
  prof_end(hs, st);
  double zn2 = 0.0;
  if (!rc) {
    hipMemcpyAsync(&zn2, w.scal, sizeof(double), hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess) rc = MVG_ERR_LAUNCH;
  }
  const double zn = std::sqrt(zn2);
  double prev = INFINITY;
  for (int it = 0; !rc; ++it) {
    int hi = prof_begin(MVG_PROF_IR, st, 2.0 * Nd * Nd, 8.0 * Nd * (Nd + 1) / 2);
    rc = launch_symv(S, w.x, w.sx, w.sym, st);
    if (!rc) rc = launch_axpy_norm(w.zp, w.sx, w.r, Np, w.part, w.scal + 1, st);  // r, ||r||^2
    if (!rc) rc = launch_dot(w.zp, w.x, Np, w.part, w.scal + 2, st);             // Z^T x
    if (!rc) rc = launch_dot(w.x, w.r, Np, w.part, w.scal + 3, st);              // x^T r
    prof_end(hi, st);
    double h[3] = {0.0, 0.0, 0.0};
    if (!rc) {
      hipMemcpyAsync(h, w.scal + 1, 3 * sizeof(double), hipMemcpyDeviceToHost, st);
      if (hipStreamSynchronize(st) != hipSuccess) rc = MVG_ERR_LAUNCH;
    }
    if (rc) break;
    // Z^T Sigma^-1 Z = Z^T x + x*^T r with x* = Sigma^-1 Z; x^T r estimates the
    // second term to first order, so q = Z^T x + x^T r is refined to second order
    const double rel = zn > 0.0 ? std::sqrt(h[0]) / zn : 0.0;
    stat->relres = rel;
    // a kept factor predicts with x itself: then only the residual criterion
    if (rel <= o.ir_tol || (!need_x && std::fabs(h[2]) <= IR_QUAD_TOL * std::fabs(h[1]))) {
      stat->converged = 1;
      break;
    }
    if (it >= o.ir_max_iter || !(rel < 0.5 * prev)) break;  // budget spent or stagnating
    prev = rel;
    int hc = prof_begin(MVG_PROF_IR, st, 2.0 * Nd * Nd, 8.0 * Nd * (Nd + 1) / 2);
    rc = trsv_forward(A, w.r, st);
    if (!rc) rc = trsv_backward(A, w.r, st);
    if (!rc) rc = launch_axpy(w.x, w.r, Np, st);
    prof_end(hc, st);
    stat->iters = it + 1;
  }
  if (!rc) {
    hipLaunchKernelGGL(k_add_pair, dim3(1), dim3(64), 0, st, (const double *)(w.scal + 2),
                       d_out2 + 1);
    rc = check_launch("add_pair");
  }
  return rc;
}

static int loglik_mixed(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
                        const mvg_theta *th, int n_theta, const mvg_opts &d, double *h_loglik,
                        double *h_logdet, double *h_quad, int64_t *h_status, mvg_factor **keep,
                        hipStream_t st) {
  mvg_opts d64 = d;
  d64.precision = MVG_FP64;
  mvg_mat *S = nullptr, *A = nullptr;
  int rc = mat_create(n_loc, d64, &th[0], d_x, d_y, st, &S);
  if (rc) return rc;
  rc = mat_create(n_loc, d, &th[0], d_x, d_y, st, &A);
  if (rc) {
    mat_free(S);
    return rc;
  }
  const int64_t Np = A->Np;
  const int64_t nt = (int64_t)A->T * (A->T + 1) / 2;
  const int nred = std::max(reduce_chunks(Np), (int)((A->N + 4095) / 4096));
  // zp x sx r yv (Np each) | part (2 nred) | sym (2 nt nb) | scal 8 | out2 | info
  const size_t ws_n = 5 * (size_t)Np + 2 * nred + 2 * (size_t)nt * A->nb + 8 + 2 * n_theta + n_theta;
  double *ws = nullptr;
  if (malloc_async((void **)&ws, sizeof(double) * ws_n, st) != hipSuccess) {
    hipGetLastError();
    mat_free(S);
    mat_free(A);
    set_error("workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  MixedWs w;
  w.zp = ws;
  w.x = ws + Np;
  w.sx = ws + 2 * Np;
  w.r = ws + 3 * Np;
  w.yv = ws + 4 * Np;
  w.part = ws + 5 * Np;
  w.sym = w.part + 2 * nred;
  w.scal = w.sym + 2 * nt * A->nb;
  double *d_out2 = w.scal + 8;
  int64_t *d_info = reinterpret_cast<int64_t *>(d_out2 + 2 * n_theta);
  g_ir.assign(n_theta, IrStat{0, 0, NAN});
  for (int i = 0; i < n_theta && !rc; ++i) {
    if (i > 0) {
      S->theta = A->theta = th[i];
      matern_setup(&th[i], &S->margs);
      A->margs = S->margs;
    }
    int hg = prof_begin(MVG_PROF_GEN, st, 0.0, 8.0 * (double)S->N * (S->N + 1) / 2);
    rc = mat_generate(S, st);
    prof_end(hg, st);
    if (!rc) rc = launch_quad_table(A->margs, A->d_qtab, st);  // for cokriging on A
    if (!rc) rc = eval_mixed(S, A, d_z, d, w, d_out2 + 2 * i, d_info + i, &g_ir[i],
                                keep != nullptr, st);
  }
  std::vector<double> out2(2 * n_theta);
  std::vector<int64_t> info(n_theta);
  hipMemcpyAsync(out2.data(), d_out2, sizeof(double) * 2 * n_theta, hipMemcpyDeviceToHost, st);
  hipMemcpyAsync(info.data(), d_info, sizeof(int64_t) * n_theta, hipMemcpyDeviceToHost, st);
  mvg_factor *F = nullptr;
  if (!rc && keep) {
    F = new mvg_factor();
    F->A = A;
    if (!(F->d_w = (double *)dev_alloc(sizeof(double) * Np * 2))) {
      hipGetLastError();
      rc = MVG_ERR_ALLOC;
      set_error("factor allocation failed");
    } else {
      F->d_y = F->d_w + Np;
      hipMemcpyAsync(F->d_y, w.yv, sizeof(double) * Np, hipMemcpyDeviceToDevice, st);
      hipMemcpyAsync(F->d_w, w.x, sizeof(double) * Np, hipMemcpyDeviceToDevice, st);
    }
  }
  hipFreeAsync(ws, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) {
    set_error("stream synchronisation failed: %s", hipGetErrorString(hipGetLastError()));
    rc = MVG_ERR_LAUNCH;
  }
  mat_free(S);
  if (rc) {
    if (F) {
      dev_free(F->d_w);
      delete F;
    }
    mat_free(A);
    return rc;
  }
  const double two_pi_term = (double)n_loc * std::log(2.0 * M_PI);
  for (int i = 0; i < n_theta; ++i) {
    const int64_t inf = info[i] == INT64_MAX ? 0 : info[i];
    if (h_status) h_status[i] = inf;
    if (inf) {
      h_loglik[i] = -INFINITY;
      if (h_logdet) h_logdet[i] = NAN;
      if (h_quad) h_quad[i] = NAN;
    } else {
      h_loglik[i] = -two_pi_term - 0.5 * out2[2 * i] - 0.5 * out2[2 * i + 1];
      if (h_logdet) h_logdet[i] = out2[2 * i];
      if (h_quad) h_quad[i] = out2[2 * i + 1];
    }
  }
  // two outcomes of the mixed factor say nothing about Sigma itself and are
  // evaluated again in FP64 (marked converged = -1 in mvg_ir_stats): a
  // non-positive pivot met by the low-precision updates (Sigma may still be
  // positive definite; the FP64 factor decides, and its pivot is the status),
  // and a refinement that stopped without meeting a criterion (sweep budget
  // or stagnation), which leaves x = Sigma^-1 Z, and so the quadratic form
  // and a kept factor's w, unconverged
  bool redo0 = false;
  for (int i = 0; i < n_theta && !rc; ++i) {
    if (info[i] == INT64_MAX && g_ir[i].converged) continue;
    if (i == 0 && F) {
      redo0 = true;
      continue;
    }
    int64_t s1 = 0;
    rc = loglik(d_x, d_y, d_z, n_loc, &th[i], 1, &d64, &h_loglik[i], h_logdet ? &h_logdet[i] : nullptr,
                h_quad ? &h_quad[i] : nullptr, &s1, nullptr, st);
    if (h_status) h_status[i] = s1;
    g_ir[i].converged = -1;
  }
  if (F && info[0] == INT64_MAX && !redo0 && !rc) {
    *keep = F;
    return 0;
  }
  if (F) {
    dev_free(F->d_w);
    delete F;
  }
  if (keep) *keep = nullptr;
  mat_free(A);
  if (!rc && redo0) {  // n_theta == 1 with a kept factor: the FP64 factor instead
    int64_t s1 = 0;
    rc = loglik(d_x, d_y, d_z, n_loc, &th[0], 1, &d64, &h_loglik[0], h_logdet, h_quad, &s1, keep,
                st);
    if (h_status) h_status[0] = s1;
    g_ir[0].converged = -1;
  }
  return rc;
}

static int run_small(const std::vector<SmallTask> &tasks, int64_t nmax, double *h_loglik,
                     double *h_logdet, double *h_quad, int64_t *h_status, hipStream_t st) {
  const int nt = (int)tasks.size();
  const int G = small_batch_workgroups(nt);
  const size_t wsd = small_workspace_doubles(nmax) * (size_t)G;
  char *buf = nullptr;
  const size_t tb = sizeof(SmallTask) * nt, ob = sizeof(double) * 4 * nt;
  const size_t bytes = tb + ob + sizeof(double) * wsd + 256;
  if (malloc_async((void **)&buf, bytes, st) != hipSuccess) {
    hipGetLastError();
    set_error("batched likelihood workspace of %.2f GB failed", bytes / 1e9);
    return MVG_ERR_ALLOC;
  }
  SmallTask *d_tasks = (SmallTask *)buf;
  double *d_out = (double *)(buf + (tb + 255) / 256 * 256);
  int *d_counter = (int *)(d_out + 4 * nt);
  double *d_ws = (double *)((char *)d_counter + 256);
  hipMemcpyAsync(d_tasks, tasks.data(), tb, hipMemcpyHostToDevice, st);
  int hp = prof_begin(MVG_PROF_POTRF, st, 0.0, 0.0);
  int rc = launch_small_loglik(d_tasks, nt, nmax, d_counter, d_ws, d_out, st);
  prof_end(hp, st);
  std::vector<double> out(4 * nt);
  if (!rc) hipMemcpyAsync(out.data(), d_out, ob, hipMemcpyDeviceToHost, st);
  hipFreeAsync(buf, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) {
    set_error("batched likelihood failed: %s", hipGetErrorString(hipGetLastError()));
    rc = MVG_ERR_LAUNCH;
  }
  if (rc) return rc;
  for (int i = 0; i < nt; ++i) {
    h_loglik[i] = out[4 * i];
    if (h_logdet) h_logdet[i] = out[4 * i + 1];
    if (h_quad) h_quad[i] = out[4 * i + 2];
    if (h_status) h_status[i] = (int64_t)out[4 * i + 3];
  }
  return 0;
}


int loglik_many(const mvg_task *h_tasks, int n_tasks, double *h_loglik, double *h_logdet,
                double *h_quad, int64_t *h_status, void *hip_stream) {
  if (!h_tasks) return -1;
  if (n_tasks < 1) return -2;
  if (!h_loglik) return -3;
  std::vector<SmallTask> tasks;
  int64_t nmax = 1;
  for (int i = 0; i < n_tasks; ++i) {
    const mvg_task &t = h_tasks[i];
    MaternArgs tmp;
    if (!t.x || !t.y || !t.z || t.n_loc < 1 || 2 * t.n_loc > SMALL_MAX ||
        matern_setup(&t.theta, &tmp))
      return -(100 + i);
    tasks.push_back(small_task(t.x, t.y, t.z, t.n_loc, t.theta));
    nmax = std::max(nmax, t.n_loc);
  }
  return run_small(tasks, nmax, h_loglik, h_logdet, h_quad, h_status, (hipStream_t)hip_stream);
}

// Several theta as independent evaluations on concurrent streams (one host
// thread and stream each, up to 4 at a time (MVG_TLR_CONCURRENT, at most 8)
// and as many as the free device memory holds).  A TLR evaluation is bound
// by its column-by-column critical path (the compressions of a tile column,
// then a host synchronisation for their ranks), so several together fill
// the device better: 7 theta at n = 100,000 in 22.7 s with 4 at a time,
// 25.7 s with 2, 26.5 s one after another; each result is the one a single
// call gives.
constexpr int TLR_CONCURRENT = 8;
constexpr int TLR_CONCURRENT_DEFAULT = 4;

static int loglik_concurrent(const double *d_x, const double *d_y, const double *d_z,
                             int64_t n_loc, const mvg_theta *th, int n_theta, const mvg_opts &d,
                             double *h_loglik, double *h_logdet, double *h_quad,
                             int64_t *h_status, hipStream_t st) {
  if (hipStreamSynchronize(st) != hipSuccess) {  // the inputs are ready on the caller's stream
    set_error("stream synchronisation failed");
    return MVG_ERR_LAUNCH;
  }
  int dev = 0;
  hipGetDevice(&dev);
  size_t free_b = 0, total_b = 0;
  hipMemGetInfo(&free_b, &total_b);
  const size_t need = std::max<size_t>(1, mvg_footprint(n_loc, &d));
  static const size_t conc = [] {  // MVG_TLR_CONCURRENT: at most this many at once
    const char *e = getenv("MVG_TLR_CONCURRENT");
    return (size_t)(e && atoi(e) > 0 ? std::min(atoi(e), TLR_CONCURRENT) : TLR_CONCURRENT_DEFAULT);
  }();
  const int nw = (int)std::max<size_t>(
      1, std::min<size_t>({(size_t)n_theta, conc, free_b / need}));
  std::atomic<int> next{0};
  std::vector<int> rcs(nw, 0);
  std::vector<std::string> errs(nw);
  std::vector<std::thread> pool;
  for (int w = 0; w < nw; ++w)
    pool.emplace_back([&, w] {
      hipSetDevice(dev);
      hipStream_t s = nullptr;
      if (hipStreamCreate(&s) != hipSuccess) {
        rcs[w] = MVG_ERR_LAUNCH;
        errs[w] = "stream creation failed";
        return;
      }
      for (;;) {
        const int i = next++;
        if (i >= n_theta) break;
        const int rc = loglik(d_x, d_y, d_z, n_loc, &th[i], 1, &d, &h_loglik[i],
                              h_logdet ? &h_logdet[i] : nullptr, h_quad ? &h_quad[i] : nullptr,
                              h_status ? &h_status[i] : nullptr, nullptr, s);
        if (rc) {
          rcs[w] = rc;
          errs[w] = mvg_last_error();
          break;
        }
      }
      hipStreamSynchronize(s);
      hipStreamDestroy(s);
    });
  for (auto &t : pool) t.join();
  for (int w = 0; w < nw; ++w)
    if (rcs[w]) {
      set_error("%s", errs[w].c_str());
      return rcs[w];
    }
  return 0;
}

// ------------------------------------------------------------ autotuning

static std::mutex g_tune_mu;
static std::map<std::tuple<int64_t, int, int>, int> g_tune;  // (n_loc, precision, band) -> nb

static bool tunable(int precision) {
  return precision == MVG_FP64 || precision == MVG_DST || is_mixed(precision);
}

int mvg_autotune_nb(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
                    const mvg_theta *th, const mvg_opts *o, const int *cand, int n_cand,
                    int *best_nb, double *h_seconds, void *hip_stream) {
  if (!d_x || !d_y || !d_z) return -1;
  if (n_loc < 1) return -4;
  MaternArgs tmp;
  if (!th || matern_setup(th, &tmp)) return -5;
  mvg_opts base{};
  if (o) base = *o;
  base.nb = 0;
  mvg_opts d;
  if (normalize_opts(&base, &d) || !tunable(d.precision)) return -6;
  static const int dflt[4] = {256, 512, 768, 1024};
  if (!cand) {
    cand = dflt;
    n_cand = 4;
  }
  if (n_cand < 1 || n_cand > 16) return -8;
  for (int i = 0; i < n_cand; ++i)
    if (cand[i] != 128 && cand[i] != 256 && cand[i] != 512 && cand[i] != 768 && cand[i] != 1024)
      return -7;
  if (!best_nb) return -9;
  const auto key = std::make_tuple(n_loc, d.precision, d.band_tiles);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *best_nb = it->second;
      return 1;
    }
  }
  hipStream_t st = (hipStream_t)hip_stream;
  double best_t = INFINITY;
  int best = 0;
  for (int i = 0; i < n_cand; ++i) {
    mvg_opts c = d;
    c.nb = cand[i];
    double ll = 0.0, t = INFINITY;
    int rc = loglik(d_x, d_y, d_z, n_loc, th, 1, &c, &ll, nullptr, nullptr, nullptr, nullptr, st);
    if (!rc) {
      const auto t0 = std::chrono::steady_clock::now();
      rc = loglik(d_x, d_y, d_z, n_loc, th, 1, &c, &ll, nullptr, nullptr, nullptr, nullptr, st);
      if (!rc) t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (rc && rc != MVG_ERR_ALLOC) return rc;  // a tile too large for memory is just skipped
    if (h_seconds) h_seconds[i] = t;
    if (t < best_t) {
      best_t = t;
      best = cand[i];
    }
  }
  if (!best) {
    set_error("autotune: no candidate tile size ran");
    return MVG_ERR_ALLOC;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
  }
  *best_nb = best;
  return 0;
}

int loglik(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
           const mvg_theta *th, int n_theta, const mvg_opts *o, double *h_loglik,
           double *h_logdet, double *h_quad, int64_t *h_status, mvg_factor **keep,
           void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (!d_z) return -3;
  if (n_loc < 1) return -4;
  if (!th) return -5;
  if (n_theta < 1) return -6;
  if (o && o->nb == MVG_NB_AUTO) {  // resolve the tile size, then evaluate as usual
    if (!tunable(o->precision)) return -7;
    mvg_opts c = *o;
    int rc = mvg_autotune_nb(d_x, d_y, d_z, n_loc, &th[0], o, nullptr, 0, &c.nb, nullptr,
                             hip_stream);
    if (rc < 0) return rc;
    return loglik(d_x, d_y, d_z, n_loc, th, n_theta, &c, h_loglik, h_logdet, h_quad, h_status,
                  keep, hip_stream);
  }
  mvg_opts d;
  if (normalize_opts(o, &d)) return -7;
  if (!h_loglik) return -8;
  if (keep && n_theta != 1) return -12;
  for (int i = 0; i < n_theta; ++i) {
    MaternArgs tmp;
    if (matern_setup(&th[i], &tmp)) return -5;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (d.precision == MVG_FP64 && n_theta > 1 && 2 * n_loc <= SMALL_MAX && !keep) {
    std::vector<SmallTask> tasks;
    for (int i = 0; i < n_theta; ++i) tasks.push_back(small_task(d_x, d_y, d_z, n_loc, th[i]));
    return run_small(tasks, n_loc, h_loglik, h_logdet, h_quad, h_status, st);
  }
  if (is_mixed(d.precision))
    return loglik_mixed(d_x, d_y, d_z, n_loc, th, n_theta, d, h_loglik, h_logdet, h_quad,
                        h_status, keep, st);
  if (d.precision == MVG_TLR && n_theta > 1 && !keep)
    return loglik_concurrent(d_x, d_y, d_z, n_loc, th, n_theta, d, h_loglik, h_logdet, h_quad,
                             h_status, st);
  const bool tlr = d.precision == MVG_TLR;
  mvg_mat *A = nullptr;
  int rc = tlr ? tlr_mat_create(n_loc, d, &th[0], d_x, d_y, st, &A)
               : mat_create(n_loc, d, &th[0], d_x, d_y, st, &A);
  if (rc) return rc;
  const int nred = (int)((A->N + 4095) / 4096);
  double *ws = nullptr;  // y (Np) | part (2 nred) | out2 (2 n_theta) | info (n_theta)
  const size_t ws_n = (size_t)A->Np + 2 * nred + 2 * n_theta + n_theta;
  if (malloc_async((void **)&ws, sizeof(double) * ws_n, st) != hipSuccess) {
    hipGetLastError();
    mat_free(A);
    set_error("workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  double *d_yv = ws, *d_part = ws + A->Np, *d_out2 = d_part + 2 * nred;
  int64_t *d_info = reinterpret_cast<int64_t *>(d_out2 + 2 * n_theta);
  for (int i = 0; i < n_theta && !rc; ++i) {
    if (i > 0) {
      A->theta = th[i];
      matern_setup(&th[i], &A->margs);
    }
    const double npair = (double)n_loc * (n_loc + 1) / 2;
    int hg = prof_begin(MVG_PROF_GEN, st, 0.0, 8.0 * (double)A->N * (A->N + 1) / 2);
    rc = tlr ? tlr_generate(A, st) : mat_generate(A, st);
    prof_end(hg, st);
    (void)npair;
    if (!rc) rc = eval_one(A, d_z, d_yv, d_part, d_out2 + 2 * i, d_info + i, st);
  }
  std::vector<double> out2(2 * n_theta);
  std::vector<int64_t> info(n_theta);
  hipMemcpyAsync(out2.data(), d_out2, sizeof(double) * 2 * n_theta, hipMemcpyDeviceToHost, st);
  hipMemcpyAsync(info.data(), d_info, sizeof(int64_t) * n_theta, hipMemcpyDeviceToHost, st);
  mvg_factor *F = nullptr;
  if (!rc && keep) {
    F = new mvg_factor();
    F->A = A;
    if (!(F->d_w = (double *)dev_alloc(sizeof(double) * A->Np * 2))) {
      hipGetLastError();
      rc = MVG_ERR_ALLOC;
      set_error("factor allocation failed");
    } else {
      F->d_y = F->d_w + A->Np;
      hipMemcpyAsync(F->d_y, d_yv, sizeof(double) * A->Np, hipMemcpyDeviceToDevice, st);
      hipMemcpyAsync(F->d_w, d_yv, sizeof(double) * A->Np, hipMemcpyDeviceToDevice, st);
      rc = trsv_backward(A, F->d_w, st);
    }
  }
  hipFreeAsync(ws, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) {
    set_error("stream synchronisation failed: %s", hipGetErrorString(hipGetLastError()));
    rc = MVG_ERR_LAUNCH;
  }
  if (rc) {
    if (F) {
      dev_free(F->d_w);
      delete F;
    }
    mat_free(A);
    return rc;
  }
  const double two_pi_term = (double)n_loc * std::log(2.0 * M_PI);
  for (int i = 0; i < n_theta; ++i) {
    const int64_t inf = info[i] == INT64_MAX ? 0 : info[i];
    if (h_status) h_status[i] = inf;
    if (inf) {
      h_loglik[i] = -INFINITY;
      if (h_logdet) h_logdet[i] = NAN;
      if (h_quad) h_quad[i] = NAN;
    } else {
      h_loglik[i] = -two_pi_term - 0.5 * out2[2 * i] - 0.5 * out2[2 * i + 1];
      if (h_logdet) h_logdet[i] = out2[2 * i];
      if (h_quad) h_quad[i] = out2[2 * i + 1];
    }
  }
  if (F) {
    if (info[0] != INT64_MAX) {  // a failed factor cannot predict
      dev_free(F->d_w);
      delete F;
      mat_free(A);
      *keep = nullptr;
    } else {
      *keep = F;
    }
  } else {
    mat_free(A);
  }
  return 0;
}

// ------------------------------------------------------------ p variables

static bool p_precision_ok(const mvg_opts &d) {
  return d.precision == MVG_FP64 || d.precision == MVG_DST;
}

int cov_generate_p(const double *d_x, const double *d_y, int64_t n_loc, const mvg_theta_p *th,
                   const mvg_opts *o, mvg_mat **out, void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (n_loc < 1) return -3;
  if (!th) return -4;
  mvg_opts d;
  if (normalize_opts(o, &d)) return -5;
  if (!out) return -6;
  MaternArgsP tmp;
  if (matern_setup_p(th, &tmp)) return -4;
  if (th->p == 2) {
    const mvg_theta t2 = theta_from_p(*th);
    return cov_generate(d_x, d_y, n_loc, &t2, o, out, hip_stream);
  }
  if (!p_precision_ok(d)) return -5;
  hipStream_t st = (hipStream_t)hip_stream;
  mvg_mat *A = nullptr;
  if (int rc = mat_create_p(n_loc, d, th, d_x, d_y, st, &A)) return rc < 0 && rc > -100 ? -4 : rc;
  if (int rc = mat_generate(A, st)) {
    mat_free(A);
    return rc;
  }
  if (int rc = mark_done(A, st)) {
    hipStreamSynchronize(st);
    mat_free(A);
    return rc;
  }
  *out = A;
  return 0;
}

// Eq. (1) for p != 2 variables, n_theta thetas on one matrix (FP64 / DST).
static int loglik_p_run(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
                        const mvg_theta_p *th, int n_theta, const mvg_opts &d, double *h_loglik,
                        double *h_logdet, double *h_quad, int64_t *h_status, hipStream_t st) {
  mvg_mat *A = nullptr;
  int rc = mat_create_p(n_loc, d, &th[0], d_x, d_y, st, &A);
  if (rc) return rc;
  const int nred = (int)((A->N + 4095) / 4096);
  double *ws = nullptr;  // y (Np) | part (2 nred) | out2 (2 n_theta) | info (n_theta)
  const size_t ws_n = (size_t)A->Np + 2 * nred + 2 * n_theta + n_theta;
  if (malloc_async((void **)&ws, sizeof(double) * ws_n, st) != hipSuccess) {
    hipGetLastError();
    mat_free(A);
    set_error("workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  double *d_yv = ws, *d_part = ws + A->Np, *d_out2 = d_part + 2 * nred;
  int64_t *d_info = reinterpret_cast<int64_t *>(d_out2 + 2 * n_theta);
  for (int i = 0; i < n_theta && !rc; ++i) {
    if (i > 0) {
      A->theta_p = th[i];
      matern_setup_p(&th[i], &A->margs_p);
    }
    int hg = prof_begin(MVG_PROF_GEN, st, 0.0, 8.0 * (double)A->N * (A->N + 1) / 2);
    rc = mat_generate(A, st);
    prof_end(hg, st);
    if (!rc) rc = eval_one(A, d_z, d_yv, d_part, d_out2 + 2 * i, d_info + i, st);
  }
  std::vector<double> out2(2 * n_theta);
  std::vector<int64_t> info(n_theta);
  hipMemcpyAsync(out2.data(), d_out2, sizeof(double) * 2 * n_theta, hipMemcpyDeviceToHost, st);
  hipMemcpyAsync(info.data(), d_info, sizeof(int64_t) * n_theta, hipMemcpyDeviceToHost, st);
  hipFreeAsync(ws, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) {
    set_error("stream synchronisation failed: %s", hipGetErrorString(hipGetLastError()));
    rc = MVG_ERR_LAUNCH;
  }
  const double two_pi_term = 0.5 * (double)A->N * std::log(2.0 * M_PI);
  mat_free(A);
  if (rc) return rc;
  for (int i = 0; i < n_theta; ++i) {
    const int64_t inf = info[i] == INT64_MAX ? 0 : info[i];
    if (h_status) h_status[i] = inf;
    if (inf) {
      h_loglik[i] = -INFINITY;
      if (h_logdet) h_logdet[i] = NAN;
      if (h_quad) h_quad[i] = NAN;
    } else {
      h_loglik[i] = -two_pi_term - 0.5 * out2[2 * i] - 0.5 * out2[2 * i + 1];
      if (h_logdet) h_logdet[i] = out2[2 * i];
      if (h_quad) h_quad[i] = out2[2 * i + 1];
    }
  }
  return 0;
}

int loglik_p(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
             const mvg_theta_p *th, int n_theta, const mvg_opts *o, double *h_loglik,
             double *h_logdet, double *h_quad, int64_t *h_status, void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (!d_z) return -3;
  if (n_loc < 1) return -4;
  if (!th || n_theta < 1) return -5;
  mvg_opts d;
  if (normalize_opts(o, &d)) return -7;
  if (!h_loglik) return -8;
  const int p = th[0].p;
  for (int i = 0; i < n_theta; ++i) {
    MaternArgsP tmp;
    if (th[i].p != p || matern_setup_p(&th[i], &tmp)) return -5;
  }
  if (p == 2) {
    std::vector<mvg_theta> t2;
    for (int i = 0; i < n_theta; ++i) t2.push_back(theta_from_p(th[i]));
    return loglik(d_x, d_y, d_z, n_loc, t2.data(), n_theta, o, h_loglik, h_logdet, h_quad,
                  h_status, nullptr, hip_stream);
  }
  if (!p_precision_ok(d)) {
    set_error("p = %d variables: precision must be FP64 or DST", p);
    return -7;
  }
  return loglik_p_run(d_x, d_y, d_z, n_loc, th, n_theta, d, h_loglik, h_logdet, h_quad, h_status,
                      (hipStream_t)hip_stream);
}


int profile_loglik_p(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
                     const mvg_theta_p *th, const mvg_opts *o, double *h_sigma_sq,
                     double *h_loglik, double *h_logdet, double *h_quad, int64_t *h_status,
                     void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (!d_z) return -3;
  if (n_loc < 1) return -4;
  if (!th) return -5;
  mvg_theta_p t = *th;
  MaternArgsP tmp;
  if (t.p < 1 || t.p > PMAX) return -5;
  for (int i = 0; i < t.p; ++i) t.sigma_sq[i] = 1.0;  // not read: only the shape is checked
  if (matern_setup_p(&t, &tmp)) return -5;
  mvg_opts d;
  if (normalize_opts(o, &d)) return -6;
  if (!h_sigma_sq) return -7;
  if (!h_loglik) return -8;
  hipStream_t st = (hipStream_t)hip_stream;
  const int p = t.p;
  // marginal variances: Z_i^T R_ii^-1 Z_i / n with R_ii univariate, unit variance (FP64)
  double *zi = nullptr;
  if (malloc_async((void **)&zi, sizeof(double) * n_loc, st) != hipSuccess) {
    hipGetLastError();
    set_error("workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  mvg_opts d1 = d;
  d1.precision = MVG_FP64;
  int rc = 0;
  for (int i = 0; i < p && !rc; ++i) {
    hipLaunchKernelGGL(k_stride_copy, dim3((unsigned)((n_loc + 255) / 256)), dim3(256), 0, st, d_z,
                       p, i, n_loc, zi);
    rc = check_launch("stride_copy");
    mvg_theta_p u{};
    u.p = 1;
    u.sigma_sq[0] = 1.0;
    u.a = t.a;
    u.nu[0] = t.nu[i];
    u.beta[0] = 1.0;
    double ll = 0.0, q = 0.0;
    int64_t status = 0;
    if (!rc) rc = loglik_p_run(d_x, d_y, zi, n_loc, &u, 1, d1, &ll, nullptr, &q, &status, st);
    if (!rc && status) {
      hipFreeAsync(zi, st);
      hipStreamSynchronize(st);
      *h_loglik = -INFINITY;
      if (h_logdet) *h_logdet = NAN;
      if (h_quad) *h_quad = NAN;
      if (h_status) *h_status = -(1 + i);
      for (int k = 0; k < p; ++k) h_sigma_sq[k] = NAN;
      return 0;
    }
    t.sigma_sq[i] = q / (double)n_loc;
  }
  hipFreeAsync(zi, st);
  if (rc) {
    hipStreamSynchronize(st);
    return rc;
  }
  for (int i = 0; i < p; ++i) h_sigma_sq[i] = t.sigma_sq[i];
  // Eq. (1) at the profiled variances
  return loglik_p(d_x, d_y, d_z, n_loc, &t, 1, o, h_loglik, h_logdet, h_quad, h_status, hip_stream);
}


// Section 5.4, Eq. (5)-(8), Algorithm 1 on two dense FP64 factors.
int mloe_mmom(const double *d_x, const double *d_y, int64_t n_loc, const mvg_theta *th,
              const mvg_theta *th_a, const double *d_x0, const double *d_y0, int64_t m,
              const mvg_opts *o, double *h_mloe, double *h_mmom, double *d_loe, double *d_mom,
              void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (n_loc < 1) return -3;
  if (!th) return -4;
  if (!th_a) return -5;
  if (!d_x0) return -6;
  if (!d_y0) return -7;
  if (m < 1 || m > 65535) return -8;
  mvg_opts d;
  if (normalize_opts(o, &d) || d.precision != MVG_FP64) return -9;
  if (!h_mloe || !h_mmom) return -10;
  MaternArgs tmp;
  if (matern_setup(th, &tmp)) return -4;
  if (matern_setup(th_a, &tmp)) return -5;
  hipStream_t st = (hipStream_t)hip_stream;
  mvg_mat *A = nullptr, *Aa = nullptr;
  int rc = mat_create(n_loc, d, th, d_x, d_y, st, &A);
  if (!rc) rc = mat_create(n_loc, d, th_a, d_x, d_y, st, &Aa);
  if (rc) {
    mat_free(A);
    return rc;
  }
  const int64_t Np = A->Np, k2 = 2 * m;
  double *ws = nullptr;  // C0t | X1 | X2 | X3 (Np x 2m) | sT sA dT sQ (2m) | loe mom (m) | info 2
  const size_t wn = 4 * (size_t)Np * k2 + 4 * k2 + 2 * m + 2;
  if (malloc_async((void **)&ws, sizeof(double) * wn, st) != hipSuccess) {
    hipGetLastError();
    mat_free(A);
    mat_free(Aa);
    set_error("MLOE/MMOM workspace of %.2f GB failed", wn * 8.0 / 1e9);
    return MVG_ERR_ALLOC;
  }
  double *C0t = ws, *X1 = C0t + Np * k2, *X2 = X1 + Np * k2, *X3 = X2 + Np * k2;
  double *sT = X3 + Np * k2, *sA = sT + k2, *dT = sA + k2, *sQ = dT + k2;
  double *loe = sQ + k2, *mom = loe + m;
  int64_t *info = reinterpret_cast<int64_t *>(mom + m);
  // Sigma(theta) = L L^T, Sigma(theta_a) = L_a L_a^T
  int hg = prof_begin(MVG_PROF_GEN, st, 0.0, 8.0 * (double)A->N * (A->N + 1));
  rc = mat_generate(A, st);
  if (!rc) rc = mat_generate(Aa, st);
  prof_end(hg, st);
  if (!rc) rc = launch_fill_i64(info, INT64_MAX, 2, st);
  const double Nd = (double)A->N;
  int hp = prof_begin(MVG_PROF_POTRF, st, 2.0 * (Nd * Nd * Nd / 3.0 + Nd * Nd / 2.0), 0.0);
  if (!rc) rc = dense_potrf(A, info, st);
  if (!rc) rc = dense_potrf(Aa, info + 1, st);
  prof_end(hp, st);
  // forward solves (3), backward solve, L^T product: N^2 k2 flops each
  int hs = prof_begin(MVG_PROF_SOLVE, st, 5.0 * Nd * Nd * (double)k2, 0.0);
  // E_t: ||L^-1 c0_t||^2 per column
  if (!rc) rc = launch_cokrige_c0(A->margs, A->d_qtab, A->d_x, A->d_y, n_loc, Np, d_x0, d_y0, m,
                                  C0t, st);
  if (!rc && hipMemcpyAsync(X1, C0t, sizeof(double) * Np * k2, hipMemcpyDeviceToDevice, st))
    rc = MVG_ERR_LAUNCH;
  if (!rc) rc = trsm_forward_multi(A, X1, (int)k2, st);
  if (!rc) rc = launch_sum_sq_cols(X1, Np, (int)k2, sT, st);
  // E_a: ||L_a^-1 c0_a||^2; w_a = Sigma_a^-1 c0_a
  if (!rc) rc = launch_cokrige_c0(Aa->margs, Aa->d_qtab, Aa->d_x, Aa->d_y, n_loc, Np, d_x0, d_y0,
                                  m, X2, st);
  if (!rc) rc = trsm_forward_multi(Aa, X2, (int)k2, st);
  if (!rc) rc = launch_sum_sq_cols(X2, Np, (int)k2, sA, st);
  if (!rc) rc = trsm_backward_multi(Aa, X2, (int)k2, st);
  // E_{t,a}: c0_t . w_a and ||L^T w_a||^2
  if (!rc) rc = launch_dot_cols(C0t, X2, Np, (int)k2, dT, st);
  if (!rc) rc = launch_trmm_t(A, X2, X3, (int)k2, st);
  if (!rc) rc = launch_sum_sq_cols(X3, Np, (int)k2, sQ, st);
  prof_end(hs, st);
  if (!rc) {
    hipLaunchKernelGGL(k_loe_mom, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                       (const double *)sT, (const double *)sA, (const double *)dT,
                       (const double *)sQ, m, th->sigma11_sq + th->sigma22_sq,
                       th_a->sigma11_sq + th_a->sigma22_sq, d_loe ? d_loe : loe,
                       d_mom ? d_mom : mom);
    rc = check_launch("loe_mom");
  }
  std::vector<double> hl(m), hm(m);
  int64_t hinfo[2] = {0, 0};
  if (!rc) {
    hipMemcpyAsync(hl.data(), d_loe ? d_loe : loe, sizeof(double) * m, hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(hm.data(), d_mom ? d_mom : mom, sizeof(double) * m, hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, st);
  }
  hipFreeAsync(ws, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = MVG_ERR_LAUNCH;
  mat_free(A);
  mat_free(Aa);
  if (rc) return rc;
  if (hinfo[0] != INT64_MAX || hinfo[1] != INT64_MAX) {
    set_error("MLOE/MMOM: a covariance matrix is not positive definite (pivot %lld / %lld)",
              (long long)(hinfo[0] == INT64_MAX ? 0 : hinfo[0]),
              (long long)(hinfo[1] == INT64_MAX ? 0 : hinfo[1]));
    return hinfo[0] != INT64_MAX ? 1 : 2;
  }
  double a = 0.0, b = 0.0;
  for (int64_t l = 0; l < m; ++l) {
    a += hl[l];
    b += hm[l];
  }
  *h_mloe = a / (double)m;
  *h_mmom = b / (double)m;
  return 0;
}

int cokrige_predict(const mvg_factor *F, const double *d_x0, const double *d_y0, int64_t m,
                    double *d_zhat, double *d_mse, void *hip_stream) {
  if (!F || !F->A || !F->d_w) return -1;
  if (!d_x0) return -2;
  if (!d_y0) return -3;
  if (m < 1 || m > 65535) return -4;
  if (!d_zhat) return -5;
  hipStream_t st = (hipStream_t)hip_stream;
  const mvg_mat *A = F->A;
  const int nchunk = (int)((A->n_loc + 2047) / 2048);
  int hc = prof_begin(MVG_PROF_COKRIGE, st, 0.0, 8.0 * (double)A->N);
  double *part = nullptr;
  if (malloc_async((void **)&part, sizeof(double) * 2 * m * nchunk, st) != hipSuccess) {
    hipGetLastError();
    set_error("workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  int rc = launch_cokrige_dot(A->margs, A->d_qtab, A->d_x, A->d_y, A->n_loc, d_x0, d_y0, m,
                              F->d_w, part, nchunk, st);
  if (!rc) {
    hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)((2 * m + 255) / 256)), dim3(256), 0, st,
                       (const double *)part, m, nchunk, d_zhat);
    rc = check_launch("reduce_chunks");
  }
  hipFreeAsync(part, st);
  prof_end(hc, st);
  if (!rc && d_mse) {
    double *V = nullptr, *ss = nullptr;
    if (malloc_async((void **)&V, sizeof(double) * (A->Np * 2 * m + 2 * m), st) != hipSuccess) {
      hipGetLastError();
      set_error("workspace allocation failed");
      return MVG_ERR_ALLOC;
    }
    ss = V + A->Np * 2 * m;
    rc = launch_cokrige_c0(A->margs, A->d_qtab, A->d_x, A->d_y, A->n_loc, A->Np, d_x0, d_y0, m, V,
                           st);
    if (!rc) rc = trsm_forward_multi(A, V, (int)(2 * m), st);
    if (!rc) rc = launch_sum_sq_cols(V, A->Np, (int)(2 * m), ss, st);
    if (!rc) {
      hipLaunchKernelGGL(k_mse_final, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                         (const double *)ss, m, A->theta.sigma11_sq + A->theta.sigma22_sq, d_mse);
      rc = check_launch("mse_final");
    }
    hipFreeAsync(V, st);
  }
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = MVG_ERR_LAUNCH;
  return rc;
}

int morton_order(const double *d_x, const double *d_y, int64_t n_loc, int64_t *d_perm,
                 double *d_xs, double *d_ys, void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (n_loc < 1 || n_loc > ((int64_t)1 << 26)) return -3;
  if (!d_perm) return -4;
  if (d_xs && (d_xs == d_x || d_xs == d_y)) return -5;
  if (d_ys && (d_ys == d_x || d_ys == d_y || d_ys == d_xs)) return -6;
  return morton_sort(d_x, d_y, n_loc, d_perm, d_xs, d_ys, (hipStream_t)hip_stream);
}

int mvg_trmv(const mvg_mat *L, const double *d_eps, double *d_z, void *hip_stream) {
  if (!L || !L->factored || L->precision != MVG_FP64) return -1;
  if (!d_eps) return -2;
  if (!d_z || d_z == d_eps) return -3;
  if (int rc = launch_trmv(L, d_eps, d_z, (hipStream_t)hip_stream)) return rc;
  return mark_done(L, (hipStream_t)hip_stream);
}

int mvg_mat_loglik(const mvg_mat *L, const double *d_z, double *h_loglik, double *h_logdet,
                   double *h_quad, void *hip_stream) {
  if (!L || !L->factored || L->precision != MVG_FP64) return -1;
  if (!d_z) return -2;
  if (!h_loglik) return -3;
  hipStream_t st = (hipStream_t)hip_stream;
  const int nred = (int)((L->N + 4095) / 4096);
  double *ws = nullptr;  // y (Np) | part (2 nred) | out2 (2)
  if (malloc_async((void **)&ws, sizeof(double) * ((size_t)L->Np + 2 * nred + 2), st) !=
      hipSuccess) {
    hipGetLastError();
    set_error("workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  double *d_y = ws, *d_part = ws + L->Np, *d_out2 = d_part + 2 * nred;
  hipLaunchKernelGGL(k_copy_pad, dim3((unsigned)((L->Np + 255) / 256)), dim3(256), 0, st, d_z,
                     L->N, d_y, L->Np);
  int rc = check_launch("copy_pad");
  if (!rc) rc = trsv_forward(L, d_y, st);
  if (!rc) rc = logdet_quad(L, d_y, d_part, d_out2, st);
  double out2[2] = {0.0, 0.0};
  if (!rc) hipMemcpyAsync(out2, d_out2, sizeof(out2), hipMemcpyDeviceToHost, st);
  hipFreeAsync(ws, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) {
    set_error("stream synchronisation failed: %s", hipGetErrorString(hipGetLastError()));
    rc = MVG_ERR_LAUNCH;
  }
  if (rc) return rc;
  *h_loglik = -(double)L->n_loc * (L->p / 2.0) * std::log(2.0 * M_PI) - 0.5 * out2[0] -
              0.5 * out2[1];
  if (h_logdet) *h_logdet = out2[0];
  if (h_quad) *h_quad = out2[1];
  return 0;
}

int mvg_mat_nvar(const mvg_mat *A) { return A ? A->p : -1; }

int mvg_mat_shape(const mvg_mat *A, int64_t *n_loc, int *nb, int *ntiles, int *precision,
                  int *factored) {
  if (!A) return -1;
  if (n_loc) *n_loc = A->n_loc;
  if (nb) *nb = A->nb;
  if (ntiles) *ntiles = A->T;
  if (precision) *precision = A->precision;
  if (factored) *factored = A->factored;
  return 0;
}

int mvg_mat_gather(const mvg_mat *A, const int64_t *d_rows, const int64_t *d_cols, int64_t m,
                   double *d_out, void *hip_stream) {
  if (!A || A->precision == MVG_TLR) return -1;
  if (!d_rows) return -2;
  if (!d_cols) return -3;
  if (m < 0) return -4;
  if (!d_out) return -5;
  if (int rc = launch_gather(A, d_rows, d_cols, m, d_out, (hipStream_t)hip_stream)) return rc;
  return mark_done(A, (hipStream_t)hip_stream);
}

int mvg_mat_to_dense(const mvg_mat *A, double *d_out, int64_t ld, void *hip_stream) {
  if (!A) return -1;
  if (!d_out) return -2;
  if (ld < A->N) return -3;
  hipStream_t st = (hipStream_t)hip_stream;
  const int rc = A->precision == MVG_TLR ? tlr_to_dense(A, d_out, ld, st)
                                         : launch_to_dense(A, d_out, ld, st);
  if (rc) return rc;
  return mark_done(A, st);
}

const mvg_mat *mvg_factor_mat(const mvg_factor *F) { return F ? F->A : nullptr; }
const double *mvg_factor_w(const mvg_factor *F) { return F ? F->d_w : nullptr; }

void mvg_mat_destroy(mvg_mat *A) {
  if (!A) return;
  if (A->done) hipEventSynchronize(A->done);  // the library's asynchronous work on A
  mat_free(A);
}

void mvg_factor_destroy(mvg_factor *F) {
  if (!F) return;
  if (F->A && F->A->done) hipEventSynchronize(F->A->done);
  dev_free(F->d_w);
  mat_free(F->A);
  delete F;
}

int tlr_compress(const double *d_x, const double *d_y, int64_t n_loc, const mvg_theta *th,
                 const mvg_opts *o, mvg_mat **out, int32_t *h_ranks, void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (n_loc < 1) return -3;
  if (!th) return -4;
  mvg_opts d;
  if (!o || o->precision != MVG_TLR || normalize_opts(o, &d)) return -5;
  if (!out) return -6;
  MaternArgs tmp;
  if (matern_setup(th, &tmp)) return -4;
  hipStream_t st = (hipStream_t)hip_stream;
  mvg_mat *A = nullptr;
  if (int rc = tlr_mat_create(n_loc, d, th, d_x, d_y, st, &A)) return rc < 0 && rc > -100 ? -4 : rc;
  int rc = tlr_generate(A, st);
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = MVG_ERR_LAUNCH;
  if (rc) {
    mat_free(A);
    return rc;
  }
  if (h_ranks) {
    const int T = A->T;
    for (int I = 0; I < T; ++I)
      for (int J = 0; J < T; ++J) {
        const int hi = std::max(I, J), lo = std::min(I, J);
        h_ranks[(int64_t)I * T + J] = (I == J) ? -1 : A->tlr->S.rank[tidx(hi, lo, T)];
      }
  }
  *out = A;
  return 0;
}

}  // extern "C"
