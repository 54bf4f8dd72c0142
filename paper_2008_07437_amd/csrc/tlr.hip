// Tile-low-rank covariance and Cholesky factorisation (Section 5.3).
//
// Compression: every off-diagonal tile of Sigma is generated densely and
// compressed by a randomized range finder (Gaussian sketch, Householder QR
// of the sketch, projection) followed by a column-pivoted QR of the
// projection stopped when the Frobenius norm of the rest is <= acc; a tile
// whose rank would exceed max_rank stays dense.  The
// sketch width starts from the rank of the previous tile at the same
// distance from the diagonal and doubles until the kept rank is at least
// OVERSAMPLE below it.
//
// Factorisation (left-looking over tile columns j): the column's tiles of the
// compressed Sigma are expanded into a dense panel, the updates of all
// earlier columns are applied as one GEMM,
//   A_ij -= sum_{k<j} U_ik (V_ik^T V_jk) U_jk^T  =  [U_ik G_ijk]_k [U_jk]_k^T,
// the diagonal tile is factored in FP64 (with its inverse W_j), and the
// sub-diagonal tiles are recompressed at acc with the triangular solve
// applied to V only (L_ij = U (W_j V)^T).  Each factor tile is compressed
// once, after all its updates.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>

#include "tlr.h"

namespace mvg {

constexpr int OVERSAMPLE = 16;

// Pinned host blocks for staged task lists, per thread.  A thread drives one
// stream at a time (every entry point synchronises its stream before it
// returns), so once HostLists::release has synchronised that stream every
// copy out of the pool has completed and the pool is rewound, also while
// other HostLists of the thread keep their device copies.
namespace {
struct PinnedPool {
  std::vector<std::pair<char *, size_t>> blocks;
  size_t bi = 0, off = 0;
  ~PinnedPool() {
    for (auto &b : blocks) hipHostFree(b.first);
  }
  void *get(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    while (bi < blocks.size() && off + bytes > blocks[bi].second) {
      ++bi;
      off = 0;
    }
    if (bi == blocks.size()) {
      const size_t sz = std::max(bytes, (size_t)8 << 20);
      char *p = nullptr;
      if (hipHostMalloc((void **)&p, sz, hipHostMallocDefault) != hipSuccess) {
        hipGetLastError();
        return nullptr;
      }
      blocks.emplace_back(p, sz);
      off = 0;
    }
    void *r = blocks[bi].first + off;
    off += bytes;
    return r;
  }
};
thread_local PinnedPool g_pinned;
}  // namespace

void *HostLists::stage(const void *p, size_t bytes, hipStream_t st, int *rc) {
  if (bytes == 0) bytes = 8;
  void *h = g_pinned.get(bytes);
  if (!h) {
    set_error("TLR: pinned staging buffer of %zu bytes failed", bytes);
    *rc = MVG_ERR_ALLOC;
    return nullptr;
  }
  memcpy(h, p, bytes);
  void *d = nullptr;
  if (malloc_async(&d, bytes, st) != hipSuccess) {
    hipGetLastError();
    set_error("TLR: staging allocation of %zu bytes failed", bytes);
    *rc = MVG_ERR_ALLOC;
    return nullptr;
  }
  dev.push_back(d);
  if (hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
    hipGetLastError();
    set_error("TLR: staging copy failed");
    *rc = MVG_ERR_LAUNCH;
    return nullptr;
  }
  return d;
}

void *HostLists::scratch(size_t bytes, hipStream_t st, int *rc) {
  void *d = nullptr;
  if (malloc_async(&d, bytes ? bytes : 8, st) != hipSuccess) {
    hipGetLastError();
    set_error("TLR: device scratch of %zu bytes failed", bytes);
    *rc = MVG_ERR_ALLOC;
    return nullptr;
  }
  dev.push_back(d);
  return d;
}

void HostLists::release(hipStream_t st) {
  for (void *d : dev) hipFreeAsync(d, st);
  dev.clear();
  hipStreamSynchronize(st);
  g_pinned.bi = 0;  // every staged copy of this thread has completed
  g_pinned.off = 0;
}

// Output block size of a product: 32 x 32 when M and N are at most 32 (the
// V^T V of low-rank tiles), 128 x 64 for tall products with a long K (the
// sketches and V <- W V of 1200-row tiles), 64 x 64 otherwise.
static int gemm_block_size(const GemmTask &g) {
  if (std::max(g.M, g.N) <= 32) return 32;
  if (g.M >= 256 && g.K >= 128) return 128;
  return 64;
}

// One launch per block size.
static int run_gemms(const std::vector<GemmTask> &v, HostLists &L, hipStream_t st) {
  struct Part {
    int bs;
    int n = 0;
    int64_t nb = 0;
    const GemmTask *dt = nullptr;
    const int64_t *ds = nullptr;
    int *dmap = nullptr;
  } parts[3] = {{32}, {64}, {128}};
  double fl = 0.0;
  int rc = 0;
  for (Part &p : parts) {
    std::vector<GemmTask> t;
    std::vector<int64_t> start;
    for (const GemmTask &g : v) {
      if (gemm_block_size(g) != p.bs) continue;
      const int64_t b = gemm_blocks(g, p.bs);
      if (b == 0) continue;
      t.push_back(g);
      start.push_back(p.nb);
      p.nb += b;
      fl += 2.0 * g.M * (double)g.N * g.K;
    }
    if (t.empty()) continue;
    p.n = (int)t.size();
    p.dt = (const GemmTask *)L.stage(t.data(), t.size() * sizeof(GemmTask), st, &rc);
    if (!rc) p.ds = (const int64_t *)L.stage(start.data(), start.size() * 8, st, &rc);
    if (!rc && p.n > GEMM_TASKS_LDS) {  // every block's task, instead of a search in global memory
      p.dmap = (int *)L.scratch(sizeof(int) * (size_t)p.nb, st, &rc);
      if (!rc) rc = launch_gemm_task_map(p.ds, p.n, p.nb, p.dmap, st);
    }
    if (rc) return rc;
  }
  const int h = prof_begin(MVG_PROF_TLRGEMM, st, fl, 0.0);  // after the task lists' copies
  for (const Part &p : parts)
    if (!rc && p.n) rc = launch_gemm_batched(p.dt, p.ds, p.n, p.nb, st, p.dmap, p.bs);
  prof_end(h, st);
  return rc;
}

template <class T, int (*F)(const T *, int, hipStream_t)>
static int run_list(const std::vector<T> &v, HostLists &L, hipStream_t st) {
  if (v.empty()) return 0;
  int rc = 0;
  const T *d = (const T *)L.stage(v.data(), v.size() * sizeof(T), st, &rc);
  if (rc) return rc;
  return F(d, (int)v.size(), st);
}

// Unpivoted QRs of a batch go to the several-launch panel form when every
// matrix fits it and the widest has at least QR_PANELS_MIN_N columns (a
// single workgroup per matrix is then the critical path); narrower batches
// stay with the one-launch blocked kernel.  MVG_QR_PANELS=0 / 1 forces the
// choice (experiments).
constexpr int QR_PANELS_MIN_N = 64;

static int qr_panels_mode() {
  static const int mode = [] {
    const char *e = getenv("MVG_QR_PANELS");
    return e ? atoi(e) : -1;
  }();
  return mode;
}

// The randomized-pivot panel form of the truncating pivoted QR (on B^T)
// replaces the blocked QR of B^T and the one-workgroup pivoted QR of R''
// for batches whose widest sketch has at least QR_PANELS_MIN_N columns.
// MVG_QRCP_PANELS=0 / 1 forces the choice (experiments).
static bool use_qrcp_panels(int nb, int smax) {
  static const int mode = [] {
    const char *e = getenv("MVG_QRCP_PANELS");
    return e ? atoi(e) : -1;
  }();
  if (mode == 0 || !qrcp_panels_ok(nb, nb, smax)) return false;
  return mode == 1 || smax >= QR_PANELS_MIN_N;
}

// the panel kernels' 16-byte loads: even leading dimensions and 16-byte
// aligned matrices
static bool panel_tasks_aligned(const std::vector<QrTask> &v) {
  for (const QrTask &t : v)
    if ((t.lda & 1) || (t.Q && (t.ldq & 1)) || ((uintptr_t)t.A & 15) || ((uintptr_t)t.Q & 15) ||
        ((uintptr_t)t.work & 15))
      return false;
  return true;
}

static int run_qr(const std::vector<QrTask> &v, int mmax, bool blocked, HostLists &L,
                  hipStream_t st) {
  if (v.empty()) return 0;
  int rc = 0;
  const QrTask *d = (const QrTask *)L.stage(v.data(), v.size() * sizeof(QrTask), st, &rc);
  if (rc) return rc;
  double fl = 0.0;
  for (const QrTask &t : v) fl += 4.0 * t.m * (double)t.n * t.n - 4.0 / 3.0 * t.n * (double)t.n * t.n;
  const int h = prof_begin(MVG_PROF_QR, st, blocked ? fl : 0.0, 0.0);
  if (blocked) {
    int mmin = v[0].m, mx = 0, nmax = 0;
    bool with_q = false;
    for (const QrTask &t : v) {
      mmin = std::min(mmin, t.m);
      mx = std::max(mx, t.m);
      nmax = std::max(nmax, t.n);
      with_q = with_q || t.Q;
    }
    const int mode = qr_panels_mode();
    const bool panels = qr_panels_ok(mmin, mx, nmax) && panel_tasks_aligned(v) &&
                        (mode == 1 || (mode != 0 && nmax >= QR_PANELS_MIN_N));
    rc = panels ? launch_qr_panels(d, (int)v.size(), mx, nmax, with_q, st)
                : launch_qr_blocked(d, (int)v.size(), mmax, st);
  } else {
    rc = launch_qr(d, (int)v.size(), mmax, st);
  }
  prof_end(h, st);
  return rc;
}

static GemmTask gemm(const double *A, int lda, int ta, const double *B, int ldb, int tb, double *C,
                     int ldc, int M, int N, int K, double alpha, double beta) {
  return GemmTask{A, B, C, M, N, K, lda, ldb, ldc, ta, tb, alpha, beta};
}

// ------------------------------------------------------------- the store

static int store_reserve(TlrStore &S, size_t n, hipStream_t st, int64_t *off) {
  if (S.used + n > S.cap) {
    if (S.reader) hipStreamSynchronize(S.reader);  // its pending work reads the old buffer
    size_t cap = std::max({S.cap * 2, S.used + n, (size_t)1 << 22});
    double *nbuf = nullptr;
    if (malloc_async((void **)&nbuf, cap * sizeof(double), st) != hipSuccess) {
      hipGetLastError();
      set_error("TLR: low-rank store allocation of %.2f GB failed", cap * 8.0 / 1e9);
      return MVG_ERR_ALLOC;
    }
    if (S.used)
      hipMemcpyAsync(nbuf, S.buf, S.used * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (S.buf) hipFreeAsync(S.buf, st);
    S.buf = nbuf;
    S.cap = cap;
  }
  *off = (int64_t)S.used;
  S.used += n;
  return 0;
}

// Capacity of at least cap doubles (contents kept).
static int store_grow(TlrStore &S, size_t cap, hipStream_t st) {
  if (cap <= S.cap) return 0;
  if (S.reader) hipStreamSynchronize(S.reader);  // its pending work reads the old buffer
  double *nbuf = nullptr;
  if (malloc_async((void **)&nbuf, cap * sizeof(double), st) != hipSuccess) {
    hipGetLastError();
    set_error("TLR: low-rank store allocation of %.2f GB failed", cap * 8.0 / 1e9);
    return MVG_ERR_ALLOC;
  }
  if (S.used) hipMemcpyAsync(nbuf, S.buf, S.used * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (S.buf) hipFreeAsync(S.buf, st);
  S.buf = nbuf;
  S.cap = cap;
  return 0;
}

static int store_init(TlrStore &S, int T, int nb, int64_t N, hipStream_t st) {
  S.T = T;
  S.nb = nb;
  S.nbp = (nb + 63) / 64 * 64;
  S.N = N;
  const int64_t nt = (int64_t)T * (T + 1) / 2;
  S.rank.assign(nt, 0);
  S.dense.assign(nt, 0);
  S.uoff.assign(nt, 0);
  S.used = 0;
  const size_t dbytes = sizeof(double) * (size_t)T * S.nbp * S.nbp;
  if (malloc_async((void **)&S.diag, dbytes, st) != hipSuccess) {
    hipGetLastError();
    set_error("TLR: diagonal tile allocation of %.2f GB failed", dbytes / 1e9);
    return MVG_ERR_ALLOC;
  }
  // identity everywhere: the padding of each nbp x nbp diagonal tile stays so
  std::vector<CopyTask> v;
  HostLists L;
  for (int j = 0; j < T; ++j)
    v.push_back(CopyTask{S.diag, S.diag + (int64_t)j * S.nbp * S.nbp, S.nbp, S.nbp, S.nbp, S.nbp,
                         nullptr, COPY_IDENTITY});
  int rc = run_list<CopyTask, launch_copy_cols>(v, L, st);
  L.release(st);
  return rc;
}

void store_free(TlrStore &S) {
  dev_free(S.diag);
  dev_free(S.buf);
  S.diag = nullptr;
  S.buf = nullptr;
  S.cap = S.used = 0;
}

// ------------------------------------------------------------ compression

struct CompressJob {
  const double *C;  // nb x nb tile, column-major
  int ldc;
  int64_t t;        // packed tile index in the destination store
  int s;            // sketch width
  uint64_t key;     // sketch stream
};

// Compresses the jobs' tiles into store D; V is replaced by W V when W
// (nb x nb, ldw, lower triangular) is given.  sguess[d] (d = I - J) is
// updated with the ranks found.
//
// Per tile C (nb x nb): Y = C Omega (Gaussian, nb x s); Y = Q R (blocked
// Householder); then a column-pivoted QR of B^T = C^T Q, stopped at the first
// k whose trailing block has ||R_22||_F <= acc, in one of two forms:
//  * large batches (the widest sketch >= QR_PANELS_MIN_N columns, tall
//    enough for the panel kernels): directly on B^T (nb x s) by the
//    randomized-pivot panel QR, B^T P = Q4 R4, so U = (Q P) R4_k^T and
//    V = Q4_k;
//  * otherwise B^T = Q'' R'' (blocked Householder), then R'' P = Q3 R3 by
//    the one-workgroup column-pivoted QR of the s x s factor, so
//    U = (Q P) R3_k^T and V = Q'' Q3_k.
// Either way ||C - U V^T||_2 <= ||C - Q B||_2 + acc (the Frobenius-norm
// tail rule; it keeps at least the ranks of the 2-norm rule s_i > acc).  A
// rank above s - OVERSAMPLE (the sketch may have missed part of the range)
// is retried with a wider sketch.
// W (nullable): the diagonal factor's inverse applied to every V; w_ready
// (nullable): an event after which W is complete, waited for only before W's
// first use, so that the sketches and QRs overlap W's computation.
// between (nullable): host work run once, after the first pass's kernels are
// queued and before the host waits for their ranks (it may record w_ready),
// so that the device runs the compression while the host prepares other
// streams' work.
static int compress_jobs(std::vector<CompressJob> jobs, TlrStore &D, double acc, int max_rank,
                         uint64_t seed, const double *W, int ldw, std::vector<int> &sguess,
                         hipStream_t st, hipEvent_t w_ready = nullptr,
                         const std::function<int()> &between = nullptr) {
  bool between_done = !between;
  const int nb = D.nb;
  const int T = D.T;
  const int smax = std::min(nb, QR_MAXN);
  while (!jobs.empty()) {
    // scratch per job: Om | Y | Z | Qp (nb x s each), R | Q3 (s x s),
    // T factors (QR_TAU_WIDTH (s + QR_TAU_WIDTH)), piv (s), pivot-sample
    // work (nb x QRS_ROWS + QRS_ROWS x s + s, randomized form only); then
    // the ranks of all jobs (contiguous: one copy to the host)
    constexpr size_t TW = QR_TAU_WIDTH;
    int smx = 1;
    for (size_t b = 0; b < jobs.size(); ++b) smx = std::max(smx, jobs[b].s);
    const bool rq = use_qrcp_panels(nb, smx);
    // every block starts at a multiple of 32 doubles and every matrix the
    // panel kernels read at an even offset (their 16-byte loads; nb is even)
    auto even = [](size_t x) { return (x + 1) & ~(size_t)1; };
    std::vector<size_t> base(jobs.size());
    size_t tot = 0;
    for (size_t b = 0; b < jobs.size(); ++b) {
      const size_t s = jobs[b].s;
      base[b] = tot;
      tot += 4 * (size_t)nb * s + 2 * s * s + TW * (s + TW) + even(s + 1);
      if (rq) tot += (size_t)QRS_ROWS * (nb + s) + s;
      tot = (tot + 31) & ~(size_t)31;
    }
    const size_t rank_off = tot;
    tot += (jobs.size() + 1) / 2;
    double *ws = nullptr;
    if (malloc_async((void **)&ws, tot * sizeof(double), st) != hipSuccess) {
      hipGetLastError();
      set_error("TLR: compression workspace of %.2f GB failed", tot * 8.0 / 1e9);
      return MVG_ERR_ALLOC;
    }
    auto Om = [&](size_t b) { return ws + base[b]; };
    auto Yb = [&](size_t b) { return ws + base[b] + (size_t)nb * jobs[b].s; };
    auto Zb = [&](size_t b) { return ws + base[b] + 2 * (size_t)nb * jobs[b].s; };
    auto Qp = [&](size_t b) { return ws + base[b] + 3 * (size_t)nb * jobs[b].s; };
    auto Rb = [&](size_t b) { return ws + base[b] + 4 * (size_t)nb * jobs[b].s; };
    auto Q3 = [&](size_t b) { return Rb(b) + (size_t)jobs[b].s * jobs[b].s; };
    auto Tb = [&](size_t b) { return Q3(b) + (size_t)jobs[b].s * jobs[b].s; };
    // T factors of the blocked QR (one block per panel of columns)
    auto Pv = [&](size_t b) { return (int *)(Tb(b) + TW * ((size_t)jobs[b].s + TW)); };
    auto Wk = [&](size_t b) { return Tb(b) + TW * ((size_t)jobs[b].s + TW) + even(jobs[b].s + 1); };
    int *d_ranks = (int *)(ws + rank_off);
    auto Rk = [&](size_t b) { return d_ranks + b; };
    HostLists L;
    int rc = 0;
    {
      std::vector<SketchTask> sk;
      std::vector<GemmTask> g;
      for (size_t b = 0; b < jobs.size(); ++b) {
        sk.push_back(SketchTask{Om(b), nb, jobs[b].s, nb, seed, jobs[b].key});
        g.push_back(gemm(jobs[b].C, jobs[b].ldc, 0, Om(b), nb, 0, Yb(b), nb, nb, jobs[b].s, nb,
                         1.0, 0.0));
      }
      rc = run_list<SketchTask, launch_gaussian>(sk, L, st);
      if (!rc) rc = run_gemms(g, L, st);  // Y = C Omega
    }
    if (!rc) {
      std::vector<QrTask> q;
      for (size_t b = 0; b < jobs.size(); ++b)
        q.push_back(QrTask{Yb(b), nb, jobs[b].s, nb, Tb(b), Om(b), nb, nullptr, 0.0, nullptr});
      rc = run_qr(q, nb, true, L, st);  // Q -> Om
    }
    if (!rc) {
      std::vector<GemmTask> g;
      for (size_t b = 0; b < jobs.size(); ++b)
        g.push_back(gemm(jobs[b].C, jobs[b].ldc, 1, Om(b), nb, 0, Yb(b), nb, nb, jobs[b].s, nb,
                         1.0, 0.0));
      rc = run_gemms(g, L, st);  // B^T = C^T Q -> Y
    }
    if (!rc && rq) {
      // B^T P = Q4 R4 (R4 in Y, Q4 -> Z), pivots from Gaussian samples
      std::vector<SketchTask> sk;
      std::vector<QrTask> q;
      for (size_t b = 0; b < jobs.size(); ++b) {
        sk.push_back(SketchTask{Wk(b), nb, QRS_ROWS, nb, seed, jobs[b].key | (1ull << 62)});
        q.push_back(QrTask{Yb(b), nb, jobs[b].s, nb, Tb(b), Zb(b), nb, Pv(b), acc, Rk(b), Wk(b)});
      }
      rc = run_list<SketchTask, launch_gaussian>(sk, L, st);
      if (!rc) {
        const QrTask *d = (const QrTask *)L.stage(q.data(), q.size() * sizeof(QrTask), st, &rc);
        const int h = prof_begin(MVG_PROF_QR, st, 0.0, 0.0);
        if (!rc) rc = launch_qrcp_panels(d, (int)q.size(), nb, smx, st);
        prof_end(h, st);
      }
    }
    if (!rc && !rq) {
      std::vector<QrTask> q;
      for (size_t b = 0; b < jobs.size(); ++b)
        q.push_back(QrTask{Yb(b), nb, jobs[b].s, nb, Tb(b), Zb(b), nb, nullptr, 0.0, nullptr});
      rc = run_qr(q, nb, true, L, st);  // B^T = Q'' R'', Q'' -> Z
    }
    if (!rc && !rq) {
      std::vector<CopyTask> c;
      std::vector<QrTask> q;
      for (size_t b = 0; b < jobs.size(); ++b) {
        const int s = jobs[b].s;
        c.push_back(CopyTask{Yb(b), Rb(b), s, s, nb, s, nullptr, COPY_UPPER_TRI});
        q.push_back(QrTask{Rb(b), s, s, s, nullptr, Q3(b), s, Pv(b), acc, Rk(b)});
      }
      rc = run_list<CopyTask, launch_copy_cols>(c, L, st);
      if (!rc) rc = run_qr(q, smx, false, L, st);  // R'' P = Q3 R3, stopped at ||R3_22||_F <= acc
    }
    if (!rc && !between_done) {
      between_done = true;
      rc = between();
    }
    // ranks to the host
    std::vector<int> ranks(jobs.size(), 0);
    if (!rc) {
      hipMemcpyAsync(ranks.data(), d_ranks, sizeof(int) * jobs.size(), hipMemcpyDeviceToHost, st);
      if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("TLR: compression kernels failed: %s", hipGetErrorString(hipGetLastError()));
        rc = MVG_ERR_LAUNCH;
      }
    }
    enum { DONE = 0, RETRY = 1 };
    std::vector<int> status(jobs.size(), DONE);
    std::vector<CompressJob> retry;
    if (!rc) {
      for (size_t b = 0; b < jobs.size(); ++b) {
        const int s = jobs[b].s, r = ranks[b];
        const int64_t t = jobs[b].t;
        int64_t q = t;  // packed index -> distance I - J
        int J = 0;
        while (q >= T - J) {
          q -= T - J;
          ++J;
        }
        const int d = (int)q;
        if (r > max_rank) {
          D.dense[t] = 1;
          D.rank[t] = -1;
          sguess[d] = r;
        } else if (r > s - OVERSAMPLE && s < smax) {
          CompressJob j = jobs[b];
          j.s = std::min(smax, (std::max(2 * s, r + 2 * OVERSAMPLE) + 15) / 16 * 16);
          retry.push_back(j);
          status[b] = RETRY;
        } else {
          D.dense[t] = 0;
          D.rank[t] = r;
          sguess[d] = r;
        }
      }
      // storage (the store may move: reserve everything before taking pointers)
      for (size_t b = 0; b < jobs.size() && !rc; ++b) {
        if (status[b] != DONE) continue;
        const int64_t t = jobs[b].t;
        const int r = D.reff(t);
        D.uoff[t] = 0;
        if (r > 0) rc = store_reserve(D, 2 * (size_t)nb * r, st, &D.uoff[t]);
      }
    }
    // U = (Q P) R'_k^T, V = W Q'_k (or the dense tile: U = tile, V = W or I)
    if (!rc) {
      std::vector<CopyTask> c;
      std::vector<GemmTask> g, g2;
      for (size_t b = 0; b < jobs.size(); ++b) {
        if (status[b] != DONE) continue;
        const int64_t t = jobs[b].t;
        const int s = jobs[b].s;
        double *U = D.buf + D.uoff[t];
        if (D.dense[t]) {
          double *V = U + (int64_t)nb * nb;
          c.push_back(CopyTask{jobs[b].C, U, nb, nb, jobs[b].ldc, nb, nullptr, COPY_PLAIN});
          if (W)
            c.push_back(CopyTask{W, V, nb, nb, ldw, nb, nullptr, COPY_PLAIN});
          else
            c.push_back(CopyTask{V, V, nb, nb, nb, nb, nullptr, COPY_IDENTITY});
          continue;
        }
        const int r = D.rank[t];
        if (r == 0) continue;
        double *V = U + (int64_t)nb * r;
        c.push_back(CopyTask{Om(b), Qp(b), nb, s, nb, nb, Pv(b), COPY_PLAIN});  // Q P
        if (rq) {
          c.push_back(CopyTask{Yb(b), Rb(b), r, s, nb, s, nullptr, COPY_UPPER_TRI});  // R4_k
          g.push_back(gemm(Qp(b), nb, 0, Rb(b), s, 1, U, nb, nb, r, s, 1.0, 0.0));
          // V = W Q4_k, or Q4_k
          if (W)
            g2.push_back(gemm(W, ldw, 0, Zb(b), nb, 0, V, nb, nb, r, nb, 1.0, 0.0));
          else
            c.push_back(CopyTask{Zb(b), V, nb, r, nb, nb, nullptr, COPY_PLAIN});
          continue;
        }
        c.push_back(CopyTask{Rb(b), Rb(b), r, s, s, s, nullptr, COPY_UPPER_TRI});  // R3_k
        g.push_back(gemm(Qp(b), nb, 0, Rb(b), s, 1, U, nb, nb, r, s, 1.0, 0.0));
        // Q'_k = Q'' Q3_k, then V = W Q'_k
        g.push_back(gemm(Zb(b), nb, 0, Q3(b), s, 0, W ? Yb(b) : V, nb, nb, r, s, 1.0, 0.0));
        if (W) g2.push_back(gemm(W, ldw, 0, Yb(b), nb, 0, V, nb, nb, r, nb, 1.0, 0.0));
      }
      if (W && w_ready && hipStreamWaitEvent(st, w_ready, 0) != hipSuccess) {
        set_error("TLR: wait for the diagonal factor failed");
        rc = MVG_ERR_LAUNCH;
      }
      if (!rc) rc = run_list<CopyTask, launch_copy_cols>(c, L, st);
      if (!rc) rc = run_gemms(g, L, st);
      if (!rc) rc = run_gemms(g2, L, st);
    }
    hipFreeAsync(ws, st);
    L.release(st);
    if (rc) return rc;
    jobs.swap(retry);
  }
  return 0;
}

static int sketch_width(const std::vector<int> &sguess, int d, int nb) {
  const int g = sguess[d] >= 0 ? sguess[d] : 16;
  return std::min({nb, QR_MAXN, (g + OVERSAMPLE + 8 + 15) / 16 * 16});
}

// ---------------------------------------------------- Sigma -> TLR Sigma

int tlr_build(mvg_mat *A, const mvg_opts &o, hipStream_t st) {
  TlrState *S = A->tlr;
  const int T = A->T, nb = A->nb;
  TlrStore &D = S->S;
  if (int rc = store_init(D, T, nb, A->N, st)) return rc;
  // tiles are generated densely a range of whole tile columns at a time
  // (packed order: the tiles of a column are contiguous), up to BUILD_BYTES
  constexpr size_t BUILD_BYTES = (size_t)16 << 30;
  const size_t tile_bytes = sizeof(double) * (size_t)nb * nb;
  const int64_t max_tiles = std::max<int64_t>(T, (int64_t)(BUILD_BYTES / tile_bytes));
  const int64_t nt = (int64_t)T * (T + 1) / 2;
  double *G = nullptr;
  const int64_t gtiles = std::min<int64_t>(nt, max_tiles);
  if (malloc_async((void **)&G, tile_bytes * gtiles, st) != hipSuccess) {
    hipGetLastError();
    set_error("TLR: tile buffer of %.2f GB failed", tile_bytes * gtiles / 1e9);
    return MVG_ERR_ALLOC;
  }
  std::vector<int> sguess(T, -1);
  int rc = 0;
  for (int J0 = 0; J0 < T && !rc;) {
    int J1 = J0;
    int64_t cnt = 0;
    while (J1 < T && cnt + (T - J1) <= gtiles) cnt += T - J1++;
    const int64_t t0 = tidx(J0, J0, T);
    std::vector<int64_t> off(nt, 0);
    for (int64_t t = t0; t < t0 + cnt; ++t) off[t] = (t - t0) * (int64_t)tile_bytes;
    HostLists L;
    const int64_t *doff = (const int64_t *)L.stage(off.data(), off.size() * 8, st, &rc);
    if (rc) break;
    const TileMap M{(char *)G, doff, nullptr, T, nb, T};
    rc = launch_cov_tiles(A->margs, A->d_qtab, A->d_x, A->d_y, A->n_loc, M, (int)t0, (int)cnt, st);
    std::vector<CopyTask> c;
    std::vector<CompressJob> jobs;
    for (int J = J0; J < J1; ++J) {
      const int64_t td = tidx(J, J, T) - t0;
      c.push_back(CopyTask{G + td * nb * nb, D.diag + (int64_t)J * D.nbp * D.nbp, nb, nb, nb, D.nbp,
                           nullptr, COPY_PLAIN});
      for (int I = J + 1; I < T; ++I) {
        const int64_t t = tidx(I, J, T);
        jobs.push_back(CompressJob{G + (t - t0) * nb * nb, nb, t, sketch_width(sguess, I - J, nb),
                                   (uint64_t)t * 2 + 0});
      }
    }
    if (!rc) rc = run_list<CopyTask, launch_copy_cols>(c, L, st);
    if (!rc) rc = compress_jobs(jobs, D, o.tlr_acc, o.tlr_max_rank, o.seed, nullptr, 0, sguess, st);
    L.release(st);
    J0 = J1;
  }
  hipFreeAsync(G, st);
  return rc;
}

// ------------------------------------------------------ TLR Cholesky

int tlr_potrf(mvg_mat *A, const mvg_opts &o, int64_t *d_info, hipStream_t st) {
  TlrState *S = A->tlr;
  const int T = A->T, nb = A->nb;
  const TlrStore &Sg = S->S;
  TlrStore &Lf = S->L;
  const int nbp = Sg.nbp;
  store_free(Lf);
  if (int rc = store_init(Lf, T, nb, A->N, st)) return rc;
  if (!A->d_winv) {
    if (!(A->d_winv = (double *)dev_alloc(sizeof(double) * (size_t)T * nbp * nbp))) {
      set_error("TLR: inverse diagonal tiles allocation failed");
      return MVG_ERR_ALLOC;
    }
  }
  // tile map of the factor's diagonal tiles (nbp x nbp each) for the dense
  // diagonal kernels
  const int64_t nt = (int64_t)T * (T + 1) / 2;
  std::vector<int64_t> doff(nt, 0);
  for (int j = 0; j < T; ++j) doff[tidx(j, j, T)] = (int64_t)j * nbp * nbp * 8;
  HostLists L0;
  int rc = 0;
  const int64_t *d_doff = (const int64_t *)L0.stage(doff.data(), doff.size() * 8, st, &rc);
  if (rc) return rc;
  const TileMap Md{(char *)Lf.diag, d_doff, nullptr, T, nbp, T};
  // Two dense panels ((T - j) nb x nb, ld (T - j) nb): while column j is
  // compressed on st, column j + 1 is expanded into the other panel and
  // receives the updates of columns k < j on a second stream (look-ahead);
  // the update from column j itself follows on st once column j is factored.
  // Column j's diagonal factor runs on a third stream beside its compression.
  double *Pbuf[2] = {nullptr, nullptr};
  for (int q = 0; q < 2 && !rc; ++q)
    if (malloc_async((void **)&Pbuf[q], sizeof(double) * (size_t)T * nb * nb, st) != hipSuccess) {
      hipGetLastError();
      set_error("TLR: panel allocation failed");
      rc = MVG_ERR_ALLOC;
    }
  std::vector<int> sguess(T, -1);
  // the factor's store sized up front from the compressed Sigma's (the factor's
  // ranks are close to it), so that it does not grow by reallocation and copy
  if (!rc) rc = store_grow(Lf, Sg.used + Sg.used / 4 + ((size_t)1 << 22), st);
  double *upd[2] = {nullptr, nullptr};  // update workspaces (look-ahead, own column), grow-only
  size_t upd_cap[2] = {0, 0};
  hipStream_t dside = side_stream();
  hipStream_t look = nullptr;
  hipEvent_t ev_upd = nullptr, ev_diag = nullptr, ev_look = nullptr;
  if (!rc && (!dside || hipStreamCreateWithFlags(&look, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&ev_upd, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&ev_diag, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&ev_look, hipEventDisableTiming) != hipSuccess)) {
    hipGetLastError();
    set_error("TLR: side streams or events unavailable");
    rc = MVG_ERR_STATE;
  }
  Lf.reader = look;  // a growth of the factor's store first drains the look-ahead

  // column jc of the compressed Sigma into panel Pp, on stream s
  auto expand = [&](int jc, double *Pp, HostLists &Lx, hipStream_t s) -> int {
    const int ldp = (T - jc) * nb;
    std::vector<CopyTask> c{CopyTask{Sg.diag + (int64_t)jc * nbp * nbp, Pp, nb, nb, nbp, ldp,
                                     nullptr, COPY_PLAIN}};
    std::vector<GemmTask> g;
    for (int i = jc + 1; i < T; ++i) {
      const int64_t t = tidx(i, jc, T);
      g.push_back(gemm(Sg.U(t), nb, 0, Sg.V(t), nb, 1, Pp + (int64_t)(i - jc) * nb, ldp, nb, nb,
                       Sg.reff(t), 1.0, 0.0));
    }
    int e = run_list<CopyTask, launch_copy_cols>(c, Lx, s);
    if (!e) e = run_gemms(g, Lx, s);
    return e;
  };
  // panel Pp of column jc -= the updates of factor columns k in [k0, k1):
  // [U_ik G_ijk]_k [U_jk]_k^T with G_ijk = V_ik^T V_jk, one large GEMM
  // workgroups of the look-ahead's column-update GEMM (0: one per block).
  // 7/4 of the CU count (448 of 256 CUs: two per CU on three quarters of
  // them, one on the rest) leaves room on a quarter of the CUs for the
  // compression kernels of the main stream, which otherwise wait for the
  // GEMM's blocks to drain: one evaluation at n = 100,000 3.52 -> 3.42 s
  // (384: 3.45 s, 512: 3.61 s, 256: 3.54 s, 128: 4.09 s)
  static const int look_wg = [] {
    const char *e = getenv("MVG_TLR_LOOK_WG");
    if (e) return std::max(0, atoi(e));
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      return 0;
    return 7 * cus / 4;
  }();
  auto update = [&](int jc, int k0, int k1, double *Pp, int w, HostLists &Lx, hipStream_t s) -> int {
    const int ldp = (T - jc) * nb;
    int64_t Kj = 0;
    std::vector<int64_t> koff(T, 0);
    for (int k = k0; k < k1; ++k) {
      koff[k] = Kj;
      Kj += Lf.reff(tidx(jc, k, T));
    }
    if (Kj == 0) return 0;
    size_t gsz = 0;
    for (int i = jc; i < T; ++i)
      for (int k = k0; k < k1; ++k) gsz += (size_t)Lf.reff(tidx(i, k, T)) * Lf.reff(tidx(jc, k, T));
    // K padded with zero columns to a multiple of 32 (the direct-to-LDS
    // GEMM streams whole slices)
    const int64_t Kp = (Kj + 31) / 32 * 32;
    const size_t qn = (size_t)nb * Kp, pn = (size_t)ldp * Kp;
    const size_t need = qn + pn + std::max<size_t>(gsz, 1);
    if (need > upd_cap[w]) {  // grow-only (x1.5): a new allocation of GBs costs ~0.1 s
      if (upd[w]) hipFreeAsync(upd[w], s);
      upd_cap[w] = std::max(need, upd_cap[w] + upd_cap[w] / 2);
      if (malloc_async((void **)&upd[w], sizeof(double) * upd_cap[w], s) != hipSuccess) {
        hipGetLastError();
        upd[w] = nullptr;
        upd_cap[w] = 0;
        set_error("TLR: update workspace of %.2f GB failed", need * 8.0 / 1e9);
        return MVG_ERR_ALLOC;
      }
    }
    double *Qc = upd[w], *Pc = Qc + qn, *Gs = Pc + pn;
    std::vector<CopyTask> c;
    std::vector<GemmTask> gG, gP;
    for (int k = k0; k < k1; ++k) {
      const int64_t tj = tidx(jc, k, T);
      const int rj = Lf.reff(tj);
      if (rj) c.push_back(CopyTask{Lf.U(tj), Qc + koff[k] * nb, nb, rj, nb, nb, nullptr, COPY_PLAIN});
    }
    size_t go = 0;
    for (int i = jc; i < T; ++i)
      for (int k = k0; k < k1; ++k) {
        const int64_t ti = tidx(i, k, T), tj = tidx(jc, k, T);
        const int ri = Lf.reff(ti), rj = Lf.reff(tj);
        if (!rj) continue;
        double *Gik = Gs + go;
        if (ri) gG.push_back(gemm(Lf.V(ti), nb, 1, Lf.V(tj), nb, 0, Gik, ri, ri, rj, nb, 1.0, 0.0));
        // K = 0 (rank-0 tile) writes zeros into its block of Pc
        gP.push_back(gemm(Lf.U(ti), nb, 0, Gik, std::max(ri, 1), 0,
                          Pc + (int64_t)(i - jc) * nb + koff[k] * ldp, ldp, nb, rj, ri, 1.0, 0.0));
        go += (size_t)ri * rj;
      }
    int e = run_list<CopyTask, launch_copy_cols>(c, Lx, s);
    if (!e && Kp > Kj) e = launch_fill_f64(Qc + (size_t)nb * Kj, 0.0, (int64_t)nb * (Kp - Kj), s);
    if (!e && Kp > Kj) e = launch_fill_f64(Pc + (size_t)ldp * Kj, 0.0, (int64_t)ldp * (Kp - Kj), s);
    if (!e) e = run_gemms(gG, Lx, s);
    if (!e) e = run_gemms(gP, Lx, s);
    if (!e) {
      const double fl = 2.0 * ldp * nb * (double)Kj;
      const int h = prof_begin(MVG_PROF_TRAILING, s, fl, 0.0);
      e = launch_gemm_nt_sub(Pc, ldp, Qc, nb, Pp, ldp, ldp, nb, (int)Kp, s, s == look ? look_wg : 0);
      prof_end(h, s);
    }
    return e;
  };

  {  // column 0's panel
    HostLists L;
    if (!rc) rc = expand(0, Pbuf[0], L, st);
    L.release(st);
  }
  bool looked = false;  // a look-ahead for the current column was issued
  for (int j = 0; j < T && !rc; ++j) {
    const int ldp = (T - j) * nb;
    double *P = Pbuf[j & 1];
    HostLists L, L2;
    // (1) the panel of column j: its look-ahead (expansion and the updates
    // of columns k < j - 1) is complete; the update of column j - 1 here
    if (looked && hipStreamWaitEvent(st, ev_look, 0) != hipSuccess) {
      set_error("TLR: look-ahead ordering failed");
      rc = MVG_ERR_LAUNCH;
    }
    if (!rc && j > 0) rc = update(j, looked ? j - 1 : 0, j, P, 1, L, st);
    if (!rc && hipEventRecord(ev_upd, st) != hipSuccess) {
      set_error("TLR: side-stream ordering failed");
      rc = MVG_ERR_LAUNCH;
    }
    // (2) and (3), queued from the host while the device already runs the
    // compression of (4) (its first kernels are queued before this runs)
    auto side_work = [&]() -> int {
      int e = 0;
      // (2) diagonal tile: FP64 Cholesky and W_j, on the side stream beside
      // the compression of the sub-diagonal tiles (which reads other rows of
      // P and needs W_j only for V <- W_j V)
      if (hipStreamWaitEvent(dside, ev_upd, 0) != hipSuccess) {
        set_error("TLR: side-stream ordering failed");
        return MVG_ERR_LAUNCH;
      }
      std::vector<CopyTask> c{CopyTask{P, Lf.diag + (int64_t)j * nbp * nbp, nb, nb, ldp, nbp,
                                       nullptr, COPY_PLAIN}};
      e = run_list<CopyTask, launch_copy_cols>(c, L, dside);
      PivotTol pt = pivot_tol(A);
      pt.gbase = (int64_t)j * nb;
      pt.lreal = nb;
      if (!e) e = diag_factor(Md, j, A->d_winv, d_info, pt, dside);
      if (!e && hipEventRecord(ev_diag, dside) != hipSuccess) {
        set_error("TLR: side-stream event failed");
        e = MVG_ERR_LAUNCH;
      }
      // (3) look-ahead on its own stream: column j + 1's panel (the other
      // buffer, last read by column j - 1's compression, complete on st
      // before ev_upd) expanded and updated by the factor columns k < j
      if (!e && j + 1 < T) {
        if (hipStreamWaitEvent(look, ev_upd, 0) != hipSuccess) {
          set_error("TLR: look-ahead ordering failed");
          return MVG_ERR_LAUNCH;
        }
        double *Pn = Pbuf[(j + 1) & 1];
        e = expand(j + 1, Pn, L2, look);
        if (!e && j > 0) e = update(j + 1, 0, j, Pn, 0, L2, look);
        if (!e && hipEventRecord(ev_look, look) != hipSuccess) {
          set_error("TLR: look-ahead event failed");
          e = MVG_ERR_LAUNCH;
        }
        looked = !e;
      }
      return e;
    };
    looked = false;
    // (4) recompress the sub-diagonal tiles, V <- W_j V
    if (!rc && j + 1 < T) {
      std::vector<CompressJob> jobs;
      for (int i = j + 1; i < T; ++i) {
        const int64_t t = tidx(i, j, T);
        const int g = Sg.dense[t] ? nb : Sg.rank[t];
        std::vector<int> sg1(1, std::max(g, sguess[i - j]));
        jobs.push_back(CompressJob{P + (int64_t)(i - j) * nb, ldp, t, sketch_width(sg1, 0, nb),
                                   (uint64_t)t * 2 + 1});
      }
      rc = compress_jobs(jobs, Lf, o.tlr_acc, o.tlr_max_rank, o.seed ^ 0x5bd1e995u,
                         A->d_winv + (int64_t)j * nbp * nbp, nbp, sguess, st, ev_diag, side_work);
    } else if (!rc) {
      rc = side_work();
    }
    // the staged lists are released only when every stream that reads them
    // is done (also on an error): the side stream's diagonal factor, then the
    // look-ahead (synchronised here; the next column needs it anyway)
    if (ev_diag) hipStreamWaitEvent(st, ev_diag, 0);
    if (look) L2.release(look);
    L.release(st);
  }
  Lf.reader = nullptr;
  if (look) {
    hipStreamSynchronize(look);
    hipStreamDestroy(look);
  }
  if (ev_upd) hipEventDestroy(ev_upd);  // complete: st waited for every event it ordered
  if (ev_diag) hipEventDestroy(ev_diag);
  if (ev_look) hipEventDestroy(ev_look);
  for (int w = 0; w < 2; ++w)
    if (upd[w]) hipFreeAsync(upd[w], st);
  for (int q = 0; q < 2; ++q)
    if (Pbuf[q]) hipFreeAsync(Pbuf[q], st);
  L0.release(st);
  if (!rc) rc = tlr_upload_meta(A, st);
  return rc;
}

// Device copies of the factor's per-tile offsets and ranks (for the solves).
int tlr_upload_meta(mvg_mat *A, hipStream_t st) {
  TlrState *S = A->tlr;
  const TlrStore &Lf = S->L;
  const int64_t nt = (int64_t)A->T * (A->T + 1) / 2;
  std::vector<int64_t> u(nt);
  std::vector<int> r(nt);
  for (int64_t t = 0; t < nt; ++t) {
    u[t] = Lf.uoff[t];
    r[t] = Lf.reff(t);
  }
  dev_free(S->d_uoff);  // idle: the caller's stream has completed the earlier solves
  dev_free(S->d_reff);
  S->d_uoff = (int64_t *)dev_alloc(nt * 8);
  S->d_reff = (int *)dev_alloc(nt * 4);
  if (!S->d_uoff || !S->d_reff) {
    set_error("TLR: metadata allocation failed");
    return MVG_ERR_ALLOC;
  }
  hipMemcpyAsync(S->d_uoff, u.data(), nt * 8, hipMemcpyHostToDevice, st);
  hipMemcpyAsync(S->d_reff, r.data(), nt * 4, hipMemcpyHostToDevice, st);
  if (hipStreamSynchronize(st) != hipSuccess) return MVG_ERR_LAUNCH;
  return 0;
}

// ------------------------------------------------------------------ solves
//
// Vectors have length Np = T nb; nrhs columns with leading dimension ldv
// (blockIdx.z selects the column).

constexpr int TLR_MAXNB = 2048;

// The triangular solves as many small workgroups per step (one workgroup
// per tile and step kept the offset-1 tile's rank-240 products on one CU,
// its loads one at a time).  Forward, per column k:
//   y_k = W_k v_k           (k_tlr_fwd_diag: 64 rows per workgroup),
//   g_ik = V_ik^T y_k       (k_tlr_solve_g<true>: 16 columns per workgroup),
//   v_i -= U_ik g_ik, i > k (k_tlr_solve_apply<true>: 64 rows per workgroup;
//                            the first tile's workgroups also store y_k as v_k).
// Backward, per row k from the last: y_k = W_k^T v_k (k_tlr_bwd_diag: 16
// columns per workgroup), g_kj = U_kj^T y_k and v_j -= V_kj g_kj for j < k.
// y and g live in a scratch of nb (y) + (T - 1) nb (g, nb per tile) doubles per
// right-hand side.  Every sum is in a fixed order.
constexpr int TLR_FWD_RB = 64;  // rows per workgroup
constexpr int TLR_FWD_GC = 16;  // columns per workgroup

// y_k = W_k v_k (lower triangular W_k, ld nbp, entries above the diagonal not
// read as values): lane = row, the four waves take every fourth column
// c <= row with eight columns' loads in flight; the waves' partial sums are
// added in a fixed order.
__global__ __launch_bounds__(256) void k_tlr_fwd_diag(int nb, int nbp, int k,
                                                      const double *__restrict__ winv,
                                                      const double *__restrict__ V, int64_t ldv,
                                                      double *__restrict__ scr, int64_t lds) {
  __shared__ double v[TLR_MAXNB];
  __shared__ double part[4][TLR_FWD_RB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double *vk = V + (int64_t)blockIdx.z * ldv + (int64_t)k * nb;
  const double *W = winv + (int64_t)k * nbp * nbp;
  const int r0 = blockIdx.x * TLR_FWD_RB, row = r0 + lane;
  const int cend = min(nb, r0 + TLR_FWD_RB);  // columns c <= the last row
  for (int i = threadIdx.x; i < cend; i += 256) v[i] = vk[i];
  __syncthreads();
  const int rr = min(row, nb - 1);  // clamped row for the loads
  double acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = 0.0;
  int c = wave;
  for (; c + 28 < cend; c += 32) {
    double w[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) w[j] = W[(int64_t)(c + 4 * j) * nbp + rr];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (c + 4 * j <= row) acc[j] += w[j] * v[c + 4 * j];
  }
  for (; c < cend; c += 4)
    if (c <= row) acc[0] += W[(int64_t)c * nbp + rr] * v[c];
  part[wave][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (wave == 0 && row < nb)
    scr[(int64_t)blockIdx.z * lds + row] =
        (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// Forward: g_ik = V_ik^T y_k for tile i = k + 1 + blockIdx.x; backward:
// g_kj = U_kj^T y_k for tile j = blockIdx.x < k.  Columns TLR_FWD_GC
// blockIdx.y .. + TLR_FWD_GC (four per wave, sixteen loads in flight per
// wave), each a lane-strided sum reduced across the wave.
template <bool FWD>
__global__ __launch_bounds__(256) void k_tlr_solve_g(int T, int nb, int k,
                                                     const double *__restrict__ buf,
                                                     const int64_t *__restrict__ uoff,
                                                     const int *__restrict__ reff,
                                                     double *__restrict__ scr, int64_t lds) {
  __shared__ double x[TLR_MAXNB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int other = FWD ? k + 1 + blockIdx.x : blockIdx.x;
  const int64_t t = FWD ? tidx(other, k, T) : tidx(k, other, T);
  const int r = reff[t];
  const int c0 = blockIdx.y * TLR_FWD_GC + wave * 4;
  if (blockIdx.y * TLR_FWD_GC >= r) return;  // uniform over the workgroup
  double *sc = scr + (int64_t)blockIdx.z * lds;
  for (int e = threadIdx.x; e < nb; e += 256) x[e] = sc[e];
  __syncthreads();
  if (c0 >= r) return;  // uniform over the wave; no barrier follows
  const double *right = buf + uoff[t] + (FWD ? (int64_t)nb * r : 0);  // V_ik, or U_kj
  const double *col[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) col[j] = right + (int64_t)min(c0 + j, r - 1) * nb;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int e0 = 0; e0 < nb; e0 += 256) {
    double a[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = min(e0 + 64 * m + lane, nb - 1);
#pragma unroll
      for (int j = 0; j < 4; ++j) a[m][j] = col[j][e];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = e0 + 64 * m + lane;
      if (e < nb)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] += a[m][j] * x[e];
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double s = acc[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0 && c0 + j < r) sc[nb + (int64_t)blockIdx.x * nb + c0 + j] = s;
  }
}

// Forward: v_i -= U_ik g_ik for tile i = k + 1 + blockIdx.x; backward:
// v_j -= V_kj g_kj for tile j = blockIdx.x < k.  Rows TLR_FWD_RB
// blockIdx.y .. + TLR_FWD_RB (lane = row, the waves take every fourth
// column with eight loads in flight, partial sums added in a fixed order);
// the workgroups of the first tile also store y_k as v_k.
template <bool FWD>
__global__ __launch_bounds__(256) void k_tlr_solve_apply(int T, int nb, int k,
                                                         const double *__restrict__ buf,
                                                         const int64_t *__restrict__ uoff,
                                                         const int *__restrict__ reff,
                                                         double *__restrict__ V, int64_t ldv,
                                                         const double *__restrict__ scr,
                                                         int64_t lds) {
  __shared__ double g[TLR_MAXNB];
  __shared__ double part[4][TLR_FWD_RB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int other = FWD ? k + 1 + blockIdx.x : blockIdx.x;
  const int64_t t = FWD ? tidx(other, k, T) : tidx(k, other, T);
  const int r = reff[t];
  const int row = blockIdx.y * TLR_FWD_RB + lane;
  const double *sc = scr + (int64_t)blockIdx.z * lds;
  double *vc = V + (int64_t)blockIdx.z * ldv;
  if (blockIdx.x == 0 && wave == 0 && row < nb) vc[(int64_t)k * nb + row] = sc[row];
  if (r == 0) return;  // uniform over the workgroup
  for (int e = threadIdx.x; e < r; e += 256) g[e] = sc[nb + (int64_t)blockIdx.x * nb + e];
  __syncthreads();
  const double *U = buf + uoff[t] + (FWD ? 0 : (int64_t)nb * r);  // U_ik, or V_kj
  const int rr = min(row, nb - 1);
  double acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = 0.0;
  int c = wave;
  for (; c + 28 < r; c += 32) {
    double u[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) u[j] = U[(int64_t)(c + 4 * j) * nb + rr];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] += u[j] * g[c + 4 * j];
  }
  for (; c < r; c += 4) acc[0] += U[(int64_t)c * nb + rr] * g[c];
  part[wave][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (wave == 0 && row < nb)
    vc[(int64_t)other * nb + row] -= (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// y_k = W_k^T v_k: output column c is the dot of column c of W_k (rows
// r >= c) with v_k; columns TLR_FWD_GC blockIdx.x .. + TLR_FWD_GC, four per
// wave, sixteen loads in flight per wave, each reduced across the wave.
__global__ __launch_bounds__(256) void k_tlr_bwd_diag(int nb, int nbp, int k,
                                                      const double *__restrict__ winv,
                                                      const double *__restrict__ V, int64_t ldv,
                                                      double *__restrict__ scr, int64_t lds) {
  __shared__ double v[TLR_MAXNB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double *vk = V + (int64_t)blockIdx.z * ldv + (int64_t)k * nb;
  const double *W = winv + (int64_t)k * nbp * nbp;
  for (int e = threadIdx.x; e < nb; e += 256) v[e] = vk[e];
  __syncthreads();
  const int c0 = blockIdx.x * TLR_FWD_GC + wave * 4;
  if (c0 >= nb) return;  // uniform over the wave; no barrier follows
  const double *col[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) col[j] = W + (int64_t)min(c0 + j, nb - 1) * nbp;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int e0 = c0 - c0 % 64; e0 < nb; e0 += 256) {  // rows from the block of c0
    double a[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = min(e0 + 64 * m + lane, nb - 1);
#pragma unroll
      for (int j = 0; j < 4; ++j) a[m][j] = col[j][e];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int e = e0 + 64 * m + lane;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (e < nb && e >= c0 + j) acc[j] += a[m][j] * v[e];
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double s = acc[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0 && c0 + j < nb) scr[(int64_t)blockIdx.z * lds + c0 + j] = s;
  }
}

// v_k = y_k (the last column, which has no tiles below)
__global__ void k_tlr_fwd_store(int nb, int k, double *__restrict__ V, int64_t ldv,
                                const double *__restrict__ scr, int64_t lds) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nb) V[(int64_t)blockIdx.z * ldv + (int64_t)k * nb + e] = scr[(int64_t)blockIdx.z * lds + e];
}

static int tlr_solve_ok(const mvg_mat *A) {
  if (!A->tlr || !A->tlr->d_uoff || A->nb > TLR_MAXNB) {
    set_error("TLR solve needs a factored TLR matrix with nb <= %d", TLR_MAXNB);
    return MVG_ERR_STATE;
  }
  return 0;
}

int tlr_trsm_forward(const mvg_mat *A, double *d_V, int nrhs, int64_t ldv, hipStream_t st) {
  if (int rc = tlr_solve_ok(A)) return rc;
  constexpr int RHS_CHUNK = 256;  // right-hand sides per pass (bounds the scratch)
  if (nrhs > RHS_CHUNK) {
    for (int c = 0; c < nrhs; c += RHS_CHUNK)
      if (int rc = tlr_trsm_forward(A, d_V + (int64_t)c * ldv, std::min(RHS_CHUNK, nrhs - c), ldv,
                                    st))
        return rc;
    return 0;
  }
  const TlrState *S = A->tlr;
  const int T = A->T, nb = A->nb, nbp = S->L.nbp;
  // scratch per right-hand side: y_k (nb) and g_ik of every tile below (nb each)
  const int64_t lds = (int64_t)T * nb;
  double *scr = nullptr;
  if (malloc_async((void **)&scr, sizeof(double) * (size_t)lds * nrhs, st) != hipSuccess) {
    hipGetLastError();
    set_error("TLR solve: scratch of %.2f MB failed", lds * nrhs * 8.0 / 1e6);
    return MVG_ERR_ALLOC;
  }
  const unsigned rb = (unsigned)((nb + TLR_FWD_RB - 1) / TLR_FWD_RB);
  const unsigned gc = (unsigned)((nb + TLR_FWD_GC - 1) / TLR_FWD_GC);
  int rc = 0;
  for (int k = 0; k < T && !rc; ++k) {
    hipLaunchKernelGGL(k_tlr_fwd_diag, dim3(rb, 1, nrhs), dim3(256), 0, st, nb, nbp, k,
                       (const double *)A->d_winv, (const double *)d_V, ldv, scr, lds);
    rc = check_launch("tlr_fwd_diag");
    if (rc) break;
    if (k + 1 < T) {
      hipLaunchKernelGGL(k_tlr_solve_g<true>, dim3(T - k - 1, gc, nrhs), dim3(256), 0, st, T, nb, k,
                         (const double *)S->L.buf, (const int64_t *)S->d_uoff,
                         (const int *)S->d_reff, scr, lds);
      rc = check_launch("tlr_fwd_g");
      if (rc) break;
      hipLaunchKernelGGL(k_tlr_solve_apply<true>, dim3(T - k - 1, rb, nrhs), dim3(256), 0, st, T, nb,
                         k,
                         (const double *)S->L.buf, (const int64_t *)S->d_uoff,
                         (const int *)S->d_reff, d_V, ldv, (const double *)scr, lds);
      rc = check_launch("tlr_fwd_apply");
    } else {
      hipLaunchKernelGGL(k_tlr_fwd_store, dim3((nb + 255) / 256, 1, nrhs), dim3(256), 0, st, nb, k,
                         d_V, ldv, (const double *)scr, lds);
      rc = check_launch("tlr_fwd_store");
    }
  }
  hipFreeAsync(scr, st);
  return rc;
}

int tlr_trsv_backward(const mvg_mat *A, double *d_v, hipStream_t st) {
  if (int rc = tlr_solve_ok(A)) return rc;
  const TlrState *S = A->tlr;
  const int T = A->T, nb = A->nb, nbp = S->L.nbp;
  // scratch: y_k (nb) and g_kj of every tile left of the diagonal (nb each)
  const int64_t lds = (int64_t)T * nb;
  double *scr = nullptr;
  if (malloc_async((void **)&scr, sizeof(double) * (size_t)lds, st) != hipSuccess) {
    hipGetLastError();
    set_error("TLR solve: scratch of %.2f MB failed", lds * 8.0 / 1e6);
    return MVG_ERR_ALLOC;
  }
  const unsigned rb = (unsigned)((nb + TLR_FWD_RB - 1) / TLR_FWD_RB);
  const unsigned gc = (unsigned)((nb + TLR_FWD_GC - 1) / TLR_FWD_GC);
  int rc = 0;
  for (int k = T - 1; k >= 0 && !rc; --k) {
    hipLaunchKernelGGL(k_tlr_bwd_diag, dim3(gc), dim3(256), 0, st, nb, nbp, k,
                       (const double *)A->d_winv, (const double *)d_v, A->Np, scr, lds);
    rc = check_launch("tlr_bwd_diag");
    if (rc) break;
    if (k > 0) {
      hipLaunchKernelGGL(k_tlr_solve_g<false>, dim3(k, gc), dim3(256), 0, st, T, nb, k,
                         (const double *)S->L.buf, (const int64_t *)S->d_uoff,
                         (const int *)S->d_reff, scr, lds);
      rc = check_launch("tlr_bwd_g");
      if (rc) break;
      hipLaunchKernelGGL(k_tlr_solve_apply<false>, dim3(k, rb), dim3(256), 0, st, T, nb, k,
                         (const double *)S->L.buf, (const int64_t *)S->d_uoff,
                         (const int *)S->d_reff, d_v, A->Np, (const double *)scr, lds);
      rc = check_launch("tlr_bwd_apply");
    } else {
      hipLaunchKernelGGL(k_tlr_fwd_store, dim3((nb + 255) / 256), dim3(256), 0, st, nb, k, d_v,
                         A->Np, (const double *)scr, lds);
      rc = check_launch("tlr_bwd_store");
    }
  }
  hipFreeAsync(scr, st);
  return rc;
}

// {2 sum log L_jj over the N real rows, y^T y}: fixed-order two-stage sums
constexpr int TLR_RED = 4096;
__global__ __launch_bounds__(256) void k_tlr_logdet_part(const double *__restrict__ diag, int nb,
                                                         int nbp, int64_t N,
                                                         const double *__restrict__ y,
                                                         double *__restrict__ part) {
  __shared__ double r0[256], r1[256];
  const int64_t base = (int64_t)blockIdx.x * TLR_RED;
  double a = 0.0, q = 0.0;
  for (int t = threadIdx.x; t < TLR_RED; t += 256) {
    const int64_t gi = base + t;
    if (gi >= N) break;
    const int64_t j = gi / nb, r = gi % nb;
    a += log(diag[j * nbp * nbp + r * nbp + r]);
    q += y[gi] * y[gi];
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = q;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0[0];
    part[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ void k_tlr_logdet_final(const double *__restrict__ part, int n, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0.0, q = 0.0;
    for (int i = 0; i < n; ++i) {
      a += part[2 * i];
      q += part[2 * i + 1];
    }
    out[0] = 2.0 * a;
    out[1] = q;
  }
}

int tlr_logdet_quad(const mvg_mat *A, const double *d_y, double *d_part, double *d_out2,
                    hipStream_t st) {
  const int nblk = (int)((A->N + TLR_RED - 1) / TLR_RED);
  hipLaunchKernelGGL(k_tlr_logdet_part, dim3(nblk), dim3(256), 0, st, (const double *)A->tlr->L.diag,
                     A->nb, A->tlr->L.nbp, A->N, d_y, d_part);
  if (int rc = check_launch("tlr_logdet_part")) return rc;
  hipLaunchKernelGGL(k_tlr_logdet_final, dim3(1), dim3(64), 0, st, (const double *)d_part, nblk,
                     d_out2);
  return check_launch("tlr_logdet_final");
}

// Lower triangle of the compressed Sigma (or of the factor once factored) as
// a dense N x N column-major matrix (inspection of small cases).
int tlr_to_dense(const mvg_mat *A, double *out, int64_t ld, hipStream_t st) {
  const TlrStore &D = A->factored ? A->tlr->L : A->tlr->S;
  const int T = A->T, nb = A->nb;
  const int64_t N = A->N;
  HostLists L;
  std::vector<CopyTask> c;
  std::vector<GemmTask> g;
  for (int J = 0; J < T; ++J) {
    const int cols = (int)std::min<int64_t>(nb, N - (int64_t)J * nb);
    for (int I = 0; I < J; ++I)  // upper tiles: zero
      c.push_back(CopyTask{out, out + (int64_t)J * nb * ld + (int64_t)I * nb, nb, cols, (int)ld,
                           (int)ld, nullptr, COPY_ZERO});
    for (int I = J; I < T; ++I) {
      const int rows = (int)std::min<int64_t>(nb, N - (int64_t)I * nb);
      double *o = out + (int64_t)J * nb * ld + (int64_t)I * nb;
      if (I == J) {
        c.push_back(CopyTask{D.diag + (int64_t)J * D.nbp * D.nbp, o, rows, cols, D.nbp, (int)ld,
                             nullptr, COPY_LOWER_TRI});
        continue;
      }
      const int64_t t = tidx(I, J, T);
      g.push_back(gemm(D.U(t), nb, 0, D.V(t), nb, 1, o, (int)ld, rows, cols, D.reff(t), 1.0, 0.0));
    }
  }
  int rc = run_list<CopyTask, launch_copy_cols>(c, L, st);
  if (!rc) rc = run_gemms(g, L, st);
  L.release(st);
  return rc;
}

void tlr_state_free(TlrState *S) {
  if (!S) return;
  store_free(S->S);
  store_free(S->L);
  dev_free(S->d_uoff);
  dev_free(S->d_reff);
  delete S;
}

}  // namespace mvg
