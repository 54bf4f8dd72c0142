// loglik_many_noalloc: the batched small-problem likelihood of loglik_many
// with its scratch memory in a fixed device array instead of an allocation,
// for callers that cannot allocate device memory.
//
// The scratch (task list, per-task outputs, the task-queue counter and one
// N x N workspace per workgroup of the persistent kernel) lives in `scratch`,
// a file-scope device array of MVG_NOALLOC_SCRATCH_BYTES.  Each device the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel (that is a host-side stand-in, not a
// device address): the first call on a device looks up the device address
// with hipGetSymbolAddress, with that device current, and keeps it per device.
// The kernels are those of loglik_many; fewer workgroups take the tasks from
// the same queue when the array holds fewer workspaces than loglik_many
// would allocate, so every task's result is the one loglik_many gives.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mvgeo.h"
#include "mvgeo_internal.h"

namespace mvg {

static __device__ __align__(256) char scratch[MVG_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;

// Host staging of the task list and the outputs (no host allocation either);
// one call at a time per process (the mutex), which also keeps two calls of
// this process from sharing a device's scratch at once.
static std::mutex g_mu;
static char *g_scratch_ptr[NOALLOC_MAX_DEVICES];
static SmallTask g_tasks[MVG_NOALLOC_MAX_TASKS];
static double g_out[4 * MVG_NOALLOC_MAX_TASKS];

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// device address of `scratch` on the current device (looked up once per device)
static int scratch_address(char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    hipGetLastError();
    set_error("loglik_many_noalloc: no usable current device");
    return MVG_ERR_STATE;
  }
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      hipGetLastError();
      set_error("loglik_many_noalloc: scratch address lookup failed: %s", hipGetErrorString(e));
      return MVG_ERR_STATE;
    }
    g_scratch_ptr[dev] = (char *)p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace mvg

using namespace mvg;

extern "C" {

int loglik_many_noalloc(const mvg_task *h_tasks, int n_tasks, double *h_loglik, double *h_logdet,
                        double *h_quad, int64_t *h_status, void *hip_stream) {
  if (!h_tasks) return -1;
  if (n_tasks < 1) return -2;
  if (!h_loglik) return -3;
  if (n_tasks > MVG_NOALLOC_MAX_TASKS) {
    set_error("loglik_many_noalloc: %d tasks above the limit of %d", n_tasks,
              MVG_NOALLOC_MAX_TASKS);
    return MVG_ERR_LIMIT;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  int64_t nmax = 1;
  for (int i = 0; i < n_tasks; ++i) {
    const mvg_task &t = h_tasks[i];
    MaternArgs tmp;
    if (!t.x || !t.y || !t.z || t.n_loc < 1 || 2 * t.n_loc > SMALL_MAX ||
        matern_setup(&t.theta, &tmp))
      return -(100 + i);
    g_tasks[i] = small_task(t.x, t.y, t.z, t.n_loc, t.theta);
    nmax = t.n_loc > nmax ? t.n_loc : nmax;
  }
  // layout: tasks | outputs (4 per task) | counter | workspaces (one per workgroup)
  const size_t tb = round256(sizeof(SmallTask) * (size_t)n_tasks);
  const size_t ob = round256(sizeof(double) * 4 * (size_t)n_tasks);
  const size_t fixed = tb + ob + 256;
  const size_t slot = sizeof(double) * small_workspace_doubles(nmax);
  if (fixed + slot > (size_t)MVG_NOALLOC_SCRATCH_BYTES) {
    set_error("loglik_many_noalloc: %d tasks of up to %lld locations need %.1f MB, above the "
              "%.1f MB scratch", n_tasks, (long long)nmax, (fixed + slot) / 1e6,
              MVG_NOALLOC_SCRATCH_BYTES / 1e6);
    return MVG_ERR_LIMIT;
  }
  const int slots = (int)(((size_t)MVG_NOALLOC_SCRATCH_BYTES - fixed) / slot);
  char *base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  SmallTask *d_tasks = (SmallTask *)base;
  double *d_out = (double *)(base + tb);
  int *d_counter = (int *)(base + tb + ob);
  double *d_ws = (double *)(base + fixed);
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipMemcpyAsync(d_tasks, g_tasks, sizeof(SmallTask) * (size_t)n_tasks, hipMemcpyHostToDevice,
                     st) != hipSuccess) {
    set_error("loglik_many_noalloc: task upload failed: %s", hipGetErrorString(hipGetLastError()));
    return MVG_ERR_LAUNCH;
  }
  // the counter is cleared by a kernel inside the launcher (no memset)
  int rc = launch_small_loglik(d_tasks, n_tasks, nmax, d_counter, d_ws, d_out, st, slots);
  if (!rc && hipMemcpyAsync(g_out, d_out, sizeof(double) * 4 * (size_t)n_tasks,
                            hipMemcpyDeviceToHost, st) != hipSuccess) {
    set_error("loglik_many_noalloc: result copy failed: %s", hipGetErrorString(hipGetLastError()));
    rc = MVG_ERR_LAUNCH;
  }
  if (hipStreamSynchronize(st) != hipSuccess && !rc) {
    set_error("loglik_many_noalloc failed: %s", hipGetErrorString(hipGetLastError()));
    rc = MVG_ERR_LAUNCH;
  }
  if (rc) return rc;
  for (int i = 0; i < n_tasks; ++i) {
    h_loglik[i] = g_out[4 * i];
    if (h_logdet) h_logdet[i] = g_out[4 * i + 1];
    if (h_quad) h_quad[i] = g_out[4 * i + 2];
    if (h_status) h_status[i] = (int64_t)g_out[4 * i + 3];
  }
  return 0;
}

}  // extern "C"
