// Request server: likelihood and cokriging requests on registered datasets,
// admitted by HBM footprint and run concurrently, one HIP stream per worker.
//
// Scheduling.  Requests wait in arrival order.  A free worker takes the
// oldest request whose footprint fits in the unreserved part of the budget
// (a request that can never fit is failed at once; the oldest waiting
// request is never overtaken by more than MAX_BYPASS others, so a large
// request is not starved by a stream of small ones).  Small likelihood
// requests (2n <= SMALL_MAX, FP64) that are waiting when a worker frees up
// are taken together and evaluated in one persistent launch.  Workers run on
// their own streams, so admitted requests overlap on the device.
//
// Resident factors.  A likelihood request keeps its factor (and Sigma^-1 Z)
// in an LRU cache keyed by (dataset, theta); a cokriging request on a cached
// key predicts from it directly; one whose key is being factored by a running
// likelihood request waits for it; otherwise it factors first (a miss).  Cached
// factors count against the budget and are evicted oldest first when an
// admission needs the room.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "mvgeo_internal.h"

namespace {

using clk = std::chrono::steady_clock;

struct Dataset {
  const double *x, *y, *z;
  int64_t n;
};

struct Req {
  int64_t id;
  int kind;  // MVG_REQ_LOGLIK / MVG_REQ_COKRIGE
  int dataset;
  mvg_theta theta;
  const double *x0, *y0;
  int64_t m;
  double *zhat;
  double t_arrive;  // seconds on the server clock
  size_t bytes;     // admission footprint
  int bypassed = 0;
};

struct Key {
  int dataset;
  double th[6];
  bool operator<(const Key &o) const {
    if (dataset != o.dataset) return dataset < o.dataset;
    return std::memcmp(th, o.th, sizeof(th)) < 0;
  }
};

Key key_of(int d, const mvg_theta &t) {
  Key k;
  k.dataset = d;
  const double v[6] = {t.sigma11_sq, t.sigma22_sq, t.a, t.nu11, t.nu22, t.beta};
  std::memcpy(k.th, v, sizeof(v));
  return k;
}

constexpr int MAX_BYPASS = 8;

}  // namespace

struct mvg_server {
  mvg_opts opts{};
  size_t budget = 0, reserved = 0, cached = 0;
  int nworkers = 1;
  std::vector<Dataset> datasets;
  std::deque<Req> waiting;
  std::vector<mvg_result> done;
  // factor cache: LRU list of keys, map key -> (factor, bytes, list position)
  struct Entry {
    mvg_factor *F;
    size_t bytes;
    std::list<Key>::iterator pos;
    int users = 0;  // in use by a running cokriging request
  };
  std::list<Key> lru;
  std::map<Key, Entry> cache;
  std::map<Key, int> inflight;  // likelihoods running whose factor will be cached
  int64_t next_id = 0, misses = 0, hits = 0, batches = 0;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::thread> threads;
  clk::time_point t0 = clk::now();
  int running = 0;

  double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }

  // Frees LRU factors not in use until `need` more bytes fit; mu held.
  bool make_room(size_t need) {
    while (reserved + cached + need > budget) {
      auto it = lru.begin();
      while (it != lru.end() && cache[*it].users > 0) ++it;
      if (it == lru.end()) return false;
      Entry &e = cache[*it];
      mvg_factor_destroy(e.F);
      cached -= e.bytes;
      cache.erase(*it);
      lru.erase(it);
    }
    return true;
  }

  void worker();
};

static size_t footprint_of(const mvg_server *S, int64_t n) {
  return mvg_footprint(n, &S->opts);
}

void mvg_server::worker() {
  int dev = 0;
  hipGetDevice(&dev);
  hipStream_t st = nullptr;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);  // default priority
  for (;;) {
    std::vector<Req> batch;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        if (stop && waiting.empty()) {
          lk.unlock();
          hipStreamDestroy(st);
          return;
        }
        // oldest request that fits; a small-likelihood head gathers its peers
        size_t pick = waiting.size();
        for (size_t i = 0; i < waiting.size(); ++i) {
          Req &r = waiting[i];
          if (r.bytes > budget) {  // can never run
            mvg_result res{};
            res.id = r.id;
            res.status = MVG_ERR_LIMIT;
            res.t_arrive = r.t_arrive;
            res.t_start = res.t_end = now();
            done.push_back(res);
            waiting.erase(waiting.begin() + i);
            cv_done.notify_all();
            --i;
            continue;
          }
          if (i > 0 && waiting[0].bypassed >= MAX_BYPASS) break;
          // a cokriging request whose factor is being computed waits for it
          if (r.kind == MVG_REQ_COKRIGE && inflight.count(key_of(r.dataset, r.theta)) &&
              !cache.count(key_of(r.dataset, r.theta)))
            continue;
          if (reserved + r.bytes + cached <= budget || make_room(r.bytes)) {
            pick = i;
            break;
          }
        }
        if (pick < waiting.size()) {
          for (size_t i = 0; i < pick; ++i) ++waiting[i].bypassed;
          Req r = waiting[pick];
          waiting.erase(waiting.begin() + pick);
          reserved += r.bytes;
          batch.push_back(r);
          if (r.kind == MVG_REQ_LOGLIK) ++inflight[key_of(r.dataset, r.theta)];
          const bool small = r.kind == MVG_REQ_LOGLIK && opts.precision == MVG_FP64 &&
                             2 * datasets[r.dataset].n <= mvg::SMALL_MAX;
          if (small) {  // continuous batching of the small likelihoods waiting now
            for (size_t i = 0; i < waiting.size();) {
              Req &q = waiting[i];
              if (q.kind == MVG_REQ_LOGLIK && 2 * datasets[q.dataset].n <= mvg::SMALL_MAX &&
                  reserved + cached + q.bytes <= budget) {
                reserved += q.bytes;
                batch.push_back(q);
                ++inflight[key_of(q.dataset, q.theta)];
                waiting.erase(waiting.begin() + i);
              } else {
                ++i;
              }
            }
          }
          ++running;
          break;
        }
        cv_work.wait(lk);
      }
    }
    const double t_start = now();
    std::vector<mvg_result> out(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
      out[i].id = batch[i].id;
      out[i].t_arrive = batch[i].t_arrive;
      out[i].t_start = t_start;
      out[i].n_loc = datasets[batch[i].dataset].n;
      out[i].kind = batch[i].kind;
      out[i].precision = opts.precision;
      out[i].batch = (int)batch.size();
    }
    if (batch.size() > 1 || (batch[0].kind == MVG_REQ_LOGLIK && opts.precision == MVG_FP64 &&
                             2 * datasets[batch[0].dataset].n <= mvg::SMALL_MAX)) {
      std::vector<mvg_task> tasks;
      for (auto &r : batch) {
        const Dataset &d = datasets[r.dataset];
        tasks.push_back(mvg_task{d.x, d.y, d.z, d.n, r.theta});
      }
      std::vector<double> ll(tasks.size()), ld(tasks.size()), q(tasks.size());
      std::vector<int64_t> stt(tasks.size());
      const int rc = loglik_many(tasks.data(), (int)tasks.size(), ll.data(), ld.data(), q.data(),
                                 stt.data(), st);
      for (size_t i = 0; i < batch.size(); ++i) {
        out[i].status = rc ? rc : (int)stt[i];
        out[i].loglik = ll[i];
        out[i].logdet = ld[i];
        out[i].quad = q[i];
      }
      std::lock_guard<std::mutex> lk(mu);
      ++batches;
    } else {
      Req &r = batch[0];
      const Dataset &d = datasets[r.dataset];
      const Key k = key_of(r.dataset, r.theta);
      mvg_factor *F = nullptr;
      bool hit = false;
      if (r.kind == MVG_REQ_COKRIGE) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(k);
        if (it != cache.end()) {
          F = it->second.F;
          ++it->second.users;
          lru.splice(lru.end(), lru, it->second.pos);
          hit = true;
          ++hits;
        } else {
          ++misses;
        }
      }
      int rc = 0;
      if (!hit) {
        double l = 0, ld = 0, q = 0;
        int64_t info = 0;
        rc = loglik(d.x, d.y, d.z, d.n, &r.theta, 1, &opts, &l, &ld, &q, &info, &F, st);
        out[0].loglik = l;
        out[0].logdet = ld;
        out[0].quad = q;
        if (!rc && info) rc = (int)info;
      }
      if (!rc && r.kind == MVG_REQ_COKRIGE && F)
        rc = cokrige_predict(F, r.x0, r.y0, r.m, r.zhat, nullptr, st);
      out[0].status = rc;
      out[0].cache_hit = hit ? 1 : 0;
      std::lock_guard<std::mutex> lk(mu);
      if (hit) {
        --cache[k].users;
      } else if (F) {
        // keep the factor resident if it fits (it replaces its own reservation)
        const size_t fb = r.bytes;
        auto it = cache.find(k);
        if (it == cache.end() && (reserved - r.bytes + cached + fb <= budget)) {
          lru.push_back(k);
          cache[k] = Entry{F, fb, std::prev(lru.end()), 0};
          cached += fb;
        } else {
          mvg_factor_destroy(F);
        }
      }
    }
    const double t_end = now();
    std::lock_guard<std::mutex> lk(mu);
    for (size_t i = 0; i < batch.size(); ++i) {
      reserved -= batch[i].bytes;
      if (batch[i].kind == MVG_REQ_LOGLIK) {
        auto it = inflight.find(key_of(batch[i].dataset, batch[i].theta));
        if (it != inflight.end() && --it->second == 0) inflight.erase(it);
      }
      out[i].t_end = t_end;
      done.push_back(out[i]);
    }
    --running;
    cv_work.notify_all();
    cv_done.notify_all();
  }
}

extern "C" {

mvg_server *mvg_server_create(size_t hbm_budget, int n_workers, const mvg_opts *o) {
  if (hbm_budget == 0 || n_workers < 1 || n_workers > 32) return nullptr;
  mvg_server *S = new mvg_server();
  if (o) S->opts = *o;
  S->budget = hbm_budget;
  S->nworkers = n_workers;
  int dev = 0;
  hipGetDevice(&dev);
  for (int i = 0; i < n_workers; ++i)
    S->threads.emplace_back([S, dev] {
      hipSetDevice(dev);
      S->worker();
    });
  return S;
}

int mvg_server_add_dataset(mvg_server *S, const double *d_x, const double *d_y, const double *d_z,
                           int64_t n_loc) {
  if (!S) return -1;
  if (!d_x || !d_y || !d_z) return -2;
  if (n_loc < 1) return -3;
  std::lock_guard<std::mutex> lk(S->mu);
  S->datasets.push_back(Dataset{d_x, d_y, d_z, n_loc});
  return (int)S->datasets.size() - 1;
}

int64_t mvg_server_submit(mvg_server *S, int kind, int dataset, const mvg_theta *th,
                          const double *d_x0, const double *d_y0, int64_t m, double *d_zhat,
                          double t_arrive) {
  if (!S || !th) return -1;
  if (kind != MVG_REQ_LOGLIK && kind != MVG_REQ_COKRIGE) return -2;
  std::lock_guard<std::mutex> lk(S->mu);
  if (dataset < 0 || dataset >= (int)S->datasets.size()) return -3;
  if (kind == MVG_REQ_COKRIGE && (!d_x0 || !d_y0 || !d_zhat || m < 1)) return -4;
  Req r;
  r.id = S->next_id++;
  r.kind = kind;
  r.dataset = dataset;
  r.theta = *th;
  r.x0 = d_x0;
  r.y0 = d_y0;
  r.m = m;
  r.zhat = d_zhat;
  r.t_arrive = t_arrive >= 0.0 ? t_arrive : S->now();
  r.bytes = footprint_of(S, S->datasets[dataset].n);
  S->waiting.push_back(r);
  S->cv_work.notify_one();
  return r.id;
}

int mvg_server_poll(mvg_server *S, mvg_result *out, int max, int wait_ms) {
  if (!S || (!out && max > 0)) return -1;
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->done.empty() && wait_ms > 0)
    S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [S] { return !S->done.empty(); });
  const int k = std::min<int>(max, (int)S->done.size());
  for (int i = 0; i < k; ++i) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + k);
  return k;
}

double mvg_server_clock(const mvg_server *S) { return S ? S->now() : 0.0; }

int mvg_server_stats(mvg_server *S, int64_t *hits, int64_t *misses, int64_t *batches,
                     size_t *cached_bytes) {
  if (!S) return -1;
  std::lock_guard<std::mutex> lk(S->mu);
  if (hits) *hits = S->hits;
  if (misses) *misses = S->misses;
  if (batches) *batches = S->batches;
  if (cached_bytes) *cached_bytes = S->cached;
  return 0;
}

void mvg_server_destroy(mvg_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto &t : S->threads) t.join();
  for (auto &kv : S->cache) mvg_factor_destroy(kv.second.F);
  delete S;
}

}  // extern "C"
