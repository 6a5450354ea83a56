// Request loop with continuous batching (include/lbm_serve.h).
//
// Scheduling is separated from execution: the loop talks to an Executor that
// either drives a GPU context (lattices in a device pool reserved once, so
// admission never calls hipMalloc) or stands in for it on the host with a
// throughput model, which lets the admission, queueing and slot-reuse logic be
// tested on a machine without a GPU.
#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_serve.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

namespace {

int sfail(int code, const std::string &msg) {
  lbm::set_last_error(msg);
  return code;
}

constexpr size_t kPoolAlign = size_t(2) << 20;  // 2 MiB granules

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, size) in 2 MiB granules.
class Pool {
 public:
  explicit Pool(size_t size) { if (size >= kPoolAlign) free_[0] = size / kPoolAlign * kPoolAlign; }
  bool alloc(size_t n, size_t *off) {
    n = align_up(n, kPoolAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n, kPoolAlign);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Req {
  int32_t id = 0;
  lbm_case cs{};
  int64_t steps = 0, done = 0, cells = 0;
  double arrival = 0.0;  // as submitted
  double t_arr = -1.0, t_adm = -1.0, t_done = -1.0;
  int status = LBM_REQ_QUEUED;
  int slot = -1;
  size_t bytes = 0, off = 0;
  lbm_stats stats{};
};

class Executor {
 public:
  virtual ~Executor() = default;
  virtual size_t slots() const = 0;
  virtual int admit(Req &r, void *mem) = 0;
  virtual int advance(const std::vector<Req *> &rs, const std::vector<int64_t> &steps) = 0;
  virtual int finish(Req &r) = 0;  // fills r.stats; LBM_EUNSTABLE when not finite
  virtual int release(Req &r) = 0;
  virtual void *base() = 0;
};

class GpuExecutor : public Executor {
 public:
  GpuExecutor(lbm_ctx *c, int max_slots) : ctx_(c), slots_(max_slots) {}
  ~GpuExecutor() override {
    if (pool_) (void)hipFree(pool_);
  }
  int reserve(size_t bytes) {
    if (hipMalloc(&pool_, bytes) != hipSuccess) {
      (void)hipGetLastError();
      pool_ = nullptr;
      return sfail(LBM_ENOMEM, "cannot reserve the serving pool of " + std::to_string(bytes) + " bytes");
    }
    return LBM_OK;
  }
  size_t slots() const override { return slots_; }
  void *base() override { return pool_; }
  int admit(Req &r, void *mem) override {
    int slot = -1;
    int rc = lbm_set_case(ctx_, &r.cs, mem, r.bytes, &slot);
    if (rc != LBM_OK) return sfail(rc, lbm_last_error());
    r.slot = slot;
    return LBM_OK;
  }
  int advance(const std::vector<Req *> &rs, const std::vector<int64_t> &steps) override {
    std::vector<int32_t> ids(rs.size());
    for (size_t j = 0; j < rs.size(); ++j) ids[j] = rs[j]->slot;
    int rc = lbm_step_many(ctx_, (int)ids.size(), ids.data(), steps.data());
    if (rc == LBM_OK) rc = lbm_sync(ctx_);
    return rc == LBM_OK ? rc : sfail(rc, lbm_last_error());
  }
  int finish(Req &r) override {
    int rc = lbm_reduce(ctx_, r.slot, &r.stats);
    if (rc != LBM_OK && rc != LBM_EUNSTABLE) return sfail(rc, lbm_last_error());
    return rc;
  }
  int release(Req &r) override {
    int rc = lbm_release(ctx_, r.slot);
    r.slot = -1;
    return rc == LBM_OK ? rc : sfail(rc, lbm_last_error());
  }

 private:
  lbm_ctx *ctx_;
  size_t slots_;
  void *pool_ = nullptr;
};

// Host-only stand-in: advancing costs cells*steps / rate of wall time.
class FakeExecutor : public Executor {
 public:
  FakeExecutor(double mlups, size_t max_slots) : rate_(mlups * 1e6), slots_(max_slots) {}
  size_t slots() const override { return slots_; }
  void *base() override { return nullptr; }
  int admit(Req &r, void *) override {
    r.slot = next_slot_++;
    return LBM_OK;
  }
  int advance(const std::vector<Req *> &rs, const std::vector<int64_t> &steps) override {
    double lu = 0.0;
    for (size_t j = 0; j < rs.size(); ++j) lu += (double)rs[j]->cells * (double)steps[j];
    std::this_thread::sleep_for(std::chrono::duration<double>(lu / rate_));
    return LBM_OK;
  }
  int finish(Req &r) override {
    std::memset(&r.stats, 0, sizeof(r.stats));
    r.stats.step = r.done;
    r.stats.finite = 1;
    return LBM_OK;
  }
  int release(Req &r) override {
    r.slot = -1;
    return LBM_OK;
  }

 private:
  double rate_;
  size_t slots_;
  int next_slot_ = 0;
};

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)std::floor(pos), hi = (size_t)std::ceil(pos);
  return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

}  // namespace

struct lbm_server {
  std::unique_ptr<Executor> exec;
  Pool pool{0};
  size_t budget = 0;
  int chunk = 100;
  std::vector<Req> reqs;
  bool ran = false;
  lbm_serve_summary summary{};
  lbm_request_fn on_finish = nullptr;
  void *user = nullptr;
};

namespace {

void fill_request(const Req &r, lbm_request *out) {
  std::memset(out, 0, sizeof(*out));
  out->id = r.id;
  out->status = r.status;
  out->precision = r.cs.precision;
  out->steps = r.steps;
  out->cells = r.cells;
  out->t_arrival = r.t_arr;
  out->t_admit = r.t_adm;
  out->t_done = r.t_done;
  out->bytes = r.bytes;
  out->stats = r.stats;
}

void notify(const lbm_server *s, const Req &r) {
  if (!s->on_finish) return;
  lbm_request out;
  fill_request(r, &out);
  s->on_finish(&out, s->user);
}

}  // namespace

extern "C" {

int lbm_server_create(lbm_server **out, lbm_ctx *ctx, size_t hbm_budget, int chunk,
                      double fake_mlups) {
  if (!out) return sfail(LBM_EINVAL, "output is NULL");
  *out = nullptr;
  if (hbm_budget < kPoolAlign || chunk < 1) return sfail(LBM_EINVAL, "budget >= 2 MiB and chunk >= 1");
  auto *s = new lbm_server();
  s->budget = hbm_budget / kPoolAlign * kPoolAlign;
  s->chunk = chunk;
  s->pool = Pool(s->budget);
  if (ctx) {
    // residency is also bounded by the context's slot table: an admission
    // that finds no free slot waits for a departure
    auto *g = new GpuExecutor(ctx, 1 << 16);
    int rc = g->reserve(s->budget);
    if (rc != LBM_OK) {
      delete g;
      delete s;
      return rc;
    }
    s->exec.reset(g);
  } else {
    if (!(fake_mlups > 0.0)) {
      delete s;
      return sfail(LBM_EINVAL, "fake executor needs a positive rate");
    }
    s->exec.reset(new FakeExecutor(fake_mlups, 1 << 16));
  }
  *out = s;
  return LBM_OK;
}

void lbm_server_destroy(lbm_server *s) { delete s; }

int lbm_server_submit(lbm_server *s, const lbm_case *cs, int64_t steps, double arrival_s,
                      int32_t *id) {
  if (!s || !cs || !id) return sfail(LBM_EINVAL, "NULL argument");
  if (s->ran) return sfail(LBM_ESTATE, "the loop has already run");
  if (steps < 1 || !(arrival_s >= 0.0)) return sfail(LBM_EINVAL, "steps >= 1 and arrival >= 0");
  lbm_lattice lat;
  if (lbm_derive(cs, &lat) != LBM_OK) return sfail(LBM_EINVAL, lbm_last_error());
  Req r;
  r.id = (int32_t)s->reqs.size();
  r.cs = *cs;
  r.steps = steps;
  r.cells = (int64_t)cs->nx * cs->ny;
  r.arrival = arrival_s;
  r.bytes = lbm_footprint(cs);
  s->reqs.push_back(r);
  *id = r.id;
  return LBM_OK;
}

int lbm_server_run(lbm_server *s, double time_scale) {
  if (!s) return sfail(LBM_EINVAL, "server is NULL");
  if (s->ran) return sfail(LBM_ESTATE, "the loop has already run");
  if (!(time_scale > 0.0)) return sfail(LBM_EINVAL, "time_scale must be positive");
  s->ran = true;
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  auto now = [&] { return std::chrono::duration<double>(clock::now() - t0).count(); };
  std::vector<int> order(s->reqs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return s->reqs[a].arrival < s->reqs[b].arrival; });
  std::deque<int> pending;
  std::vector<int> resident;
  size_t next = 0, finished = 0, used = 0;
  lbm_serve_summary &sum = s->summary;
  std::memset(&sum, 0, sizeof(sum));
  double busy = 0.0;
  char *base = static_cast<char *>(s->exec->base());
  while (finished < s->reqs.size()) {
    double t = now();
    while (next < order.size() && s->reqs[order[next]].arrival / time_scale <= t) {
      Req &r = s->reqs[order[next]];
      r.t_arr = r.arrival / time_scale;
      pending.push_back(order[next]);
      ++next;
    }
    // admission: first fit in arrival order
    for (auto it = pending.begin(); it != pending.end();) {
      Req &r = s->reqs[*it];
      if (r.bytes > s->budget) {
        r.status = LBM_REQ_REJECTED;
        r.t_done = t;
        ++sum.rejected;
        ++finished;
        it = pending.erase(it);
        notify(s, r);
        continue;
      }
      size_t off = 0;
      if (resident.size() < s->exec->slots() && s->pool.alloc(r.bytes, &off)) {
        r.off = off;
        int rc = s->exec->admit(r, base ? base + off : nullptr);
        if (rc != LBM_OK) {
          s->pool.release(off, r.bytes);
          if (rc == LBM_ENOMEM && !resident.empty()) {  // no free slot: wait for a departure
            ++it;
            continue;
          }
          return rc;
        }
        r.status = LBM_REQ_RESIDENT;
        r.t_adm = t;
        used += align_up(r.bytes, kPoolAlign);
        sum.peak_bytes = std::max(sum.peak_bytes, used);
        resident.push_back(*it);
        sum.max_resident = std::max<int32_t>(sum.max_resident, (int32_t)resident.size());
        it = pending.erase(it);
      } else {
        ++it;
      }
    }
    if (resident.empty()) {
      if (next < order.size()) {
        const double wait = s->reqs[order[next]].arrival / time_scale - now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
        continue;
      }
      if (!pending.empty()) return sfail(LBM_ESTATE, "queued requests can never be admitted");
      break;
    }
    // one chunk: every resident cavity advances min(chunk, steps left)
    std::vector<Req *> rs;
    std::vector<int64_t> n;
    for (int id : resident) {
      Req &r = s->reqs[id];
      rs.push_back(&r);
      n.push_back(std::min<int64_t>(s->chunk, r.steps - r.done));
    }
    const double c0 = now();
    int rc = s->exec->advance(rs, n);
    if (rc != LBM_OK) return rc;
    ++sum.chunks;
    t = now();
    busy += t - c0;
    for (size_t j = 0; j < rs.size(); ++j) rs[j]->done += n[j];
    for (auto it = resident.begin(); it != resident.end();) {
      Req &r = s->reqs[*it];
      if (r.done < r.steps) {
        ++it;
        continue;
      }
      rc = s->exec->finish(r);
      if (rc != LBM_OK && rc != LBM_EUNSTABLE) return rc;
      r.status = rc == LBM_OK ? LBM_REQ_DONE : LBM_REQ_FAILED;
      r.t_done = now();
      rc = s->exec->release(r);
      if (rc != LBM_OK) return rc;
      s->pool.release(r.off, r.bytes);
      used -= align_up(r.bytes, kPoolAlign);
      if (r.status == LBM_REQ_DONE) ++sum.completed; else ++sum.failed;
      ++finished;
      it = resident.erase(it);
      notify(s, r);
    }
  }
  std::vector<double> lat;
  double first = 1e300, last = 0.0, lu = 0.0;
  for (const Req &r : s->reqs) {
    if (r.t_arr >= 0) first = std::min(first, r.t_arr);
    if (r.status != LBM_REQ_DONE) continue;
    lat.push_back(r.t_done - r.t_arr);
    last = std::max(last, r.t_done);
    lu += (double)r.cells * (double)r.steps;
  }
  sum.makespan_s = lat.empty() ? 0.0 : last - first;
  sum.p50_s = percentile(lat, 0.50);
  sum.p99_s = percentile(lat, 0.99);
  sum.max_s = lat.empty() ? 0.0 : *std::max_element(lat.begin(), lat.end());
  double m = 0.0;
  for (double v : lat) m += v;
  sum.mean_s = lat.empty() ? 0.0 : m / lat.size();
  sum.mlups = sum.makespan_s > 0 ? lu / sum.makespan_s / 1e6 : 0.0;
  sum.busy_frac = sum.makespan_s > 0 ? std::min(1.0, busy / sum.makespan_s) : 0.0;
  return LBM_OK;
}

int lbm_server_on_finish(lbm_server *s, lbm_request_fn fn, void *user) {
  if (!s) return sfail(LBM_EINVAL, "server is NULL");
  if (s->ran) return sfail(LBM_ESTATE, "the loop has already run");
  s->on_finish = fn;
  s->user = user;
  return LBM_OK;
}

int lbm_server_request(lbm_server *s, int32_t id, lbm_request *out) {
  if (!s || !out) return sfail(LBM_EINVAL, "NULL argument");
  if (id < 0 || id >= (int32_t)s->reqs.size()) return sfail(LBM_EINVAL, "unknown request");
  fill_request(s->reqs[id], out);
  return LBM_OK;
}

int lbm_server_summary(lbm_server *s, lbm_serve_summary *out) {
  if (!s || !out) return sfail(LBM_EINVAL, "NULL argument");
  *out = s->summary;
  return LBM_OK;
}

}  // extern "C"
