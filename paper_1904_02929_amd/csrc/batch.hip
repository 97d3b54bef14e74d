// batch.hip -- many independent simulations stepped together on one GPU (C ABI in
// include/susp.h).  Each job keeps its own device block (carved from the batch's arena) and
// stream; a batch step queues every job's steps (graph replays) before waiting for any, so
// that jobs too small to fill the GPU run side by side.  Admission is by device footprint
// against the batch's budget.
#include <stdio.h>
#include <string.h>

#include <array>
#include <iterator>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "susp_impl.h"

using namespace susp;

// Device memory of the jobs: one arena of the budget's size, allocated once, carved first
// fit (256-byte granules) into job blocks.  Admitting and releasing a job then never calls
// hipMalloc or hipFree, which would wait for the whole device (every other job) to drain.
struct Arena {
  char *base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length of each free range (coalesced)

  size_t take(size_t n) {  // offset, or SIZE_MAX if no free range is large enough
    n = (n + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      return off;
    }
    return (size_t)-1;
  }
  void give(size_t off, size_t n) {
    n = (n + 255) / 256 * 256;
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
};

struct susp_batch {
  int max_jobs = 0;
  size_t budget = 0, used = 0;
  int autotune = 0;
  Arena arena;
  std::vector<hipStream_t> stream;
  std::vector<susp_sim *> job;
  std::vector<size_t> bytes, offset;
  std::vector<hipEvent_t> done;   // recorded after a job's queued steps
  std::map<std::array<int, 5>, std::pair<int, int>> shape;  // tuned brick per lattice kind
};

static std::array<int, 5> shape_key(const susp_params *p) {
  return {p->lx, p->ly, p->lz, p->precision, p->n > 0 ? 1 : 0};
}

// Mean lattice-kernel time of a scratch copy of the job with the given brick, over a few
// steps after a warm-up; a negative value if the shape is not valid for the job.
static double time_shape(const susp_params *p, int by, int bz, hipStream_t st) {
  susp_params q = *p;
  q.brick_y = by;
  q.brick_z = bz;
  susp_sim *tmp = nullptr;
  if (susp_create(&q, st, nullptr, 0, &tmp) != SUSP_OK) return -1.0;
  double ms = -1.0, t = 0.0;
  int64_t n = 0;
  if (susp_profile(tmp, 1) == SUSP_OK && susp_step(tmp, 2) == SUSP_OK &&
      susp_profile_read(tmp, &t, &n) == SUSP_OK && susp_step(tmp, 4) == SUSP_OK &&
      susp_profile_read(tmp, &t, &n) == SUSP_OK && n > 0)
    ms = t / (double)n;
  susp_destroy(tmp);
  return ms;
}

extern "C" int susp_batch_tune(susp_batch *b, const susp_params *p, int32_t *brick_y, int32_t *brick_z) {
  if (!b || !p || !brick_y || !brick_z) return set_error(SUSP_EINVAL, "NULL argument");
  if (susp_footprint_bytes(p) == 0) return SUSP_EINVAL;  // invalid parameters (error set)
  const auto key = shape_key(p);
  auto it = b->shape.find(key);
  if (it == b->shape.end()) {
    static const int cand[][2] = {{0, 0}, {4, 1}, {4, 4}, {8, 4}, {8, 8}, {16, 8}, {16, 16}};
    double best = -1.0;
    std::pair<int, int> pick(0, 0);
    for (const auto &c : cand) {
      if (c[0] > ((p->ly + 3) / 4) * 4 || c[1] > p->lz) continue;
      const double ms = time_shape(p, c[0], c[1], b->stream.empty() ? nullptr : b->stream[0]);
      if (ms > 0.0 && (best < 0.0 || ms < best)) {
        best = ms;
        pick = {c[0], c[1]};
      }
    }
    it = b->shape.emplace(key, pick).first;
  }
  *brick_y = it->second.first;
  *brick_z = it->second.second;
  return SUSP_OK;
}

extern "C" int susp_batch_create(int32_t max_jobs, size_t hbm_budget, int32_t autotune, susp_batch **out) {
  if (!out) return set_error(SUSP_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_jobs < 1 || max_jobs > 4096) return set_error(SUSP_EINVAL, "max_jobs must be in [1, 4096]");
  if (hbm_budget == 0) return set_error(SUSP_EINVAL, "hbm_budget must be positive");
  susp_batch *b = new susp_batch;
  b->max_jobs = max_jobs;
  b->budget = hbm_budget;
  b->autotune = autotune ? 1 : 0;
  b->job.assign(max_jobs, nullptr);
  b->bytes.assign(max_jobs, 0);
  b->offset.assign(max_jobs, 0);
  hipError_t e = hipMalloc((void **)&b->arena.base, hbm_budget);
  if (e != hipSuccess) {
    b->arena.base = nullptr;
    susp_batch_destroy(b);
    return set_error(SUSP_ENOMEM, "device arena of the batch budget could not be allocated");
  }
  b->arena.size = hbm_budget;
  b->arena.free_[0] = hbm_budget / 256 * 256;
  b->stream.assign(max_jobs, nullptr);
  b->done.assign(max_jobs, nullptr);
  for (int i = 0; i < max_jobs; ++i) {
    if (hipStreamCreateWithFlags(&b->stream[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming) != hipSuccess) {
      susp_batch_destroy(b);
      return set_error(SUSP_EDEVICE, "stream or event creation failed");
    }
  }
  *out = b;
  return SUSP_OK;
}

extern "C" int susp_batch_add(susp_batch *b, const susp_params *p, int32_t *slot) {
  if (!b || !p || !slot) return set_error(SUSP_EINVAL, "NULL argument");
  *slot = -1;
  susp_params q = *p;
  if (susp_footprint_bytes(&q) == 0) return SUSP_EINVAL;  // invalid parameters (error set)
  int k = 0;
  while (k < b->max_jobs && b->job[k]) ++k;
  if (k == b->max_jobs) return set_error(SUSP_ESTATE, "every slot of the batch is taken");
  if (b->autotune && q.brick_y == 0 && q.brick_z == 0) {
    int32_t by = 0, bz = 0;
    int rc = susp_batch_tune(b, &q, &by, &bz);
    if (rc) return rc;
    q.brick_y = by;
    q.brick_z = bz;
  }
  const size_t need = susp_footprint_bytes(&q);
  const size_t off = b->used + need <= b->budget ? b->arena.take(need) : (size_t)-1;
  if (off == (size_t)-1) {
    char msg[160];
    snprintf(msg, sizeof msg, "job needs %zu bytes, %zu of %zu in use", need, b->used, b->budget);
    return set_error(SUSP_ENOMEM, msg);
  }
  susp_sim *h = nullptr;
  int rc = susp_create(&q, b->stream[k], b->arena.base + off, need, &h);
  if (rc) {
    b->arena.give(off, need);
    return rc;
  }
  b->job[k] = h;
  b->bytes[k] = need;
  b->offset[k] = off;
  b->used += need;
  *slot = k;
  return SUSP_OK;
}

extern "C" int susp_batch_remove(susp_batch *b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_jobs || !b->job[slot]) return set_error(SUSP_EINVAL, "no such job");
  susp_destroy(b->job[slot]);  // waits for the job's stream only; its block is the arena's
  b->job[slot] = nullptr;
  b->arena.give(b->offset[slot], b->bytes[slot]);
  b->used -= b->bytes[slot];
  b->bytes[slot] = 0;
  return SUSP_OK;
}

extern "C" int susp_batch_step(susp_batch *b, int64_t nsteps) {
  if (!b) return set_error(SUSP_EINVAL, "NULL batch");
  if (nsteps < 0) return set_error(SUSP_EINVAL, "negative step count");
  // queue every job first, then wait: the streams run side by side
  for (int k = 0; k < b->max_jobs; ++k) {
    if (!b->job[k]) continue;
    int rc = launch_steps(b->job[k], nsteps);
    if (rc) return rc;
  }
  std::string bad;
  for (int k = 0; k < b->max_jobs; ++k) {
    if (!b->job[k]) continue;
    int rc = check_flags(b->job[k]);
    if (rc == SUSP_EUNSTABLE) bad += (bad.empty() ? "" : ", ") + std::to_string(k);
    else if (rc) return rc;
  }
  if (!bad.empty()) return set_error(SUSP_EUNSTABLE, ("instability in job slots " + bad).c_str());
  return SUSP_OK;
}

extern "C" int susp_batch_launch(susp_batch *b, int32_t slot, int64_t nsteps) {
  if (!b || slot < 0 || slot >= b->max_jobs || !b->job[slot]) return set_error(SUSP_EINVAL, "no such job");
  int rc = launch_steps(b->job[slot], nsteps);
  if (rc) return rc;
  if (hipEventRecord(b->done[slot], b->stream[slot]) != hipSuccess) return set_error(SUSP_EDEVICE, "event record");
  return SUSP_OK;
}

extern "C" int susp_batch_poll(susp_batch *b, int32_t slot, int32_t *done) {
  if (!b || !done || slot < 0 || slot >= b->max_jobs || !b->job[slot]) return set_error(SUSP_EINVAL, "no such job");
  const hipError_t e = hipEventQuery(b->done[slot]);
  if (e == hipErrorNotReady) {
    *done = 0;
    return SUSP_OK;
  }
  if (e != hipSuccess) return set_error(SUSP_EDEVICE, "event query failed");
  *done = 1;
  return check_flags(b->job[slot]);
}

extern "C" int susp_batch_stress(susp_batch *b, int32_t slot, double out[5][6], double gg[2]) {
  if (!b || slot < 0 || slot >= b->max_jobs || !b->job[slot]) return set_error(SUSP_EINVAL, "no such job");
  return susp_stress(b->job[slot], out, gg);
}

extern "C" susp_sim *susp_batch_sim(susp_batch *b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_jobs) return nullptr;
  return b->job[slot];
}

extern "C" size_t susp_batch_bytes(const susp_batch *b) { return b ? b->used : 0; }

extern "C" int susp_batch_destroy(susp_batch *b) {
  if (!b) return SUSP_OK;
  for (int k = 0; k < b->max_jobs; ++k)
    if (b->job[k]) susp_destroy(b->job[k]);
  for (hipStream_t st : b->stream)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->done)
    if (ev) (void)hipEventDestroy(ev);
  if (b->arena.base) (void)hipFree(b->arena.base);
  delete b;
  return SUSP_OK;
}
