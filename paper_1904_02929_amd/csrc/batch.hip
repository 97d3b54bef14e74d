// batch.hip -- many independent simulations stepped together on one GPU (C ABI in
// include/susp.h).  Each job keeps its own device block (carved from the batch's arena) and
// stream; a batch step queues every job's steps (graph replays) before waiting for any, so
// that jobs too small to fill the GPU run side by side.  Admission is by device footprint
// against the batch's budget.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <iterator>
#include <map>
#include <memory>
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

// One launch of a multi-job step: kernel, total work-groups, block size, and where its
// argument table and work-group offsets sit in the batch's device tables.
struct MultiLaunch {
  const void *fn;
  unsigned total, blk;
  size_t tab, pre;
  int nj;
};

// Lockstep runs use this many streams: the jobs are dealt to them by size, so that one
// part's latency-bound particle kernels run beside another part's lattice kernel.
constexpr int LS_STREAMS = 4;

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
  // lockstep runs (susp_batch_launch_all): per part (stream), the launches of two steps of
  // every group of its jobs with the same kernel sequence, built from each job's recorded
  // launches
  hipStream_t gstream[LS_STREAMS] = {};
  hipEvent_t gjoin[LS_STREAMS] = {};         // end of a part's run (parts 1.. join part 0)
  hipEvent_t gev = nullptr;                  // after the last lockstep run (all parts)
  std::vector<std::unique_ptr<Collect>> col;  // per slot
  std::vector<MultiLaunch> seq[LS_STREAMS];  // per part, the groups' sequences in turn
  std::vector<int> part;                     // per slot: its part in the last build
  hipEvent_t gfork = nullptr;                // fork of the parts inside the recorded pair
  hipGraphExec_t gexec = nullptr;            // the pair of steps of all parts, recorded
  std::vector<std::array<int64_t, 3>> key;   // slot, parity, handle the sequence was built for
  std::vector<char> host;                    // staging of the tables
  char *mt = nullptr;                        // device tables
  size_t mt_cap = 0;
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
  b->col.resize(max_jobs);
  for (int i = 0; i < max_jobs; ++i) {
    if (hipStreamCreateWithFlags(&b->stream[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming) != hipSuccess) {
      susp_batch_destroy(b);
      return set_error(SUSP_EDEVICE, "stream or event creation failed");
    }
  }
  b->part.assign(max_jobs, 0);
  for (int g = 0; g < LS_STREAMS; ++g) {
    if (hipStreamCreateWithFlags(&b->gstream[g], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->gjoin[g], hipEventDisableTiming) != hipSuccess) {
      susp_batch_destroy(b);
      return set_error(SUSP_EDEVICE, "stream or event creation failed");
    }
  }
  if (hipEventCreateWithFlags(&b->gev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->gfork, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(b->gev, b->gstream[0]) != hipSuccess) {
    susp_batch_destroy(b);
    return set_error(SUSP_EDEVICE, "stream or event creation failed");
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
  b->key.clear();  // the lockstep sequence is rebuilt for the new set of jobs
  b->bytes[k] = need;
  b->offset[k] = off;
  b->used += need;
  *slot = k;
  return SUSP_OK;
}

extern "C" int susp_batch_remove(susp_batch *b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_jobs || !b->job[slot]) return set_error(SUSP_EINVAL, "no such job");
  if (hipEventSynchronize(b->gev) != hipSuccess) return set_error(SUSP_EDEVICE, "event wait failed");
  susp_destroy(b->job[slot]);  // waits for the job's stream only; its block is the arena's
  b->job[slot] = nullptr;
  b->key.clear();
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
    if (hipStreamWaitEvent(b->stream[k], b->gev, 0) != hipSuccess) return set_error(SUSP_EDEVICE, "stream wait");
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
  if (hipStreamWaitEvent(b->stream[slot], b->gev, 0) != hipSuccess) return set_error(SUSP_EDEVICE, "stream wait");
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
  if (hipEventSynchronize(b->gev) != hipSuccess) return set_error(SUSP_EDEVICE, "event wait failed");
  return susp_stress(b->job[slot], out, gg);
}

extern "C" susp_sim *susp_batch_sim(susp_batch *b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_jobs) return nullptr;
  return b->job[slot];
}

extern "C" size_t susp_batch_bytes(const susp_batch *b) { return b ? b->used : 0; }

extern "C" int susp_batch_destroy(susp_batch *b) {
  if (!b) return SUSP_OK;
  for (hipStream_t st : b->gstream)
    if (st) (void)hipStreamSynchronize(st);
  for (int k = 0; k < b->max_jobs; ++k)
    if (b->job[k]) susp_destroy(b->job[k]);
  for (hipStream_t st : b->stream)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->done)
    if (ev) (void)hipEventDestroy(ev);
  for (hipStream_t st : b->gstream)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->gjoin)
    if (ev) (void)hipEventDestroy(ev);
  if (b->gfork) (void)hipEventDestroy(b->gfork);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->gev) (void)hipEventDestroy(b->gev);
  if (b->mt) (void)hipFree(b->mt);
  if (b->arena.base) (void)hipFree(b->arena.base);
  delete b;
  return SUSP_OK;
}

// ---------------------------------------------------------------------------------------
// Lockstep runs: every job of the batch takes the same number of steps, and each kernel of a
// step runs once for all jobs whose steps have the same kernel sequence (one multi-job launch
// per kernel, its work-groups dealt to the jobs by the offsets table), instead of once per job.
// The kernels are the ones a job runs alone, with its own arguments, so its results are the
// same bit for bit.

// Issue one pair of steps of every part: the parts' sequences on their streams, forked from
// and joined back to stream 0 (recorded into a graph, or issued directly).
static int issue_pair(susp_batch *b) {
  if (hipEventRecord(b->gfork, b->gstream[0]) != hipSuccess) return set_error(SUSP_EDEVICE, "event record");
  for (int g = 1; g < LS_STREAMS; ++g)
    if (!b->seq[g].empty() && hipStreamWaitEvent(b->gstream[g], b->gfork, 0) != hipSuccess)
      return set_error(SUSP_EDEVICE, "stream wait");
  for (int g = 0; g < LS_STREAMS; ++g) {
    for (const MultiLaunch &L : b->seq[g]) {
      const void *tab = b->mt + L.tab;
      const int32_t *pre = (const int32_t *)(b->mt + L.pre);
      int nj = L.nj;
      void *kp[] = {(void *)&tab, (void *)&pre, (void *)&nj};
      if (hipLaunchKernel(L.fn, dim3(L.total), dim3(L.blk), kp, 0, b->gstream[g]) != hipSuccess)
        return set_error(SUSP_EDEVICE, "lockstep launch failed");
    }
  }
  for (int g = 1; g < LS_STREAMS; ++g) {
    if (b->seq[g].empty()) continue;
    if (hipEventRecord(b->gjoin[g], b->gstream[g]) != hipSuccess ||
        hipStreamWaitEvent(b->gstream[0], b->gjoin[g], 0) != hipSuccess)
      return set_error(SUSP_EDEVICE, "event record");
  }
  return SUSP_OK;
}

// Record one pair of steps of all parts as a graph (replayed once per pair: one host call
// instead of a launch per kernel, part and job group).  Kernels and event nodes only.
static int record_pair(susp_batch *b) {
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  hipGraph_t gr = nullptr;
  if (hipStreamBeginCapture(b->gstream[0], hipStreamCaptureModeThreadLocal) != hipSuccess)
    return set_error(SUSP_EDEVICE, "graph capture");
  int rc = issue_pair(b);
  const hipError_t e = hipStreamEndCapture(b->gstream[0], &gr);
  if (rc || e != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc ? rc : set_error(SUSP_EDEVICE, "graph capture");
  }
  const hipError_t ei = hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (ei != hipSuccess) {
    b->gexec = nullptr;
    return set_error(SUSP_EDEVICE, "graph instantiate");
  }
  return SUSP_OK;
}

// (Re)build the multi-job launch sequences of two steps for the jobs now in the batch, if the
// jobs or their buffer parities differ from the last build.  The lockstep streams are idle.
// The jobs are dealt to the parts largest first, each to the part with the fewest nodes.
static int build_sequence(susp_batch *b, const std::vector<int> &slots, bool *built) {
  std::vector<std::array<int64_t, 3>> key;
  for (int k : slots) key.push_back({k, step_parity(b->job[k]), (int64_t)(intptr_t)b->job[k]});
  *built = false;
  if (key == b->key) return SUSP_OK;
  *built = true;
  b->key.clear();
  for (auto &q : b->seq) q.clear();
  std::vector<int> order(slots);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return sim_of(b->job[x]).nodes > sim_of(b->job[y]).nodes; });
  int64_t load[LS_STREAMS] = {};
  for (int k : order) {
    int g = 0;
    for (int u = 1; u < LS_STREAMS; ++u)
      if (load[u] < load[g]) g = u;
    b->part[k] = g;
    load[g] += sim_of(b->job[k]).nodes;
  }
  // each job's launches of two steps, grouped by part and kernel sequence
  std::map<std::pair<int, std::vector<std::pair<const void *, unsigned>>>, std::vector<int>> groups;
  for (int k : slots) {
    if (!b->col[k]) b->col[k].reset(new Collect);
    Collect *c = b->col[k].get();
    int rc = record_two_steps(b->job[k], c);
    if (rc) return rc;
    std::vector<std::pair<const void *, unsigned>> sig;
    for (int r = 0; r < c->nrec; ++r) sig.push_back({c->rec[r].fn, c->rec[r].blk});
    groups[{b->part[k], sig}].push_back(k);
  }
  std::vector<char> &h = b->host;
  h.clear();
  auto align = [&](size_t a) { h.resize((h.size() + a - 1) / a * a); };
  for (auto &g : groups) {
    const std::vector<int> &js = g.second;
    const auto &sig = g.first.second;
    const int nrec = (int)sig.size();
    for (int r = 0; r < nrec; ++r) {
      MultiLaunch L;
      L.fn = sig[r].first;
      L.blk = sig[r].second;
      L.nj = (int)js.size();
      // the kernel indexes its table as an array of the argument struct: entries sizeof apart
      const size_t sz = b->col[js[0]]->rec[r].sz;
      const size_t stride = sz;
      align(256);
      L.tab = h.size();
      h.resize(h.size() + stride * js.size());
      int64_t tot = 0;
      std::vector<int32_t> pre;
      for (size_t u = 0; u < js.size(); ++u) {
        const Collect::Rec &rr = b->col[js[u]]->rec[r];
        if (rr.sz != sz) return set_error(SUSP_ESTATE, "argument sizes of one kernel differ");
        memcpy(h.data() + L.tab + u * stride, b->col[js[u]]->bytes + rr.off, sz);
        pre.push_back((int32_t)tot);
        tot += rr.grid;
      }
      if (tot <= 0 || tot > 0x7fffffff) return set_error(SUSP_EINVAL, "work-groups of a lockstep launch out of range");
      pre.push_back((int32_t)tot);
      L.total = (unsigned)tot;
      align(16);
      L.pre = h.size();
      h.resize(h.size() + pre.size() * sizeof(int32_t));
      memcpy(h.data() + L.pre, pre.data(), pre.size() * sizeof(int32_t));
      b->seq[g.first.first].push_back(L);
    }
  }
  if (h.size() > b->mt_cap) {
    if (b->mt) (void)hipFree(b->mt);
    b->mt = nullptr;
    b->mt_cap = 0;
    const size_t cap = h.size() * 2 + 4096;
    if (hipMalloc((void **)&b->mt, cap) != hipSuccess) {
      b->mt = nullptr;
      for (auto &q : b->seq) q.clear();
      return set_error(SUSP_ENOMEM, "lockstep launch tables could not be allocated");
    }
    b->mt_cap = cap;
  }
  if (hipMemcpy(b->mt, h.data(), h.size(), hipMemcpyHostToDevice) != hipSuccess) {
    for (auto &q : b->seq) q.clear();
    return set_error(SUSP_EDEVICE, "upload of the lockstep launch tables failed");
  }
  if (b->gexec) {  // recorded for the jobs before; recorded again once these jobs stay
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  b->key = key;
  return SUSP_OK;
}

extern "C" int susp_batch_launch_all(susp_batch *b, int64_t nsteps) {
  if (!b) return set_error(SUSP_EINVAL, "NULL batch");
  if (nsteps < 0) return set_error(SUSP_EINVAL, "negative step count");
  // the previous lockstep run owns the clocks and tables until it has finished
  if (hipEventSynchronize(b->gev) != hipSuccess) return set_error(SUSP_EDEVICE, "event wait failed");
  std::vector<int> slots;
  for (int k = 0; k < b->max_jobs; ++k) {
    if (!b->job[k]) continue;
    if (multi_ok(b->job[k])) {
      slots.push_back(k);
      continue;
    }
    // a job whose kernels have no multi-job form steps on its own stream
    int rc = launch_steps(b->job[k], nsteps);
    if (rc) return rc;
    if (hipEventRecord(b->done[k], b->stream[k]) != hipSuccess) return set_error(SUSP_EDEVICE, "event record");
  }
  if (slots.empty()) return SUSP_OK;
  int64_t left = nsteps;
  while (left >= 2) {
    const int m = (int)(left < CLK_CAP ? left : CLK_CAP) & ~1;
    if (left < nsteps) {  // the clock tables are rewritten: the run before must have read them
      if (hipEventRecord(b->gev, b->gstream[0]) != hipSuccess) return set_error(SUSP_EDEVICE, "event record");
      for (int k : slots)
        if (hipStreamWaitEvent(b->stream[k], b->gev, 0) != hipSuccess) return set_error(SUSP_EDEVICE, "stream wait");
    }
    for (int k : slots) {
      int rc = prepare_run(b->job[k], m);  // waits for the job's own stream
      if (rc) return rc;
    }
    bool built = false;
    int rc = build_sequence(b, slots, &built);
    if (rc) return rc;
    // the first run after the jobs changed issues its kernels directly (recording and
    // instantiating the graph would keep the GPU waiting); a run of the same jobs again
    // records the pair once and replays it
    if (!built && !b->gexec) {
      rc = record_pair(b);
      if (rc) return rc;
    }
    for (int p = 0; p < m / 2; ++p) {
      if (b->gexec) {
        if (hipGraphLaunch(b->gexec, b->gstream[0]) != hipSuccess) return set_error(SUSP_EDEVICE, "lockstep launch failed");
      } else {
        rc = issue_pair(b);
        if (rc) return rc;
      }
    }
    for (int k : slots) advance_steps(b->job[k], m);
    left -= m;
  }
  // every pair ends with the parts joined on stream 0, whose event marks the end of the run
  for (int k : slots)
    if (hipEventRecord(b->done[k], b->gstream[0]) != hipSuccess) return set_error(SUSP_EDEVICE, "event record");
  if (hipEventRecord(b->gev, b->gstream[0]) != hipSuccess) return set_error(SUSP_EDEVICE, "event record");
  if (left) {  // an odd last step: on each job's own stream, after the lockstep run
    for (int k : slots) {
      if (hipStreamWaitEvent(b->stream[k], b->gev, 0) != hipSuccess) return set_error(SUSP_EDEVICE, "stream wait");
      int rc = launch_steps(b->job[k], left);
      if (rc) return rc;
      if (hipEventRecord(b->done[k], b->stream[k]) != hipSuccess) return set_error(SUSP_EDEVICE, "event record");
    }
  }
  return SUSP_OK;
}
