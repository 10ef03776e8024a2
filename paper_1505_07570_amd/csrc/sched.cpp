// Admission of requests under a device-memory budget, for the serving loop.
//
// Pure host code (no device calls), so its policy is testable without a GPU.
// Policy: first come, first served.  A request is admitted when its bytes
// (its matrix, workspace and outputs) fit next to the bytes of the requests
// already running; admission stops at the first queued request that does not
// fit, so a large request is never overtaken indefinitely by smaller ones
// (no starvation).  A request larger than the whole budget can never run and
// is rejected at submission.
#include <cstdint>
#include <deque>
#include <new>
#include <unordered_map>

#include "rmm.h"

struct rmm_sched {
  size_t budget = 0;
  size_t in_use = 0;
  std::deque<std::pair<int64_t, size_t>> queue;
  std::unordered_map<int64_t, size_t> running;
};

extern "C" {

int rmm_sched_create(size_t budget_bytes, rmm_sched_t* out) {
  if (!out || budget_bytes == 0) return RMM_ERR_INVALID_ARG;
  rmm_sched* s = new (std::nothrow) rmm_sched();
  if (!s) return RMM_ERR_HIP;
  s->budget = budget_bytes;
  *out = s;
  return RMM_OK;
}

int rmm_sched_destroy(rmm_sched_t s) {
  delete s;
  return RMM_OK;
}

int rmm_sched_submit(rmm_sched_t s, int64_t id, size_t bytes) {
  if (!s || bytes > s->budget || s->running.count(id)) return RMM_ERR_INVALID_ARG;
  for (const auto& q : s->queue)
    if (q.first == id) return RMM_ERR_INVALID_ARG;
  s->queue.emplace_back(id, bytes);
  return RMM_OK;
}

int rmm_sched_admit(rmm_sched_t s, int64_t max_ids, int64_t* ids, int64_t* n) {
  if (!s || !n || max_ids < 0 || (max_ids > 0 && !ids)) return RMM_ERR_INVALID_ARG;
  int64_t k = 0;
  while (k < max_ids && !s->queue.empty()) {
    const auto q = s->queue.front();
    if (s->in_use + q.second > s->budget) break;
    s->queue.pop_front();
    s->in_use += q.second;
    s->running.emplace(q.first, q.second);
    ids[k++] = q.first;
  }
  *n = k;
  return RMM_OK;
}

int rmm_sched_complete(rmm_sched_t s, int64_t id) {
  if (!s) return RMM_ERR_INVALID_ARG;
  auto it = s->running.find(id);
  if (it == s->running.end()) return RMM_ERR_INVALID_ARG;
  s->in_use -= it->second;
  s->running.erase(it);
  return RMM_OK;
}

int rmm_sched_stats(rmm_sched_t s, size_t* in_use, int64_t* queued, int64_t* running) {
  if (!s) return RMM_ERR_INVALID_ARG;
  if (in_use) *in_use = s->in_use;
  if (queued) *queued = (int64_t)s->queue.size();
  if (running) *running = (int64_t)s->running.size();
  return RMM_OK;
}

}  // extern "C"
