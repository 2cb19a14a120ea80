// Multi-graph scheduling on one GPU: the batched entry point and the serving loop.
//
// Every ldl_handle owns its HIP stream, so batch updates of different graphs issued from
// different host threads overlap on the device while each graph's own batches stay strictly
// ordered.  Results are per-handle deterministic, hence identical alone and in any mix.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "ldl.h"

namespace {

typedef std::chrono::steady_clock Clock;

// device bytes a batch may allocate while it runs: the larger of a linear estimate in its
// updates (records, sorted copies, entries) and the most the handle's recent batch calls have
// allocated beyond what they held (tuple buffers, hub pools, row growth), measured by the handle
uint64_t footprint(ldl_handle* h, uint64_t updates) {
  const uint64_t linear = ((uint64_t)1 << 20) + updates * 256ull;
  uint64_t held = 0, growth = 0;
  if (ldl_memory(h, &held, &growth) != LDL_OK) growth = 0;
  return linear > growth ? linear : growth;
}

}  // namespace

struct ldl_server {
  struct Request {
    uint64_t ticket;
    ldl_handle* h;
    std::vector<ldl_edge> ins;
    std::vector<ldl_pair> del;
    std::vector<ldl_edge> chg;
    uint64_t fp;
    Clock::time_point submit;
    bool done = false;
    bool claimed = false;   // a waiter owns the result (a second wait on the ticket is refused)
    int rc = LDL_OK;
    ldl_batch_stats stats{};
    double latency_ms = 0;
  };

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;                 // arrival order
  std::unordered_set<ldl_handle*> busy;       // handles held by a worker
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t budget = 0, in_use = 0, next_ticket = 1, running = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  // first admissible request in arrival order, preferring the handle just served (so a
  // graph's queued batches run back to back); caller holds mu
  Request* pick(ldl_handle* prefer) {
    std::unordered_set<ldl_handle*> blocked;
    Request* first = nullptr;
    auto it_first = queue.end();
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      Request* r = *it;
      if (blocked.count(r->h)) continue;
      blocked.insert(r->h);                   // later requests of this handle wait for it
      if (busy.count(r->h)) continue;
      r->fp = footprint(r->h, r->ins.size() + r->del.size() + r->chg.size());
      const bool fits = in_use + r->fp <= budget || running == 0;
      if (!fits) continue;
      if (r->h == prefer) {
        queue.erase(it);
        return r;
      }
      if (!first) {
        first = r;
        it_first = it;
      }
    }
    if (first) queue.erase(it_first);
    return first;
  }

  void work() {
    ldl_handle* last = nullptr;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      Request* r = nullptr;
      cv_work.wait(lk, [&] { return stop || (r = pick(last)) != nullptr; });
      if (!r) return;                         // stop with nothing admissible
      busy.insert(r->h);
      in_use += r->fp;
      ++running;
      lk.unlock();
      ldl_batch_stats st{};
      const int rc = ldl_apply_batch(r->h, r->ins.data(), r->ins.size(), r->del.data(), r->del.size(),
                                     r->chg.data(), r->chg.size(), &st);
      const double ms = std::chrono::duration<double, std::milli>(Clock::now() - r->submit).count();
      lk.lock();
      r->rc = rc;
      r->stats = st;
      r->latency_ms = ms;
      r->done = true;
      busy.erase(r->h);
      in_use -= r->fp;
      --running;
      last = r->h;
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

int ldl_server_create(uint32_t workers, uint64_t mem_budget_bytes, ldl_server** out) {
  if (!out || workers == 0 || workers > 256) return LDL_EINVAL;
  ldl_server* s = new (std::nothrow) ldl_server();
  if (!s) return LDL_ENOMEM;
  s->budget = mem_budget_bytes;
  for (uint32_t i = 0; i < workers; ++i) s->workers.emplace_back([s] { s->work(); });
  *out = s;
  return LDL_OK;
}

int ldl_server_submit(ldl_server* s, ldl_handle* h, const ldl_edge* ins, uint64_t n_ins, const ldl_pair* del,
                      uint64_t n_del, const ldl_edge* chg, uint64_t n_chg, uint64_t* ticket) {
  if (!s || !h || !ticket || (n_ins && !ins) || (n_del && !del) || (n_chg && !chg)) return LDL_EINVAL;
  auto* r = new (std::nothrow) ldl_server::Request();
  if (!r) return LDL_ENOMEM;
  r->h = h;
  r->ins.assign(ins, ins + n_ins);
  r->del.assign(del, del + n_del);
  r->chg.assign(chg, chg + n_chg);
  r->fp = 0;   // measured when the request is considered for admission (its handle idle then)
  r->submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      return LDL_EINVAL;
    }
    r->ticket = s->next_ticket++;
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
  }
  s->cv_work.notify_all();
  return LDL_OK;
}

int ldl_server_wait(ldl_server* s, uint64_t ticket, int* status, ldl_batch_stats* stats, double* latency_ms) {
  if (!s) return LDL_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return LDL_EINVAL;
  ldl_server::Request* r = it->second;
  if (r->claimed) return LDL_EINVAL;   // another thread waits on this ticket and will free it
  r->claimed = true;
  s->cv_done.wait(lk, [&] { return r->done; });
  if (status) *status = r->rc;
  if (stats) *stats = r->stats;
  if (latency_ms) *latency_ms = r->latency_ms;
  s->reqs.erase(it);
  delete r;
  return LDL_OK;
}

int ldl_server_drain(ldl_server* s) {
  if (!s) return LDL_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
  return LDL_OK;
}

void ldl_server_destroy(ldl_server* s) {
  if (!s) return;
  ldl_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
}

int ldl_apply_batches(ldl_handle* const* hs, const ldl_batch* bs, uint32_t count, uint32_t workers, int* status,
                      ldl_batch_stats* stats) {
  if (count == 0) return LDL_OK;
  if (!hs || !bs) return LDL_EINVAL;
  // entries grouped by handle in index order; each group runs on one thread
  std::vector<ldl_handle*> order;
  std::unordered_map<ldl_handle*, std::vector<uint32_t>> groups;
  for (uint32_t i = 0; i < count; ++i) {
    if (!hs[i]) return LDL_EINVAL;
    auto& g = groups[hs[i]];
    if (g.empty()) order.push_back(hs[i]);
    g.push_back(i);
  }
  uint32_t nt = workers ? workers : (uint32_t)order.size();
  if (nt > order.size()) nt = (uint32_t)order.size();
  if (nt > 64 && !workers) nt = 64;
  std::vector<int> rcs(count, LDL_OK);
  std::mutex mu;
  size_t next = 0;
  auto run = [&] {
    for (;;) {
      ldl_handle* h;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (next >= order.size()) return;
        h = order[next++];
      }
      for (uint32_t i : groups[h]) {
        ldl_batch_stats st{};
        rcs[i] = ldl_apply_batch(h, bs[i].ins, bs[i].n_ins, bs[i].del, bs[i].n_del, bs[i].chg, bs[i].n_chg, &st);
        if (stats) stats[i] = st;
      }
    }
  };
  std::vector<std::thread> ts;
  for (uint32_t t = 1; t < nt; ++t) ts.emplace_back(run);
  run();
  for (auto& t : ts) t.join();
  int first = LDL_OK;
  for (uint32_t i = 0; i < count; ++i) {
    if (status) status[i] = rcs[i];
    if (first == LDL_OK && rcs[i] != LDL_OK) first = rcs[i];
  }
  return first;
}

}  // extern "C"
