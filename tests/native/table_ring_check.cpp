// Check of the work-list table ring (csrc/table_ring.h) against simulated
// asynchronous streams.  Each stream is an in-order queue of operations that
// completes at random times; an event marks a position in one stream.  The
// simulation asks for tables under random keys on random streams, writes the
// fresh ones (a copy queued on the asking stream) and queues reads of them, the
// way the runtime does.  It checks:
//   1. a slot is rewritten only when every read of its previous contents has
//      completed, whichever stream it was queued on;
//   2. a read queued on a stream is ordered after the write of the contents it
//      reads: the write is earlier on the same stream, or the stream has been
//      made to wait for the write's event;
//   3. a key that is still in the ring is handed out again without a rewrite.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "table_ring.h"

namespace {

struct Op {
  int slot, gen;        // the slot and the generation of its contents
  bool write;
  int wait_ev = -1;     // a wait for an event instead of a table operation: the
  int wait_st = -1;     // stream and position that event marked when the wait
  size_t wait_pos = 0;  // was queued
};

struct Sim {
  std::vector<std::vector<Op>> q;      // per stream: queued operations
  std::vector<size_t> done;            // per stream: completed prefix
  std::map<int, std::pair<int, size_t>> ev;   // event -> (stream, position)
  int next_ev = 1;
  std::mt19937_64 rng{7};
  int syncs = 0;

  explicit Sim(int streams) : q(streams), done(streams, 0) {}

  bool passed(int e) {
    auto it = ev.find(e);
    if (it == ev.end()) return true;   // never recorded: nothing to wait for
    return done[it->second.first] >= it->second.second;
  }
  // complete stream s up to position pos (waits inside it complete their events first)
  void complete(int s, size_t pos) {
    while (done[s] < pos && done[s] < q[s].size()) {
      const Op &o = q[s][done[s]];
      if (o.wait_ev >= 0 && o.wait_st >= 0) complete(o.wait_st, o.wait_pos);
      ++done[s];
    }
  }
  void progress() {
    for (size_t s = 0; s < q.size(); ++s)
      if (rng() % 3 == 0) complete((int)s, done[s] + rng() % 4);
  }
};

struct SimOps {
  using Stream = int;   // stream index + 1 (0 = none)
  using Event = int;    // 0 = none
  Sim *sim;
  bool create(int *e) { *e = sim->next_ev++; return true; }
  bool record(int e, int st) { sim->ev[e] = {st - 1, sim->q[st - 1].size()}; return true; }
  bool sync(int e) {
    ++sim->syncs;
    auto it = sim->ev.find(e);
    if (it != sim->ev.end()) sim->complete(it->second.first, it->second.second);
    return true;
  }
  bool stream_wait(int st, int e) {
    Op o{-1, -1, false, e};
    auto it = sim->ev.find(e);
    if (it != sim->ev.end()) { o.wait_st = it->second.first; o.wait_pos = it->second.second; }
    sim->q[st - 1].push_back(o);
    return true;
  }
  void destroy(int) {}
};

int fails = 0;
void expect(bool ok, const char *what, int step) {
  if (!ok && fails++ < 20) std::printf("step %d: %s\n", step, what);
}

}  // namespace

int main(int argc, char **argv) {
  const int steps = argc > 1 ? atoi(argv[1]) : 20000;
  const int nstreams = 3, nkeys = 40, cap = 16;
  Sim sim(nstreams);
  SimOps ops{&sim};
  nfhmm::TableRing<SimOps> ring(ops, cap);
  std::vector<int> gen(cap, 0);          // current generation of each slot
  std::vector<int> holder(cap, -1);      // key held by each slot
  std::vector<std::pair<int, int>> write_pos(cap, {-1, 0});   // (stream, position) of the last write
  int rewrites = 0, reuses = 0;
  for (int step = 0; step < steps; ++step) {
    const int key = (int)(sim.rng() % nkeys);
    const int st = (int)(sim.rng() % nstreams);
    bool rewrite = false;
    const int slot = ring.acquire({(uint64_t)key + 100}, st + 1, &rewrite);
    expect(slot >= 0 && slot < cap, "slot out of range", step);
    if (slot < 0) break;
    int held = -1;
    for (int i = 0; i < cap; ++i)
      if (holder[i] == key) held = i;
    if (rewrite) {
      ++rewrites;
      expect(held < 0 || held == slot, "a key still in the ring was rewritten into another slot", step);
      // 1: every read of the old contents has completed
      for (int s = 0; s < nstreams; ++s)
        for (size_t i = sim.done[s]; i < sim.q[s].size(); ++i) {
          const Op &o = sim.q[s][i];
          if (o.wait_ev < 0 && o.slot == slot && !o.write) expect(false, "slot rewritten under a pending read", step);
        }
      for (int i = 0; i < cap; ++i)
        if (holder[i] == key) holder[i] = -1;
      holder[slot] = key;
      ++gen[slot];
      write_pos[slot] = {st, (int)sim.q[st].size()};
      sim.q[st].push_back(Op{slot, gen[slot], true});
      ring.written(slot, st + 1);
    } else {
      ++reuses;
      expect(held == slot, "reused slot does not hold the key", step);   // 3
    }
    // 2: the read is ordered after the write of this generation
    const auto wp = write_pos[slot];
    bool ordered = wp.first == st;
    if (!ordered)
      for (const Op &o : sim.q[st])
        if (o.wait_ev >= 0 && o.wait_st == wp.first && (int)o.wait_pos > wp.second) ordered = true;
    expect(ordered, "read not ordered after the write it reads", step);
    const int nreads = 1 + (int)(sim.rng() % 3);
    for (int r = 0; r < nreads; ++r) sim.q[st].push_back(Op{slot, gen[slot], false});
    ring.used(slot, st + 1);
    sim.progress();
  }
  std::printf("%d steps: %d rewrites, %d reuses, %d host waits, %d failures\n", steps, rewrites, reuses, sim.syncs,
              fails);
  return fails == 0 && rewrites > cap && reuses > 0 ? 0 : 1;
}
