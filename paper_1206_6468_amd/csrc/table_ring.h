// Bookkeeping of a context's ring of work-list tables (host code only).
//
// A table describes a set of jobs for every launch of a round: their
// descriptors and, per launch kind, the prefix sums of blocks per job.  It is
// identified by the ids of those jobs (its key).  Kernels read a table's device
// copy asynchronously, on whatever stream they were launched, so a slot may be
// rewritten only once every launch that read it has finished, whichever stream
// it ran on:
//   * each stream that launched work reading a slot records an event after the
//     last such launch (used); recycling a slot first waits for all of them;
//   * the write itself (a host-to-device copy on the stream that asked for the
//     table) leaves an event (written); the next rewrite of the pinned host copy
//     waits for it, and a stream other than the writer that is handed the same
//     slot under the same key is made to wait for it on the device.
// The operations on streams and events come from Ops, so that the policy can be
// checked on the CPU with simulated streams:
//   Ops::Stream, Ops::Event             handle types (value-initialised = none)
//   bool Ops::create(Event *)           a new event
//   bool Ops::record(Event, Stream)     mark the current end of a stream
//   bool Ops::sync(Event)               host waits until the event has passed
//   bool Ops::stream_wait(Stream, Event) the stream waits for the event
//   void Ops::destroy(Event)
#pragma once
#include <cstdint>
#include <vector>

namespace nfhmm {

template <class Ops>
class TableRing {
 public:
  using Stream = typename Ops::Stream;
  using Event = typename Ops::Event;

  TableRing(Ops &ops, int capacity) : ops_(ops), slots_(capacity > 0 ? capacity : 1) {}
  TableRing(const TableRing &) = delete;
  TableRing &operator=(const TableRing &) = delete;
  ~TableRing() {
    for (Slot &s : slots_) {
      if (s.has_written) ops_.destroy(s.written);
      for (Use &u : s.uses) ops_.destroy(u.ev);
    }
  }

  int capacity() const { return (int)slots_.size(); }

  // The slot for `key`, to be read by launches on `st`.  *rewrite is set when
  // the caller must fill the slot and then call written(); false means the slot
  // already holds this key (and `st` has been ordered after its write).
  // Returns -1 when a stream or event operation failed.
  int acquire(const std::vector<uint64_t> &key, Stream st, bool *rewrite) {
    *rewrite = false;
    if (!key.empty())
      for (int i = 0; i < (int)slots_.size(); ++i) {
        Slot &s = slots_[i];
        if (s.valid && s.key == key) {
          if (!(s.writer == st) && s.has_written && !ops_.stream_wait(st, s.written)) return -1;
          return i;
        }
      }
    const int i = next_;
    next_ = (next_ + 1) % (int)slots_.size();
    Slot &s = slots_[i];
    // every launch that read the old contents, on every stream, has finished;
    // and so has the copy out of the host buffer about to be overwritten
    for (Use &u : s.uses)
      if (u.live) {
        if (!ops_.sync(u.ev)) return -1;
        u.live = false;
      }
    if (s.has_written && !ops_.sync(s.written)) return -1;
    s.valid = false;
    s.key = key;
    *rewrite = true;
    return i;
  }

  // The caller has queued the copy of slot i's contents on st.
  bool written(int i, Stream st) {
    Slot &s = slots_[i];
    if (!s.has_written) {
      if (!ops_.create(&s.written)) return false;
      s.has_written = true;
    }
    if (!ops_.record(s.written, st)) return false;
    s.writer = st;
    s.valid = true;
    return true;
  }

  // The caller has queued, on st, the last launch that reads slot i for now.
  bool used(int i, Stream st) {
    Slot &s = slots_[i];
    Use *u = nullptr;
    for (Use &x : s.uses)
      if (x.live && x.st == st) { u = &x; break; }
    if (!u)
      for (Use &x : s.uses)
        if (!x.live) { u = &x; break; }
    if (!u) {
      Event e{};
      if (!ops_.create(&e)) return false;
      s.uses.push_back(Use{Stream{}, e, false});
      u = &s.uses.back();
    }
    if (!ops_.record(u->ev, st)) return false;
    u->st = st;
    u->live = true;
    return true;
  }

 private:
  struct Use {
    Stream st;
    Event ev;
    bool live;
  };
  struct Slot {
    std::vector<uint64_t> key;
    bool valid = false;
    Stream writer{};
    Event written{};
    bool has_written = false;
    std::vector<Use> uses;
  };
  Ops &ops_;
  std::vector<Slot> slots_;
  int next_ = 0;
};

}  // namespace nfhmm
