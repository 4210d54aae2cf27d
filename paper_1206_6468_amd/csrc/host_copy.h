// Host memory copies split over a few worker threads (host code only).
//
// The serving loop moves every job's inputs into the pinned staging ring and
// every job's outputs from the ring into the caller's arrays.  One thread copies
// at single-core memcpy speed, slower still into freshly allocated caller arrays
// (first-touch page faults), which for long jobs takes longer per round than the
// device takes to run the round.  A copy here is cut into 1 MiB chunks that the
// calling thread and the pool's workers claim from a shared counter.  A piece
// may ask for its floats to be checked (finite and >= 0) as they are copied,
// which costs nothing beside the copy and spares a separate pass over the input.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

namespace nfhmm {

class CopyPool {
 public:
  struct Piece {
    void *dst;
    const void *src;
    size_t bytes;
    bool check = false;   // the bytes are floats that must be finite and >= 0
  };

  explicit CopyPool(int workers) {
    for (int i = 0; i < workers; ++i) th_.emplace_back([this] { loop(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto &t : th_) t.join();
  }
  CopyPool(const CopyPool &) = delete;
  CopyPool &operator=(const CopyPool &) = delete;

  // Copy every piece (dst and src ranges must not overlap); returns when all
  // bytes are in place: true when every checked piece held only finite,
  // non-negative floats.  Several threads may call this at once.
  bool run(const Piece *p, int n) {
    Batch b;
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
      if (!p[i].bytes) continue;
      total += p[i].bytes;
      for (size_t o = 0; o < p[i].bytes; o += kChunk)   // kChunk is a multiple of 4
        b.chunks.push_back({static_cast<char *>(p[i].dst) + o, static_cast<const char *>(p[i].src) + o,
                            std::min(kChunk, p[i].bytes - o), p[i].check});
    }
    if (th_.empty() || total < 2 * kChunk) {
      int bad = 0;
      for (const Chunk &c : b.chunks) bad |= copy_chunk(c);
      return !bad;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      q_.push_back(&b);
    }
    cv_.notify_all();
    work(b);
    std::unique_lock<std::mutex> lk(mu_);
    auto it = std::find(q_.begin(), q_.end(), &b);
    if (it != q_.end()) q_.erase(it);
    // every chunk is claimed; wait for the workers still copying theirs
    done_.wait(lk, [&] { return b.users == 0; });
    return b.bad.load(std::memory_order_relaxed) == 0;
  }

 private:
  static constexpr size_t kChunk = size_t(1) << 20;
  struct Chunk {
    char *d;
    const char *s;
    size_t n;
    bool check;
  };
  struct Batch {
    std::vector<Chunk> chunks;
    std::atomic<size_t> next{0};
    std::atomic<int> bad{0};
    int users = 0;   // workers inside work(); guarded by mu_
  };

  // copy one chunk; 1 if it is checked and holds a negative or non-finite float
  static int copy_chunk(const Chunk &c) {
    memcpy(c.d, c.s, c.n);
    if (!c.check) return 0;
    const float *x = reinterpret_cast<const float *>(c.d);
    int bad = 0;
    for (size_t i = 0; i < c.n / 4; ++i) bad |= !(x[i] >= 0.0f && x[i] <= 3.40282347e38f);
    return bad;
  }

  static void work(Batch &b) {
    int bad = 0;
    for (size_t i; (i = b.next.fetch_add(1, std::memory_order_relaxed)) < b.chunks.size();)
      bad |= copy_chunk(b.chunks[i]);
    if (bad) b.bad.store(1, std::memory_order_relaxed);
  }

  void loop() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      // drop batches whose chunks are all claimed
      while (!q_.empty() && q_.front()->next.load(std::memory_order_relaxed) >= q_.front()->chunks.size())
        q_.pop_front();
      if (stop_) return;
      if (q_.empty()) {
        cv_.wait(lk);
        continue;
      }
      Batch *b = q_.front();
      ++b->users;
      lk.unlock();
      work(*b);
      lk.lock();
      if (--b->users == 0) done_.notify_all();
    }
  }

  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  std::deque<Batch *> q_;
  bool stop_ = false;
};

}  // namespace nfhmm
