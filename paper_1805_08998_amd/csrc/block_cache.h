// Caching of device memory blocks for the library's allocator.
//
// A freed block keeps its size class, the stream that was current at the free and an
// event recorded there. It is handed out again to work on the same stream at once
// (stream order puts the new use after the old one), and to other streams only once the
// event has completed, so work still queued on the old buffer never sees it reused.
//
// Blocks go back to the device
//   * before an allocation that would take the bytes held from the device (live and
//     cached) past `soft_cap`: cached blocks are released, those freed longest ago
//     first, down to the cap less a sixteenth of it, so that the device never runs full
//     of cached blocks;
//   * when an allocation fails: idle blocks are released, largest first, and the
//     allocation is retried;
//   * on trim().
// With `trim_on_free` a free that takes the cache past `limit` also releases blocks
// down to half the limit. The library does not use that: releasing (hipFree) waits for
// the device, so every thread that frees a block past the limit would wait for the
// queued work of all streams, and with several products in flight these waits repeat
// block after block.
//
// The class holds the host logic only; the device calls come from `Ops`, so the
// policy can be exercised on the CPU with a simulated device:
//   void* malloc(size_t)           nullptr when out of memory
//   void  release(void*)           may wait for the device
//   void* record(void* stream)     an event recorded on the stream (nullptr on failure:
//                                  the block is then released at once)
//   bool  done(void* ev)           the event has completed
//   void  wait(void* ev)           wait for the event
//   void  destroy(void* ev)
//   double now()                   seconds
#pragma once

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <iterator>
#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>
#include <vector>

namespace hm {

struct CacheCounters {
  double seconds = 0;    // in malloc / release
  int64_t mallocs = 0;   // device allocations
  int64_t releases = 0;  // times blocks were handed back (OOM or trim)
  int64_t freed = 0;     // blocks handed back
};

template <class Ops>
class BlockCache {
 public:
  BlockCache(Ops ops, size_t limit, bool trim_on_free, size_t soft_cap = SIZE_MAX)
      : ops_(ops), limit_(limit), trim_on_free_(trim_on_free), soft_cap_(soft_cap) {}

  // One line per event to `f` (not owned): "a <thread> <stream> <block> <bytes> <block bytes>
  // <hit> <time>" for an allocation (hit 1: from the cache), "f <thread> <stream> <block>
  // <block bytes> <time>" for a free, "r <thread> <blocks> <seconds> <time>" for a release.
  void set_trace(FILE* f) { trace_ = f; }

  static size_t round_size(size_t b) {
    if (b <= (size_t(1) << 20)) {
      size_t r = 256;
      while (r < b) r <<= 1;
      return r;
    }
    const size_t g = size_t(2) << 20;
    return (b + g - 1) / g * g;
  }

  // A block of at least `bytes` on device `dev` for work on `stream`; nullptr when the
  // device is out of memory even after releasing every idle block.
  void* alloc(size_t bytes, int dev, void* stream) {
    if (bytes == 0) bytes = 8;
    const size_t rs = round_size(bytes);
    {
      std::lock_guard<std::mutex> lk(mu_);
      // best fit: the smallest cached class of at least rs and at most 1.5 rs whose last
      // use is ordered before this one
      for (auto it = cache_.lower_bound({dev, rs});
           it != cache_.end() && it->first.first == dev && it->first.second <= rs + rs / 2; ++it) {
        auto& v = it->second;
        for (size_t i = 0; i < v.size(); ++i) {
          if (v[i].ev && v[i].stream != stream && !ops_.done(v[i].ev)) continue;
          void* p = v[i].p;
          const size_t got = it->first.second;
          if (v[i].ev) ops_.destroy(v[i].ev);
          v.erase(v.begin() + i);
          if (v.empty()) cache_.erase(it);
          cached_ -= got;
          live_[p] = {dev, got};
          if (trace_) std::fprintf(trace_, "a %d %p %p %zu %zu 1 %.6f\n", tid(), stream, p, bytes, got, ops_.now());
          return p;
        }
      }
    }
    {
      std::vector<Cached> victims;
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (held_ + rs > soft_cap_ && cached_ > 0)
          victims = take_locked(held_ + rs - soft_cap_ + soft_cap_ / 16);
      }
      release(victims);
    }
    const double t0 = ops_.now();
    void* p = ops_.malloc(rs);
    const double t1 = ops_.now();
    for (int attempt = 0; !p && attempt < 2; ++attempt) {
      std::vector<Cached> victims;
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (cached_ == 0) break;
        // half the cache (at least the request and 1 GiB), then everything: a release
        // waits for the device, so it should not have to come again soon
        victims = take_locked(attempt == 0 ? std::max(cached_ / 2, rs + (size_t(1) << 30)) : SIZE_MAX);
      }
      release(victims);
      p = ops_.malloc(rs);
    }
    std::lock_guard<std::mutex> lk(mu_);
    cnt_.mallocs++;
    cnt_.seconds += t1 - t0;
    if (p) {
      live_[p] = {dev, rs};
      held_ += rs;
    }
    if (trace_ && p) std::fprintf(trace_, "a %d %p %p %zu %zu 0 %.6f\n", tid(), stream, p, bytes, rs, t1);
    return p;
  }

  // Returns false when p is not a live block of this cache.
  bool free(void* p, void* stream) {
    std::vector<Cached> victims;
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = live_.find(p);
      if (it == live_.end()) return false;
      const auto key = it->second;
      live_.erase(it);
      if (trace_) std::fprintf(trace_, "f %d %p %p %zu %.6f\n", tid(), stream, p, key.second, ops_.now());
      void* ev = ops_.record(stream);
      if (!ev) {
        victims.push_back({p, nullptr, nullptr, key.second, 0});  // no event: release now (waits for the device)
        cnt_.releases++;
      } else {
        cache_[key].push_back({p, ev, stream, key.second, ++seq_});
        cached_ += key.second;
        if (trim_on_free_ && cached_ > limit_) victims = take_locked(cached_ - limit_ / 2);
      }
    }
    release(victims);
    return true;
  }

  // Hands idle blocks back, largest first, until at most half the limit is cached, when
  // more than the limit is.
  void trim() {
    std::vector<Cached> victims;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (cached_ <= limit_) return;
      victims = take_locked(cached_ - limit_ / 2);
    }
    release(victims);
  }

  // The stream has been synchronized and is about to be destroyed: its blocks are idle.
  void forget_stream(void* s) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : cache_)
      for (auto& cb : kv.second)
        if (cb.ev && cb.stream == s) {
          ops_.wait(cb.ev);
          ops_.destroy(cb.ev);
          cb.ev = nullptr;
          cb.stream = nullptr;
        }
  }

  size_t cached_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return cached_;
  }
  // bytes held from the device: live blocks and cached ones
  size_t held_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return held_;
  }
  size_t soft_cap() const { return soft_cap_; }
  CacheCounters counters() {
    std::lock_guard<std::mutex> lk(mu_);
    return cnt_;
  }
  Ops& ops() { return ops_; }

 private:
  struct Cached {
    void* p;
    void* ev;
    void* stream;
    size_t bytes;
    uint64_t seq;  // order of the frees
  };
  // Takes cached blocks out of the cache until at least `need` bytes are collected:
  // largest first, or (oldest) those freed longest ago first.
  std::vector<Cached> take_locked(size_t need, bool oldest = false) {
    std::vector<Cached> out;
    cnt_.releases++;
    size_t got = 0;
    if (oldest) {
      std::vector<std::pair<uint64_t, std::pair<int, size_t>>> order;  // (seq, class)
      for (const auto& kv : cache_)
        for (const auto& cb : kv.second) order.push_back({cb.seq, kv.first});
      std::sort(order.begin(), order.end());
      for (const auto& o : order) {
        if (got >= need) break;
        auto it = cache_.find(o.second);
        auto& v = it->second;
        for (size_t i = 0; i < v.size(); ++i)
          if (v[i].seq == o.first) {
            out.push_back(v[i]);
            v.erase(v.begin() + i);
            break;
          }
        got += o.second.second;
        cached_ -= o.second.second;
        if (v.empty()) cache_.erase(it);
      }
      return out;
    }
    while (got < need && !cache_.empty()) {
      auto it = std::prev(cache_.end());
      auto& v = it->second;
      while (!v.empty() && got < need) {
        out.push_back(v.back());
        v.pop_back();
        got += it->first.second;
        cached_ -= it->first.second;
      }
      if (v.empty()) cache_.erase(it);
    }
    return out;
  }
  void release(std::vector<Cached>& v) {
    if (v.empty()) return;
    const double t0 = ops_.now();
    for (auto& cb : v) {
      if (cb.ev) {
        ops_.wait(cb.ev);
        ops_.destroy(cb.ev);
      }
      ops_.release(cb.p);
    }
    const double dt = ops_.now() - t0;
    std::lock_guard<std::mutex> lk(mu_);
    cnt_.seconds += dt;
    cnt_.freed += int64_t(v.size());
    for (const auto& cb : v) held_ -= cb.bytes;
    if (trace_) std::fprintf(trace_, "r %d %zu %.3f %.6f\n", tid(), v.size(), dt, t0);
    v.clear();
  }

  static int tid() {
    static std::atomic<int> next{0};
    thread_local int id = next++;
    return id;
  }

  Ops ops_;
  FILE* trace_ = nullptr;
  size_t limit_;
  bool trim_on_free_;
  size_t soft_cap_;
  size_t held_ = 0;
  uint64_t seq_ = 0;
  std::mutex mu_;
  std::map<std::pair<int, size_t>, std::vector<Cached>> cache_;
  std::unordered_map<void*, std::pair<int, size_t>> live_;
  size_t cached_ = 0;
  CacheCounters cnt_;
};

}  // namespace hm
