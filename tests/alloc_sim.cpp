// The device block cache (paper_1805_08998_amd/csrc/block_cache.h) on a simulated
// device, on the CPU.
//
// Host threads, streams, events, allocation and release run on a virtual clock. One
// host thread runs at a time: the runnable thread with the earliest clock (a baton
// passed at every device call), so runs are deterministic. The device executes the work
// of all streams in submission order (a busy device shared by the streams); an event
// completes when the work queued before it on its stream has; releasing a block
// (hipFree) waits until the device is idle, as hipFree may.
//
// Modes:
//   unit                      properties of the cache, one line each: "ok <name>"
//   batch <policy> <pin>      a batch of synthetic products on 4 host threads and streams,
//                             called twice; prints one JSON line per call.
//   replay <trace> <policy> [calls]
//                             the allocations of recorded products, replayed as a batch
//     policy: free  = release on the free path past the limit (down to half of it)
//             oom   = release only when an allocation fails
//             cap   = release before an allocation that would take the bytes held past
//                     three quarters of the device, and when an allocation fails (the
//                     library's policy)
//     pin:    lock  = one pinned staging buffer behind a mutex held across the stream
//                     synchronisation of each copy
//             pool  = a staging buffer per copy, no lock held while waiting
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "block_cache.h"

namespace {

[[noreturn]] void fail(const std::string& m) {
  std::fprintf(stdout, "FAIL %s\n", m.c_str());
  std::fflush(stdout);
  std::exit(1);
}

struct Sim {
  // scheduler
  std::mutex m;
  std::condition_variable cv;
  std::vector<double> clk;
  std::vector<char> fin;
  int run = 0;
  // device
  double busy = 0;           // the device is busy until then
  std::vector<double> last;  // per stream: completion of its last queued work
  size_t cap = 0, used = 0;
  std::unordered_map<uintptr_t, size_t> blocks;
  uintptr_t next_addr = 0x100000;
  double malloc_s = 50e-6, malloc_per_byte = 1e-12, free_s = 20e-6, launch_s = 5e-6;
  size_t peak = 0;           // most bytes allocated at once
  int64_t device_waits = 0;  // releases that waited for queued work
  double device_wait_s = 0;  // host time spent in those waits
  bool fail_record = false;

  void pick() {
    run = -1;
    double best = std::numeric_limits<double>::infinity();
    for (size_t i = 0; i < clk.size(); ++i)
      if (!fin[i] && clk[i] < best) best = clk[i], run = int(i);
  }
  void enter(int me) {
    std::unique_lock<std::mutex> lk(m);
    cv.wait(lk, [&] { return run == me; });
  }
  void yield(int me) {
    std::unique_lock<std::mutex> lk(m);
    pick();
    cv.notify_all();
    cv.wait(lk, [&] { return run == me; });
  }
  void finish(int me) {
    std::unique_lock<std::mutex> lk(m);
    fin[me] = 1;
    pick();
    cv.notify_all();
  }
  void reset(int threads, int streams) {
    clk.assign(threads, 0.0);
    fin.assign(threads, 0);
    last.assign(streams, 0.0);
    run = 0;
  }
};

Sim g;
thread_local int t_me = 0;

int stream_id(void* s) { return int(reinterpret_cast<uintptr_t>(s)) - 1; }
void* stream_of(int i) { return reinterpret_cast<void*>(uintptr_t(i + 1)); }

struct SimOps {
  void* malloc(size_t b) {
    g.clk[t_me] += g.malloc_s + g.malloc_per_byte * double(b);
    void* p = nullptr;
    if (g.used + b <= g.cap) {
      g.used += b;
      g.peak = std::max(g.peak, g.used);
      p = reinterpret_cast<void*>(g.next_addr);
      g.blocks[g.next_addr] = b;
      g.next_addr += (b + 4095) / 4096 * 4096 + 4096;
    }
    g.yield(t_me);
    return p;
  }
  void release(void* p) {
    double& c = g.clk[t_me];
    if (g.busy > c) {
      g.device_waits++;
      g.device_wait_s += g.busy - c;
      c = g.busy;
    }
    c += g.free_s;
    auto it = g.blocks.find(reinterpret_cast<uintptr_t>(p));
    if (it == g.blocks.end()) fail("release of an unknown block");
    g.used -= it->second;
    g.blocks.erase(it);
    g.yield(t_me);
  }
  void* record(void* s) {
    if (g.fail_record) return nullptr;
    return new double(g.last[stream_id(s)]);
  }
  bool done(void* ev) { return g.clk[t_me] >= *static_cast<double*>(ev); }
  void wait(void* ev) { g.clk[t_me] = std::max(g.clk[t_me], *static_cast<double*>(ev)); }
  void destroy(void* ev) { delete static_cast<double*>(ev); }
  double now() { return g.clk[t_me]; }
};

using Cache = hm::BlockCache<SimOps>;

// ---------------------------------------------------------------- workload side
struct Use {  // last use of a block: its stream and when that work completes
  int stream;
  double done;
};
std::unordered_map<void*, Use> g_last_use;
std::unordered_map<void*, int> g_held;  // blocks handed out and not yet freed

void launch(int s, double dur) {
  double& c = g.clk[t_me];
  c += g.launch_s;
  const double start = std::max(g.busy, c);
  g.busy = start + dur;
  g.last[s] = g.busy;
  g.yield(t_me);
}
void sync(int s) {
  g.clk[t_me] = std::max(g.clk[t_me], g.last[s]);
  g.yield(t_me);
}

void* take(Cache& c, size_t bytes, int s) {
  void* p = c.alloc(bytes, 0, stream_of(s));
  if (!p)
    fail("out of memory: " + std::to_string(bytes >> 20) + " MiB requested, " + std::to_string(g.used >> 20) +
         " MiB allocated, " + std::to_string(c.cached_bytes() >> 20) + " MiB cached");
  if (g_held.count(p)) fail("block handed out twice");
  auto it = g_last_use.find(p);
  // reuse by another stream is only safe once the last use has completed
  if (it != g_last_use.end() && it->second.stream != s && g.clk[t_me] < it->second.done)
    fail("block reused by another stream before its last use completed");
  g_held[p] = s;
  return p;
}
void give(Cache& c, void* p, int s) {
  g_held.erase(p);
  g_last_use[p] = Use{s, g.last[s]};
  if (!c.free(p, stream_of(s))) fail("free of an unknown block");
}

// ---------------------------------------------------------------- unit properties
void unit() {
  g.reset(1, 2);
  g.cap = size_t(1) << 30;
  {
    Cache c(SimOps{}, size_t(256) << 20, false);
    // same stream: a freed block is handed out again at once, with no device call
    void* a = take(c, 1000, 0);
    launch(0, 1.0);
    give(c, a, 0);
    void* b = take(c, 900, 0);
    if (b != a || c.counters().mallocs != 1) fail("same-stream reuse");
    std::printf("ok same_stream_reuse\n");
    // another stream: not before the last use completes, then yes
    give(c, b, 0);
    void* d = take(c, 1000, 1);
    if (d == a) fail("cross-stream reuse before completion");
    g.clk[0] = g.last[0] + 1e-3;
    void* e = take(c, 1000, 1);
    if (e != a) fail("cross-stream reuse after completion");
    std::printf("ok cross_stream_after_event\n");
    // best fit within 1.5x of the rounded size, not beyond
    give(c, d, 1);
    give(c, e, 1);
    void* big = take(c, size_t(8) << 20, 1);
    give(c, big, 1);
    void* small = take(c, size_t(4) << 20, 1);
    if (small == big) fail("a block more than 1.5x the request was handed out");
    void* fit = take(c, size_t(7) << 20, 1);
    if (fit != big) fail("best fit within 1.5x");
    std::printf("ok best_fit\n");
    give(c, small, 1);
    give(c, fit, 1);
    // no release on the free path, however much is cached
    const int64_t r0 = c.counters().releases;
    std::vector<void*> v;
    for (int i = 0; i < 20; ++i) v.push_back(take(c, size_t(24) << 20, 0));
    for (void* p : v) give(c, p, 0);
    if (c.cached_bytes() <= (size_t(256) << 20) || c.counters().releases != r0) fail("release on free");
    std::printf("ok no_release_on_free\n");
    // trim(): back to half the limit, largest first
    c.trim();
    if (c.cached_bytes() > (size_t(128) << 20)) fail("trim");
    std::printf("ok trim\n");
  }
  {
    // out of memory: idle blocks are released and the allocation retried
    g.reset(1, 2);
    g.cap = size_t(100) << 20;
    g.used = 0;
    g.blocks.clear();
    g_held.clear();
    g_last_use.clear();
    Cache c(SimOps{}, size_t(1) << 40, false);
    void* a = take(c, size_t(60) << 20, 0);
    launch(0, 0.5);
    give(c, a, 0);
    void* b = take(c, size_t(90) << 20, 0);  // does not fit next to the cached 60 MiB
    if (!b || c.counters().releases != 1 || g.clk[0] < 0.5) fail("release on OOM");
    std::printf("ok oom_release_retry\n");
    give(c, b, 0);
  }
  {
    // the free path with trim_on_free past the limit waits for the device
    g.reset(1, 2);
    g.cap = size_t(1) << 30;
    g.used = 0;
    g.blocks.clear();
    g_held.clear();
    g_last_use.clear();
    Cache c(SimOps{}, size_t(64) << 20, true);
    std::vector<void*> v;
    for (int i = 0; i < 5; ++i) v.push_back(take(c, size_t(20) << 20, 0));
    launch(0, 2.0);
    for (void* p : v) give(c, p, 0);
    // the release waited for the 2 s of queued work
    if (c.counters().releases < 1 || c.counters().freed < 1 || g.clk[0] < 2.0) fail("trim on free");
    std::printf("ok trim_on_free_waits\n");
  }
  {
    // no event: the block is released at once instead of cached
    g.reset(1, 1);
    g.cap = size_t(1) << 30;
    g.used = 0;
    g.blocks.clear();
    g_held.clear();
    g_last_use.clear();
    Cache c(SimOps{}, size_t(1) << 30, false);
    void* a = take(c, 4096, 0);
    g.fail_record = true;
    give(c, a, 0);
    g.fail_record = false;
    if (c.cached_bytes() != 0 || g.used != 0) fail("record failure");
    std::printf("ok record_failure_releases\n");
  }
  {
    // forget_stream: blocks freed on a finished stream become idle for every stream
    g.reset(1, 2);
    g.cap = size_t(1) << 30;
    g.used = 0;
    g.blocks.clear();
    g_held.clear();
    g_last_use.clear();
    Cache c(SimOps{}, size_t(1) << 30, false);
    void* a = take(c, 4096, 1);
    launch(1, 3.0);
    give(c, a, 1);
    sync(1);
    c.forget_stream(stream_of(1));
    void* b = take(c, 4096, 0);
    if (b != a) fail("forget_stream");
    std::printf("ok forget_stream\n");
  }
}

// ---------------------------------------------------------------- a batch of products
// Each product: its output blocks (kept until the end of the call), subtree batches with
// a term pool each, and per batch chunks of buffers whose sizes vary continuously, an
// upload of the chunk's work lists and a few kernels. Sizes and times follow n.
struct Product {
  int64_t n;
  uint64_t seed;
};

struct PinLock {
  double free_at = 0;
};

void upload(int s, size_t bytes, bool lock, PinLock& pin) {
  double& c = g.clk[t_me];
  double t = c;
  if (lock) t = std::max(t, pin.free_at);  // wait for the holder of the staging buffer
  // the copy is ordered after the stream's queued work, and the caller waits for it
  const double start = std::max(t, g.last[s]);
  const double end = start + double(bytes) / 25e9;
  g.last[s] = std::max(g.last[s], end);
  if (lock) pin.free_at = end;
  c = end;
  g.yield(t_me);
}

void product(Cache& c, const Product& p, int s, bool lock, PinLock& pin, std::vector<void*>& outputs) {
  std::mt19937_64 rng(p.seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const double scale = double(p.n) / 65536.0;
  const double t_prod = 2.0 * scale * std::log2(double(p.n)) / 16.0;  // device seconds
  // device memory available to one of 4 products in flight
  const size_t budget = std::min<size_t>(size_t(16) << 30, g.cap / (16 * 4));
  for (int i = 0; i < 4; ++i) outputs.push_back(take(c, size_t(scale * double(size_t(256) << 20) * (0.5 + U(rng))), s));
  const int batches = 1 + int(3 * U(rng));
  const int chunks = std::max(2, int(8 * scale));
  for (int b = 0; b < batches; ++b) {
    void* pool = take(c, size_t(scale * double(size_t(6) << 30) * (0.3 + U(rng))), s);
    for (int k = 0; k < chunks; ++k) {
      std::vector<void*> buf;
      for (int j = 0; j < 24; ++j) {
        // log-uniform from 64 KiB to an eighth of the chunk budget
        const double lo = std::log(65536.0), hi = std::log(double(budget) / 8 * std::max(scale, 0.1));
        buf.push_back(take(c, size_t(std::exp(lo + (hi - lo) * U(rng))), s));
      }
      upload(s, size_t(scale * double(size_t(64) << 20)), lock, pin);
      for (int j = 0; j < 6; ++j) launch(s, t_prod / (batches * chunks * 6));
      for (void* q : buf) give(c, q, s);
    }
    give(c, pool, s);
  }
}

void batch(const char* policy, bool lock) {
  const bool trim_on_free = std::strcmp(policy, "free") == 0;
  const int S = 4;
  g.cap = size_t(288) << 30;
  g.used = 0;
  g.blocks.clear();
  g_held.clear();
  g_last_use.clear();
  g.reset(S, S);
  Cache c(SimOps{}, g.cap / 4, trim_on_free, std::strcmp(policy, "cap") == 0 ? g.cap / 4 * 3 : SIZE_MAX);
  PinLock pin;
  std::mt19937_64 rng(7);
  std::vector<Product> prods(64);
  for (auto& p : prods) {
    p.n = int64_t(std::exp(std::log(4096.0) + (std::log(65536.0) - std::log(4096.0)) *
                                                  std::uniform_real_distribution<double>(0, 1)(rng)));
    p.seed = rng();
  }
  std::vector<std::vector<void*>> outs(2);
  double t_begin = 0;
  for (int call = 0; call < 2; ++call) {
    const hm::CacheCounters c0 = c.counters();
    const int64_t w0 = g.device_waits;
    const double ws0 = g.device_wait_s;
    std::vector<std::vector<void*>> per(S);
    int next = 0;
    std::mutex next_mu;
    std::vector<std::thread> th;
    for (int w = 0; w < S; ++w) {
      g.clk[w] = t_begin;
      g.fin[w] = 0;
    }
    {
      std::lock_guard<std::mutex> lk(g.m);
      g.pick();
    }
    for (int w = 0; w < S; ++w)
      th.emplace_back([&, w] {
        t_me = w;
        g.enter(w);
        for (;;) {
          int k;
          {
            std::lock_guard<std::mutex> lk(next_mu);
            k = next++;
          }
          if (k >= int(prods.size())) break;
          product(c, prods[k], w, lock, pin, per[w]);
        }
        sync(w);
        g.finish(w);
      });
    for (auto& x : th) x.join();
    double t_end = 0;
    for (double x : g.clk) t_end = std::max(t_end, x);
    const hm::CacheCounters c1 = c.counters();
    std::printf(
        "{\"call\": %d, \"wall_s\": %.3f, \"mallocs\": %lld, \"releases\": %lld, \"freed_blocks\": %lld, "
        "\"alloc_s\": %.3f, \"device_waits\": %lld, \"device_wait_s\": %.3f, \"cached_gib\": %.2f, "
        "\"used_gib\": %.2f, \"peak_gib\": %.2f}\n",
        call, t_end - t_begin, (long long)(c1.mallocs - c0.mallocs), (long long)(c1.releases - c0.releases),
        (long long)(c1.freed - c0.freed), c1.seconds - c0.seconds, (long long)(g.device_waits - w0),
        g.device_wait_s - ws0, double(c.cached_bytes()) / double(size_t(1) << 30),
        double(g.used) / double(size_t(1) << 30), double(g.peak) / double(size_t(1) << 30));
    std::fflush(stdout);
    g.peak = g.used;
    for (auto& v : per) outs[call].insert(outs[call].end(), v.begin(), v.end());
    t_begin = t_end;
  }
  // the outputs of both calls are live until here, as in a caller that compares them
  t_me = 0;
  {
    std::lock_guard<std::mutex> lk(g.m);
    g.fin[0] = 0;
    g.pick();
  }
  for (auto& v : outs)
    for (void* p : v) give(c, p, 0);
}

// ---------------------------------------------------------------- replay of a trace
// Recorded allocations of products run one at a time (tests/data/record_alloc_trace.py:
// "p <product> <n>", "a <id> <bytes> <gap_us>", "f <id> <gap_us>") are replayed as a
// batch on 4 host threads and streams: each product's allocations and frees in their
// order, the time between two of them as device work on the product's stream that its
// thread waits for. Blocks a product does not free are its output, live until the end.
struct Op {
  bool alloc;
  size_t bytes;
  int64_t id;  // allocation number within the product
  double gap;  // device seconds before the operation
};

std::vector<std::vector<Op>> read_trace(const char* path) {
  std::vector<std::vector<Op>> prods;
  FILE* f = std::fopen(path, "r");
  if (!f) fail("cannot open the trace");
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    long long a = 0, b = 0, c = 0;
    if (line[0] == 'p') {
      prods.emplace_back();
    } else if (line[0] == 'a' && std::sscanf(line + 1, "%lld %lld %lld", &a, &b, &c) == 3) {
      if (prods.empty()) fail("trace: allocation outside a product");
      prods.back().push_back(Op{true, size_t(b), a, double(c) * 1e-6});
    } else if (line[0] == 'f' && std::sscanf(line + 1, "%lld %lld", &a, &c) == 2) {
      if (prods.empty()) fail("trace: free outside a product");
      prods.back().push_back(Op{false, 0, a, double(c) * 1e-6});
    }
  }
  std::fclose(f);
  return prods;
}

void replay(const char* trace, const char* policy, int calls) {
  const bool trim_on_free = std::strcmp(policy, "free") == 0;
  const int S = 4;
  const auto prods = read_trace(trace);
  g.cap = size_t(288) << 30;
  g.used = 0;
  g.blocks.clear();
  g_held.clear();
  g_last_use.clear();
  g.reset(S, S);
  Cache c(SimOps{}, g.cap / 4, trim_on_free, std::strcmp(policy, "cap") == 0 ? g.cap / 4 * 3 : SIZE_MAX);
  double t_begin = 0;
  std::vector<std::vector<void*>> kept;  // blocks still live at a product's end (its output C)
  for (int call = 0; call < calls; ++call) {
    const hm::CacheCounters c0 = c.counters();
    const int64_t w0 = g.device_waits;
    const double ws0 = g.device_wait_s;
    int next = 0;
    std::mutex next_mu;
    std::vector<std::thread> th;
    std::vector<std::vector<void*>> outs(S);
    for (int w = 0; w < S; ++w) {
      g.clk[w] = t_begin;
      g.fin[w] = 0;
    }
    {
      std::lock_guard<std::mutex> lk(g.m);
      g.pick();
    }
    for (int w = 0; w < S; ++w)
      th.emplace_back([&, w] {
        t_me = w;
        g.enter(w);
        for (;;) {
          int k;
          {
            std::lock_guard<std::mutex> lk(next_mu);
            k = next++;
          }
          if (k >= int(prods.size())) break;
          std::unordered_map<int64_t, void*> blk;
          for (const Op& op : prods[k]) {
            if (op.gap > 0) {
              launch(w, op.gap);
              sync(w);
            }
            if (op.alloc) {
              blk[op.id] = take(c, op.bytes, w);
            } else {
              auto it = blk.find(op.id);
              if (it == blk.end()) fail("replay: free of a block not allocated");
              give(c, it->second, w);
              blk.erase(it);
            }
          }
          for (auto& kv : blk) outs[w].push_back(kv.second);
        }
        sync(w);
        g.finish(w);
      });
    for (auto& x : th) x.join();
    double t_end = 0;
    for (double x : g.clk) t_end = std::max(t_end, x);
    const hm::CacheCounters c1 = c.counters();
    std::printf(
        "{\"call\": %d, \"wall_s\": %.3f, \"mallocs\": %lld, \"releases\": %lld, \"freed_blocks\": %lld, "
        "\"alloc_s\": %.3f, \"device_waits\": %lld, \"device_wait_s\": %.3f, \"cached_gib\": %.2f, "
        "\"used_gib\": %.2f, \"peak_gib\": %.2f}\n",
        call, t_end - t_begin, (long long)(c1.mallocs - c0.mallocs), (long long)(c1.releases - c0.releases),
        (long long)(c1.freed - c0.freed), c1.seconds - c0.seconds, (long long)(g.device_waits - w0),
        g.device_wait_s - ws0, double(c.cached_bytes()) / double(size_t(1) << 30),
        double(g.used) / double(size_t(1) << 30), double(g.peak) / double(size_t(1) << 30));
    std::fflush(stdout);
    g.peak = g.used;
    std::vector<void*> all;
    for (auto& v : outs) all.insert(all.end(), v.begin(), v.end());
    kept.push_back(all);
    t_begin = t_end;
  }
  t_me = 0;
  {
    std::lock_guard<std::mutex> lk(g.m);
    g.fin[0] = 0;
    g.pick();
  }
  for (auto& v : kept)
    for (void* p : v) give(c, p, 0);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc >= 4 && std::strcmp(argv[1], "replay") == 0) {
    replay(argv[2], argv[3], argc >= 5 ? std::atoi(argv[4]) : 2);
    return 0;
  }
  if (argc >= 2 && std::strcmp(argv[1], "unit") == 0) {
    unit();
    return 0;
  }
  if (argc >= 4 && std::strcmp(argv[1], "batch") == 0) {
    batch(argv[2], std::strcmp(argv[3], "lock") == 0);
    return 0;
  }
  std::fprintf(stderr, "usage: alloc_sim unit | batch free|oom|cap lock|pool | replay <trace> free|oom|cap [calls]\n");
  return 2;
}
