// CPU build of the library's HIP sources, for bounds checking under
// AddressSanitizer / UndefinedBehaviorSanitizer (test infrastructure only).
//
// Every GPU thread runs as a host thread.  The lanes of one 64-wide wave meet
// at each cross-lane operation (__shfl*, __any, the wave barrier) and the
// threads of a workgroup at __syncthreads, so code whose lanes exchange data
// only through those operations computes what it computes on the device.
// Workgroups run one after another; __shared__ variables become static
// storage, which one workgroup at a time owns.  A barrier that is not
// reached by every live thread of its wave or workgroup within the time
// limit aborts the process with a message (divergent collective).
#pragma once
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <type_traits>
#include <utility>
#include <vector>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__ __restrict
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) ((const void*)&(x))

enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
typedef struct simt_stream* hipStream_t;
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 };

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace simt {

// Reusable barrier over a set of threads that may leave it (thread exit).
class Barrier {
 public:
  explicit Barrier(int n = 0) : expected_(n) {}
  void reset(int n) {
    expected_ = n;
    count_ = 0;
  }
  void wait(const char* what) {
    std::unique_lock<std::mutex> l(m_);
    const unsigned g = gen_;
    if (++count_ >= expected_) {
      release();
      return;
    }
#ifdef __SANITIZE_THREAD__
    // ThreadSanitizer does not follow the clocked condition wait of wait_for
    cv_.wait(l, [&] { return gen_ != g; });
    if (false) {
#else
    if (!cv_.wait_for(l, std::chrono::seconds(timeout_s()), [&] { return gen_ != g; })) {
#endif
      fprintf(stderr, "simt: %s barrier not reached by all live threads (%d of %d)\n", what,
              count_, expected_);
      fflush(stderr);
      abort();
    }
  }
  void drop() {
    std::lock_guard<std::mutex> l(m_);
    --expected_;
    if (count_ > 0 && count_ >= expected_) release();
  }

 private:
  static int timeout_s() {
    const char* e = getenv("SIMT_BARRIER_TIMEOUT");
    return e ? atoi(e) : 60;
  }
  void release() {
    count_ = 0;
    ++gen_;
    cv_.notify_all();
  }
  std::mutex m_;
  std::condition_variable cv_;
  int expected_ = 0, count_ = 0;
  unsigned gen_ = 0;
};

struct Wave {
  Barrier bar;
  uint64_t slot[2][64];  // exchange buffers, used alternately
  unsigned tag[2][64];    // the exchange each entry was written for
};

struct Block {
  Barrier bar;
  std::vector<Wave> waves;
};

struct Tls {
  dim3 tid, bid, bdim, gdim;
  Block* block = nullptr;
  Wave* wave = nullptr;
  int lane = 0;
  unsigned exchanges = 0;  // cross-lane operations this thread has taken part in
};
// Initial-exec TLS (a few dozen bytes of the static TLS reserve): no
// __tls_get_addr calls, whose ThreadSanitizer interceptor fails on the
// dynamic TLS of a dlopen'ed library once a launch creates a few hundred
// threads.
inline Tls& tls() {
  static thread_local Tls t __attribute__((tls_model("initial-exec")));
  return t;
}

inline int lane_id() { return tls().lane; }

// One barrier per exchange: exchange n uses buffer n % 2, and no lane can
// write that buffer again (exchange n + 2) before every lane has passed the
// barrier of exchange n + 1, i.e. has read its value of exchange n.  Each
// entry carries the exchange number it was written for; a lane that has left
// the kernel writes no more, and reading its entry gives the NaN pattern.
template <typename T>
inline T exchange(T v, int src) {
  static_assert(sizeof(T) <= 8, "exchange of a value wider than 64 bits");
  Tls& s = tls();
  Wave& w = *s.wave;
  const unsigned n = s.exchanges++;
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  w.slot[n & 1][s.lane] = bits;
  w.tag[n & 1][s.lane] = n;
  w.bar.wait("wave (shuffle)");
  const int l = src & 63;
  const uint64_t got = w.tag[n & 1][l] == n ? w.slot[n & 1][l] : ~0ull;
  T r;
  memcpy(&r, &got, sizeof(T));
  return r;
}

inline void wave_barrier() { tls().wave->bar.wait("wave"); }

// The threads of a workgroup are created once per launch and run the
// workgroups one after another: the launching thread prepares a workgroup's
// barriers, releases the threads through `start`, and waits at `done` until
// every thread has returned from the kernel.
template <typename... P, typename... A>
void launch(void (*kernel)(P...), dim3 grid, dim3 block, A&&... a) {
  std::tuple<std::decay_t<P>...> args(std::forward<A>(a)...);
  const int nthreads = (int)(block.x * block.y * block.z);
  const int nwaves = (nthreads + 63) / 64;
  const long long nblocks = (long long)grid.x * grid.y * grid.z;
  if (nthreads <= 0 || nblocks <= 0) return;
  Barrier start(nthreads + 1), done(nthreads + 1);
  std::unique_ptr<Block> cur;
  dim3 cur_bid;
  std::vector<std::thread> th;
  th.reserve(nthreads);
  for (int t = 0; t < nthreads; ++t) {
    th.emplace_back([&, t] {
      Tls& s = tls();
      s.tid = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
      s.bdim = block;
      s.gdim = grid;
      s.lane = t % 64;
      for (long long i = 0; i < nblocks; ++i) {
        start.wait("launch (start)");
        s.bid = cur_bid;
        s.block = cur.get();
        s.wave = &cur->waves[t / 64];
        s.exchanges = 0;
        auto local = args;  // kernel arguments are passed by value
        std::apply(kernel, local);
        s.wave->bar.drop();
        s.block->bar.drop();
        done.wait("launch (done)");
      }
    });
  }
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        cur = std::make_unique<Block>();  // fresh storage per workgroup
        Block& b = *cur;
        b.bar.reset(nthreads);
        b.waves = std::vector<Wave>(nwaves);
        for (int w = 0; w < nwaves; ++w) {
          const int n = std::min(64, nthreads - 64 * w);
          b.waves[w].bar.reset(n);
          for (int l = 0; l < 64; ++l) b.waves[w].tag[0][l] = b.waves[w].tag[1][l] = ~0u;
        }
        cur_bid = dim3(bx, by, bz);
        start.wait("launch (start)");
        done.wait("launch (done)");
      }
  for (auto& x : th) x.join();
}

}  // namespace simt

#define threadIdx (simt::tls().tid)
#define blockIdx (simt::tls().bid)
#define blockDim (simt::tls().bdim)
#define gridDim (simt::tls().gdim)

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  simt::launch(kernel, dim3(grid), dim3(block), __VA_ARGS__)

inline void __syncthreads() { simt::tls().block->bar.wait("workgroup"); }
inline void __builtin_amdgcn_wave_barrier() { simt::wave_barrier(); }
#define __builtin_amdgcn_fence(order, scope) __atomic_thread_fence(order)

// Cross-lane operations with HIP's index rules (width a power of two <= 64).
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  const int self = simt::lane_id();
  return simt::exchange(v, src + (self & ~(width - 1)));
}
template <typename T>
inline T __shfl_up(T v, unsigned delta, int width = 64) {
  const int self = simt::lane_id();
  int idx = self - (int)delta;
  idx = idx < (self & ~(width - 1)) ? self : idx;
  return simt::exchange(v, idx);
}
template <typename T>
inline T __shfl_down(T v, unsigned delta, int width = 64) {
  const int self = simt::lane_id();
  int idx = self + (int)delta;
  idx = (int)((self & (width - 1)) + delta) >= width ? self : idx;
  return simt::exchange(v, idx);
}
template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  const int self = simt::lane_id();
  int idx = self ^ mask;
  idx = idx >= ((self + width) & ~(width - 1)) ? self : idx;
  return simt::exchange(v, idx);
}
inline int __any(int pred) {
  simt::Tls& s = simt::tls();
  simt::Wave& w = *s.wave;
  const unsigned n = s.exchanges++;  // an exchange round, as in simt::exchange
  w.slot[n & 1][s.lane] = pred ? 1 : 0;
  w.tag[n & 1][s.lane] = n;
  w.bar.wait("wave (vote)");
  int r = 0;
  for (int l = 0; l < 64; ++l) r |= (w.tag[n & 1][l] == n && w.slot[n & 1][l]) ? 1 : 0;
  return r;
}

inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline int __clz(int x) { return x == 0 ? 32 : __builtin_clz((unsigned)x); }

// runtime
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
  const char* e = getenv("SIMT_CUS");
  *v = e ? atoi(e) : 2;
  return hipSuccess;
}
// workgroups the emulated CU holds at once: SIMT_BLOCKS_PER_CU, else 64 (every
// wave of the small test launches at once)
template <class F>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, F, int, size_t) {
  const char* e = getenv("SIMT_BLOCKS_PER_CU");
  *n = e ? atoi(e) : 64;
  return hipSuccess;
}
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
inline hipError_t hipMalloc(void** p, size_t n) {
  *p = malloc(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
