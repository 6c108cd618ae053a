// emulation.h -- host emulation of the HIP constructs used by the kernels in
// gks.hip, for a bounds-checked CPU build of the kernel code
// (make_hostcheck.py).  The blocks of a launch run one after the other; the
// threads of a block run as coroutines (ucontext fibers) on one host thread,
// each until it finishes or reaches a cross-lane operation or __syncthreads,
// which are barriers: when every thread of the block has finished or waits,
// the waiting ones continue.  A shuffle publishes the lane's value, waits,
// reads the source lane's value and waits again; a lane that has finished
// supplies a NaN bit pattern.  __shared__ arrays are function-static.  The
// arithmetic and every memory access of the kernels are those of the device
// code, so AddressSanitizer on this build checks each access of each launch
// against the exact size of its allocation.
#pragma once
#include <sys/mman.h>
#include <ucontext.h>
#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#endif
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <functional>
#include <memory>
#include <vector>

using std::erfc;
using std::exp;
using std::fabs;
using std::fmax;
using std::fmin;
using std::isfinite;
using std::sqrt;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __builtin_amdgcn_sched_barrier(x) ((void)0)

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
inline thread_local dim3 blockIdx(0, 0, 0), threadIdx(0, 0, 0), blockDim(1, 1, 1), gridDim(1, 1, 1);

// ---- fibers: the threads of the running block ----
struct EmuFibers {
  static constexpr size_t kStack = 8u << 20;  // per thread, with a guard page below
  ucontext_t sched;
  std::vector<ucontext_t> ctx;
  std::vector<char*> stacks;
  std::vector<int> state;  // 0 runnable, 1 waiting at a barrier, 2 finished
  std::vector<unsigned long long> slot;
  std::vector<char> slot_set;
  std::function<void()>* body = nullptr;
  int cur = -1;
  void* fake_stack = nullptr;
  const void* sched_bottom = nullptr;
  size_t sched_size = 0;
  ~EmuFibers() {
    for (char* s : stacks) munmap(s, kStack);
  }
};
inline EmuFibers& emu_fibers() {
  static EmuFibers f;
  return f;
}
inline void emu_switch_to_fiber(EmuFibers& F, int t) {
#if defined(__SANITIZE_ADDRESS__)
  __sanitizer_start_switch_fiber(&F.fake_stack, F.stacks[t] + 4096, EmuFibers::kStack - 4096);
#endif
  swapcontext(&F.sched, &F.ctx[t]);
#if defined(__SANITIZE_ADDRESS__)
  __sanitizer_finish_switch_fiber(F.fake_stack, nullptr, nullptr);
#endif
}
inline void emu_switch_to_sched(EmuFibers& F, bool finished) {
  const int t = F.cur;
#if defined(__SANITIZE_ADDRESS__)
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(finished ? nullptr : &fake, F.sched_bottom, F.sched_size);
#endif
  swapcontext(&F.ctx[t], &F.sched);
#if defined(__SANITIZE_ADDRESS__)
  __sanitizer_finish_switch_fiber(fake, &F.sched_bottom, &F.sched_size);
#endif
}
inline void emu_fiber_entry() {
  EmuFibers& F = emu_fibers();
#if defined(__SANITIZE_ADDRESS__)
  __sanitizer_finish_switch_fiber(nullptr, &F.sched_bottom, &F.sched_size);
#endif
  (*F.body)();
  F.state[F.cur] = 2;
  emu_switch_to_sched(F, true);
}
// barrier of the calling thread (a wave barrier is emulated as a block barrier)
inline void emu_wait() {
  EmuFibers& F = emu_fibers();
  F.state[F.cur] = 1;
  emu_switch_to_sched(F, false);
}
inline void __syncthreads() { emu_wait(); }
template <typename T>
inline T emu_exchange(T v, int src_lane_in_wave) {
  static_assert(sizeof(T) <= 8, "exchange of at most 64 bits");
  EmuFibers& F = emu_fibers();
  const int t = F.cur, base = t - (t & 63);
  std::memcpy(&F.slot[t], &v, sizeof(T));
  F.slot_set[t] = 1;
  emu_wait();
  T r;
  const int s = base + src_lane_in_wave;
  if (s < (int)F.slot.size() && F.slot_set[s]) {
    std::memcpy(&r, &F.slot[s], sizeof(T));
  } else {
    std::memset(&r, 0xff, sizeof(T));  // an inactive lane: NaN / all ones
  }
  emu_wait();
  F.slot_set[t] = 0;
  return r;
}
inline int emu_lane() { return emu_fibers().cur & 63; }
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  const int lane = emu_lane();
  return emu_exchange(v, (lane & ~(width - 1)) + (src & (width - 1)));
}
template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  const int lane = emu_lane();
  const int s = lane ^ mask;
  return emu_exchange(v, (s & ~(width - 1)) == (lane & ~(width - 1)) ? s : lane);
}
template <typename T>
inline T __shfl_down(T v, unsigned delta, int width = 64) {
  const int lane = emu_lane();
  const int s = lane + (int)delta;
  return emu_exchange(v, (s & ~(width - 1)) == (lane & ~(width - 1)) ? s : lane);
}
inline unsigned long long atomicCAS(unsigned long long* p, unsigned long long cmp, unsigned long long val) {
  unsigned long long old = *p;
  if (old == cmp) *p = val;
  return old;
}

inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  unsigned long long old = *p;
  *p = old + v;
  return old;
}

inline unsigned long long atomicMin(unsigned long long* p, unsigned long long v) {
  unsigned long long old = *p;
  if (v < old) *p = v;
  return old;
}
inline long long __double_as_longlong(double d) {
  long long r;
  std::memcpy(&r, &d, 8);
  return r;
}
inline double __longlong_as_double(long long l) {
  double r;
  std::memcpy(&r, &l, 8);
  return r;
}

typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum { hipSuccess = 0, hipStreamNonBlocking = 1, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
// allocations of the emulated device (for the pointer queries below)
inline std::map<const char*, size_t>& emu_allocations() {
  static std::map<const char*, size_t> m;
  return m;
}
inline hipError_t hipMalloc(void** p, size_t n) {
  *p = std::calloc(1, n ? n : 1);
  if (*p) emu_allocations()[(const char*)*p] = n;
  return *p ? hipSuccess : 2;
}
enum hipMemoryType { hipMemoryTypeUnregistered = 0, hipMemoryTypeHost = 1, hipMemoryTypeDevice = 2 };
struct hipPointerAttribute_t {
  hipMemoryType type;
  int device;
};
inline bool emu_find(const void* p, const char** base, size_t* size) {
  auto& m = emu_allocations();
  auto it = m.upper_bound((const char*)p);
  if (it == m.begin()) return false;
  --it;
  if ((const char*)p >= it->first + it->second) return false;
  *base = it->first;
  *size = it->second;
  return true;
}
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) {
  const char* b;
  size_t n;
  if (!emu_find(p, &b, &n)) return 1;
  a->type = hipMemoryTypeDevice;
  a->device = 0;
  return hipSuccess;
}
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
// a small device: 2 compute units, 2 blocks of any shape per unit
enum { hipDeviceAttributeMultiprocessorCount = 1 };
inline hipError_t hipDeviceGetAttribute(int* v, int attr, int) {
  *v = attr == hipDeviceAttributeMultiprocessorCount ? 2 : 0;
  return hipSuccess;
}
template <typename F>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, F, int, size_t) {
  *n = 2;
  return hipSuccess;
}
inline hipError_t hipMemGetAddressRange(void** base, size_t* size, void* p) {
  const char* b;
  if (!emu_find(p, &b, size)) return 1;
  *base = (void*)b;
  return hipSuccess;
}
template <typename T>
inline hipError_t hipMalloc(T** p, size_t n) {
  return hipMalloc((void**)p, n);
}
inline hipError_t hipFree(void* p) {
  emu_allocations().erase((const char*)p);
  std::free(p);
  return hipSuccess;
}
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, int) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t sp, size_t w, size_t h, int,
                                   hipStream_t) {
  for (size_t r = 0; r < h; ++r) std::memmove((char*)d + r * dp, (const char*)s + r * sp, w);
  return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  std::memset(d, v, n);
  return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  static int dummy;
  *s = &dummy;
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
// device symbols are host objects here: their address is the symbol's own
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
inline const char* hipGetErrorString(hipError_t) { return "emulated"; }
inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = nullptr;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }

// a launch: every block, every thread, in order (recorded instead while a
// stream capture is open, and run by hipGraphLaunch)
struct EmuGraph {
  std::vector<std::function<void()>> ops;
};
typedef EmuGraph* hipGraph_t;
typedef EmuGraph* hipGraphExec_t;
enum { hipStreamCaptureModeThreadLocal = 2 };
inline thread_local EmuGraph* g_emu_capture = nullptr;
inline hipError_t hipStreamBeginCapture(hipStream_t, int) {
  g_emu_capture = new EmuGraph;
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = g_emu_capture;
  g_emu_capture = nullptr;
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) {
  *e = g;
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& op : e->ops) op();
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}

// dynamic LDS of the running launch (one block at a time): allocated at its
// exact size per launch, so that an access beyond it is caught
inline std::unique_ptr<unsigned char[]>& emu_lds_buffer() {
  static std::unique_ptr<unsigned char[]> b;
  return b;
}
inline unsigned char* emu_dynamic_lds() { return emu_lds_buffer().get(); }

template <class F>
inline void gks_emulated_run(dim3 grid, dim3 block, const F& body, size_t shmem = 0) {
  gridDim = grid;
  blockDim = block;
  emu_lds_buffer().reset(new unsigned char[shmem ? shmem : 1]);
  EmuFibers& E = emu_fibers();
  const int n = (int)(block.x * block.y * block.z);
  while ((int)E.stacks.size() < n) {
    void* m = mmap(nullptr, EmuFibers::kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE,
                   -1, 0);
    if (m == MAP_FAILED) std::abort();
    mprotect(m, 4096, PROT_NONE);  // guard page: a stack overflow faults
    E.stacks.push_back((char*)m);
  }
  E.ctx.resize(n);
  E.state.assign(n, 0);
  E.slot.assign(n, 0);
  E.slot_set.assign(n, 0);
  std::function<void()> fn = body;
  E.body = &fn;
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        blockIdx = dim3(bx, by, bz);
        for (int t = 0; t < n; ++t) {
          getcontext(&E.ctx[t]);
          E.ctx[t].uc_stack.ss_sp = E.stacks[t] + 4096;
          E.ctx[t].uc_stack.ss_size = EmuFibers::kStack - 4096;
          E.ctx[t].uc_link = nullptr;
          makecontext(&E.ctx[t], emu_fiber_entry, 0);
          E.state[t] = 0;
          E.slot_set[t] = 0;
        }
        for (;;) {
          bool any = false;
          for (int t = 0; t < n; ++t) {
            if (E.state[t] != 0) continue;
            threadIdx = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
            E.cur = t;
            emu_switch_to_fiber(E, t);
            any = true;
          }
          // every thread has finished or waits at a barrier: release them
          bool waiting = false;
          for (int t = 0; t < n; ++t)
            if (E.state[t] == 1) {
              E.state[t] = 0;
              waiting = true;
            }
          if (!waiting) break;
          (void)any;
        }
      }
  E.body = nullptr;
  E.cur = -1;
}

template <class F>
inline void gks_emulated_launch(dim3 grid, dim3 block, F body, size_t shmem = 0) {
  if (g_emu_capture) {
    g_emu_capture->ops.push_back([=]() { gks_emulated_run(grid, block, body, shmem); });
    return;
  }
  gks_emulated_run(grid, block, body, shmem);
}
