// emulation.h -- serial host emulation of the HIP constructs used by the
// kernels in gks.hip, for a bounds-checked CPU build of the kernel code
// (make_hostcheck.py).  Every block and every thread of a launch runs one
// after the other on the host; __syncthreads is a no-op, __shared__ arrays are
// function-static, warp shuffles return the lane's own value.  The arithmetic
// and every memory access of the kernels are those of the device code, so
// AddressSanitizer on this build checks each access of each launch against
// the exact size of its allocation.  Warp shuffles return the lane's own
// value; make_hostcheck.py lets every lane reach the wave minimum's atomic.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <functional>
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

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
inline thread_local dim3 blockIdx(0, 0, 0), threadIdx(0, 0, 0), blockDim(1, 1, 1), gridDim(1, 1, 1);

inline void __syncthreads() {}
template <typename T>
inline T __shfl_down(T v, unsigned, int) {
  return v;
}
inline unsigned long long atomicCAS(unsigned long long* p, unsigned long long cmp, unsigned long long val) {
  unsigned long long old = *p;
  if (old == cmp) *p = val;
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

template <class F>
inline void gks_emulated_run(dim3 grid, dim3 block, const F& body) {
  gridDim = grid;
  blockDim = block;
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        blockIdx = dim3(bx, by, bz);
        for (unsigned tz = 0; tz < block.z; ++tz)
          for (unsigned ty = 0; ty < block.y; ++ty)
            for (unsigned tx = 0; tx < block.x; ++tx) {
              threadIdx = dim3(tx, ty, tz);
              body();
            }
      }
}

template <class F>
inline void gks_emulated_launch(dim3 grid, dim3 block, F body) {
  if (g_emu_capture) {
    g_emu_capture->ops.push_back([=]() { gks_emulated_run(grid, block, body); });
    return;
  }
  gks_emulated_run(grid, block, body);
}
