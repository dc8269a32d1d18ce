// A CPU stand-in for the part of the HIP runtime API that the library's
// host code calls, for running that host code under AddressSanitizer on a
// machine without a GPU.  It is test infrastructure, never linked into the
// library.
//
// Device memory is ordinary host memory.  Every asynchronous operation
// (copy, kernel launch, graph launch, event record) is queued on its stream
// and runs only when that stream is synchronised (or an event recorded
// after it is waited for), which is the latest point the HIP stream
// semantics allow.  A copy therefore reads its source, and writes its
// destination, as late as a real device could: a source or destination
// that is freed or goes out of scope before the synchronisation that
// covers the copy is reported by the sanitizer as a use after free or
// after return.
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <vector>

#define __host__
#define __device__
#define __global__

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorNotSupported = 801,
} hipError_t;

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
} hipMemcpyKind;

typedef enum hipMemoryType {
  hipMemoryTypeHost = 0,
  hipMemoryTypeDevice = 1,
  hipMemoryTypeManaged = 2,
} hipMemoryType;

typedef struct hipPointerAttribute_t {
  hipMemoryType type;
  int device;
} hipPointerAttribute_t;

typedef enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 0 } hipDeviceAttribute_t;
typedef enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal = 1 } hipStreamCaptureMode;

constexpr unsigned hipStreamNonBlocking = 1;
constexpr unsigned hipEventDisableTiming = 2;

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace hipstub {

struct Stream {
  std::deque<std::function<void()>> ops;
  void drain() {
    while (!ops.empty()) {
      auto op = std::move(ops.front());
      ops.pop_front();
      op();
    }
  }
};

struct Event {
  Stream* stream = nullptr;
  std::shared_ptr<bool> done = std::make_shared<bool>(true);
};

// A recorded kernel: the function and the bytes of its arguments, copied at
// node creation as the runtime does.
struct Node {
  const void* func;
  std::vector<std::vector<unsigned char>> args;
};
struct Graph {
  std::vector<Node> nodes;
};
struct GraphExec {
  std::vector<Node> nodes;
};

inline Stream& null_stream() {
  static Stream s;
  return s;
}
inline Stream& of(void* s) { return s ? *static_cast<Stream*>(s) : null_stream(); }

// Host simulations of kernels, registered by the test's launcher stubs:
// called with the argument bytes of a launch when the launch executes.
using KernelSim = void (*)(const std::vector<std::vector<unsigned char>>& args);
inline std::vector<std::pair<const void*, KernelSim>>& sims() {
  static std::vector<std::pair<const void*, KernelSim>> v;
  return v;
}
inline void run_node(const Node& n) {
  for (auto& p : sims())
    if (p.first == n.func) p.second(n.args);
}
// Argument sizes of each simulated kernel (by function), for copying the
// arguments of a graph node.
inline std::vector<std::pair<const void*, std::vector<size_t>>>& arg_sizes() {
  static std::vector<std::pair<const void*, std::vector<size_t>>> v;
  return v;
}

}  // namespace hipstub

typedef hipstub::Stream* hipStream_t;
typedef hipstub::Event* hipEvent_t;
typedef hipstub::Graph* hipGraph_t;
typedef hipstub::GraphExec* hipGraphExec_t;
typedef hipstub::Node* hipGraphNode_t;

typedef struct hipKernelNodeParams {
  dim3 blockDim;
  void* extra;
  void* func;
  dim3 gridDim;
  void** kernelParams;
  unsigned sharedMemBytes;
} hipKernelNodeParams;

inline const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "stub error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
  *v = 256;
  return hipSuccess;
}
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void*) {
  a->type = hipMemoryTypeDevice;
  a->device = 0;
  return hipSuccess;
}

inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  hipstub::of(s).ops.push_back([dst, src, n] { std::memcpy(dst, src, n); });
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t s) {
  hipstub::of(s).drain();
  return hipSuccess;
}
inline hipError_t hipStreamCreate(hipStream_t* s) {
  *s = new hipstub::Stream();
  return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { return hipStreamCreate(s); }
inline hipError_t hipStreamDestroy(hipStream_t s) {
  if (s) {
    s->drain();
    delete s;
  }
  return hipSuccess;
}
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = nullptr;
  return hipErrorNotSupported;
}

inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new hipstub::Event();
  return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  e->stream = &hipstub::of(s);
  e->done = std::make_shared<bool>(false);
  auto flag = e->done;
  e->stream->ops.push_back([flag] { *flag = true; });
  return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t e) {
  while (e->stream && !*e->done && !e->stream->ops.empty()) {
    auto op = std::move(e->stream->ops.front());
    e->stream->ops.pop_front();
    op();
  }
  return hipSuccess;
}
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f;
  return hipSuccess;
}
// Work queued on s after this call waits for e: drain e's stream first.
inline hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  hipEvent_t ev = e;
  auto flag = e->done;
  hipstub::Stream* from = e->stream;
  hipstub::of(s).ops.push_back([from, flag] {
    while (from && !*flag && !from->ops.empty()) {
      auto op = std::move(from->ops.front());
      from->ops.pop_front();
      op();
    }
  });
  (void)ev;
  return hipSuccess;
}

inline std::vector<std::vector<unsigned char>> hipstub_copy_args(const void* func, void** params) {
  std::vector<std::vector<unsigned char>> out;
  for (auto& p : hipstub::arg_sizes())
    if (p.first == func)
      for (size_t i = 0; i < p.second.size(); ++i) {
        const unsigned char* b = static_cast<const unsigned char*>(params[i]);
        out.emplace_back(b, b + p.second[i]);
      }
  return out;
}

inline hipError_t hipLaunchKernel(const void* func, dim3, dim3, void** params, size_t, hipStream_t s) {
  hipstub::Node n{func, hipstub_copy_args(func, params)};
  hipstub::of(s).ops.push_back([n] { hipstub::run_node(n); });
  return hipSuccess;
}

inline hipError_t hipGraphCreate(hipGraph_t* g, unsigned) {
  *g = new hipstub::Graph();
  return hipSuccess;
}
inline hipError_t hipGraphAddKernelNode(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t*, size_t,
                                        const hipKernelNodeParams* p) {
  g->nodes.push_back({p->func, hipstub_copy_args(p->func, p->kernelParams)});
  *node = &g->nodes.back();
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, void*, void*, size_t) {
  *x = new hipstub::GraphExec{g->nodes};
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  hipstub::GraphExec* exec = x;
  // the exec must outlive the launch: the copy of its nodes taken here
  // would hide a destroyed exec, so the launch reads the exec itself
  hipstub::of(s).ops.push_back([exec] {
    for (const auto& n : exec->nodes) hipstub::run_node(n);
  });
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
