// CPU stand-in of the HIP runtime calls made by libga's host files.  Device
// memory is host memory (so AddressSanitizer sees every stale or freed
// buffer a launch would touch), streams run their work when it is enqueued,
// and a capture records the enqueued work into a graph that a launch replays
// in order.  Work that must not be captured (allocation, synchronous copies,
// synchronization) aborts when a capture is open on the calling thread.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <vector>
#include <memory>

dim3 threadIdx, blockIdx, blockDim, gridDim;
struct MockStream { int id; };
struct MockEvent { int id; };
struct MockGraph { std::vector<std::function<void()>> ops; };

static thread_local MockGraph* t_capture = nullptr;
static std::mutex g_mu;  // device-side effects are serialized

void mock_enqueue(hipStream_t, std::function<void()> op) {
  if (t_capture) { t_capture->ops.push_back(std::move(op)); return; }
  std::lock_guard<std::mutex> lk(g_mu);
  op();
}

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, int, int) { *v = 256; return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock error"; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) {
  if (t_capture) { fprintf(stderr, "hipMalloc during capture\n"); abort(); }
  *p = malloc(n ? n : 1);
  if (!*p) return hipErrorOutOfMemory;
  memset(*p, 0xAB, n < 4096 ? n : 4096);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = malloc(n ? n : 1); return hipSuccess; }
hipError_t hipFree(void* p) {
  if (t_capture) { fprintf(stderr, "hipFree during capture\n"); abort(); }
  std::lock_guard<std::mutex> lk(g_mu);
  free(p);
  return hipSuccess;
}
hipError_t hipHostFree(void* p) { std::lock_guard<std::mutex> lk(g_mu); free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (t_capture) { fprintf(stderr, "hipMemcpy during capture\n"); abort(); }
  std::lock_guard<std::mutex> lk(g_mu);
  memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) {
  mock_enqueue(st, [=] { memcpy(d, s, n); });
  return hipSuccess;
}
hipError_t hipMemset(void* d, int v, size_t n) { std::lock_guard<std::mutex> lk(g_mu); memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st) {
  if (t_capture) { fprintf(stderr, "hipMemsetAsync during capture\n"); abort(); }
  mock_enqueue(st, [=] { memset(d, v, n); });
  return hipSuccess;
}
static int g_ids = 0;
hipError_t hipStreamCreate(hipStream_t* s) { *s = new MockStream{++g_ids}; return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { return hipStreamCreate(s); }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) {
  if (t_capture) { fprintf(stderr, "sync during capture\n"); abort(); }
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) { if (!e) abort(); return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  if (t_capture) { fprintf(stderr, "nested capture\n"); abort(); }
  t_capture = new MockGraph();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = t_capture; t_capture = nullptr; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) { *e = new MockGraph(*g); return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  if (t_capture) { fprintf(stderr, "graph launch during capture\n"); abort(); }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& op : e->ops) op();
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t g) { delete g; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new MockEvent{++g_ids}; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { if (!e) abort(); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.f; return hipSuccess; }
