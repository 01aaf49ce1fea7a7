// A host-only stand-in for the HIP runtime, for running the library's host code (the C ABI, the
// plan and autotuner logic, every launcher's grid computation) under AddressSanitizer and
// UndefinedBehaviorSanitizer without a GPU.  Device memory is host memory; kernels are not run:
// a launch is checked against the hardware limits and counted.  Streams, events and graphs are
// host objects that enforce the capture rules the library relies on: nothing is created,
// destroyed, allocated, freed or synchronised while a capture is open, and every stream forked
// into a capture is joined back before it ends.  Any violation prints a message and aborts.
#include <hip/hip_runtime.h>

#include <sanitizer/common_interface_defs.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>

struct ihipStream_t {
  int capture = 0;        // id of the capture this stream belongs to, 0 if none
  bool origin = false;    // the stream hipStreamBeginCapture was called on
  long ops = 0;           // work enqueued since it joined the capture
  long joined_at = -1;    // value of ops when the origin last waited on its event
};
struct ihipEvent_t {
  ihipStream_t* stream = nullptr;
  int capture = 0;
  long ops = 0;
  long stamp = 0;
};
struct ihipGraph {
  int id = 0;
};
struct hipGraphExec {
  int id = 0;
};

namespace {
std::mutex g_mu;
int g_next_capture = 1;
int g_open_captures = 0;
long g_launches = 0;
long g_stamp = 0;
std::set<ihipStream_t*> g_streams;

[[noreturn]] void fail(const char* what) {
  std::fprintf(stderr, "hip stub: %s\n", what);
  __sanitizer_print_stack_trace();   // the library call that broke the rule
  std::fflush(stderr);
  std::abort();
}
void no_capture(const char* what) {
  if (g_open_captures) {
    std::string m = std::string(what) + " while a stream capture is open";
    fail(m.c_str());
  }
}
void enqueue(hipStream_t s) {
  if (s == nullptr) {
    if (g_open_captures) fail("work on the null stream while a stream capture is open");
    return;
  }
  if (!g_streams.count(s)) fail("work on a stream that does not exist");
  s->ops++;
}
}  // namespace

extern "C" long hip_stub_launches() { return g_launches; }
extern "C" int hip_stub_open_captures() { return g_open_captures; }

hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "hip stub error"; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
  std::memset(p, 0, sizeof(*p));
  std::strcpy(p->name, "host stub");
  std::strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
  p->multiProcessorCount = 256;
  p->sharedMemPerBlock = 65536;
  p->maxThreadsPerBlock = 1024;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  switch (a) {
    case hipDeviceAttributeMultiprocessorCount: *v = 256; break;
    case hipDeviceAttributeMaxSharedMemoryPerBlock: *v = 65536; break;
    case hipDeviceAttributeMaxSharedMemoryPerMultiprocessor: *v = 163840; break;
    default: *v = 0; break;
  }
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { no_capture("hipDeviceSynchronize"); return hipSuccess; }

hipError_t hipMalloc(void** p, size_t n) {
  no_capture("hipMalloc");
  *p = std::calloc(n ? n : 1, 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) { no_capture("hipFree"); std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
  no_capture("hipHostMalloc");
  *p = std::calloc(n ? n : 1, 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) { no_capture("hipHostFree"); std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  no_capture("hipMemcpy");
  if (n) std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) {
  enqueue(st);
  if (n) std::memmove(d, s, n);
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  no_capture("hipStreamCreateWithFlags");
  *s = new ihipStream_t();
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  no_capture("hipStreamDestroy");
  if (!g_streams.erase(s)) fail("hipStreamDestroy of an unknown stream");
  delete s;
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (s == nullptr || !g_streams.count(s)) fail("capture on the null or an unknown stream");
  if (s->capture) fail("hipStreamBeginCapture on a stream already capturing");
  s->capture = g_next_capture++;
  s->origin = true;
  s->ops = 0;
  g_open_captures++;
  return hipSuccess;
}
hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus* st) {
  *st = (s && s->capture) ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!s || !s->capture || !s->origin) fail("hipStreamEndCapture on a stream not capturing");
  const int id = s->capture;
  for (ihipStream_t* o : g_streams) {
    if (o != s && o->capture == id) {
      if (o->joined_at != o->ops) fail("stream capture ended with a forked stream not joined back");
      o->capture = 0;
      o->joined_at = -1;
    }
  }
  s->capture = 0;
  s->origin = false;
  g_open_captures--;
  *g = new ihipGraph{id};
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  if (!e) fail("hipStreamWaitEvent on a null event");
  if (s && !g_streams.count(s)) fail("hipStreamWaitEvent on an unknown stream");
  if (e->capture) {
    if (!s) fail("null stream waits on an event of an open capture");
    if (!s->capture) {                         // fork: s joins the capture
      s->capture = e->capture;
      s->ops = 0;
      s->joined_at = -1;
    } else if (s->capture != e->capture) {
      fail("hipStreamWaitEvent across two captures");
    }
    if (s->origin && e->stream && e->stream != s) e->stream->joined_at = e->ops;   // join
  }
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  no_capture("hipEventCreate");
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { no_capture("hipEventDestroy"); delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (!e) fail("hipEventRecord of a null event");
  if (s && !g_streams.count(s)) fail("hipEventRecord on an unknown stream");
  if (!s && g_open_captures) fail("hipEventRecord on the null stream while a capture is open");
  e->stream = s;
  e->capture = s ? s->capture : 0;
  e->ops = s ? s->ops : 0;
  e->stamp = ++g_stamp;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (e && e->capture) fail("hipEventSynchronize on an event recorded in an open capture");
  no_capture("hipEventSynchronize");
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  no_capture("hipEventElapsedTime");
  if (!a || !b || !a->stamp || !b->stamp) return hipErrorInvalidHandle;
  *ms = 0.001f * (float)(b->stamp - a->stamp) + 0.01f;   // positive, deterministic
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  no_capture("hipGraphInstantiate");
  *x = new hipGraphExec{g->id};
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  if (!x) fail("hipGraphLaunch of a null graph");
  enqueue(s);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete x; return hipSuccess; }

hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute a, int v) {
  if (a == hipFuncAttributeMaxDynamicSharedMemorySize && (v < 0 || v > 163840))
    fail("dynamic LDS request beyond 160 KiB");
  return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int block, size_t) {
  *n = block <= 256 ? 4 : (block <= 512 ? 2 : 1);
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);          // the host shadow of the device variable
  return hipSuccess;
}

namespace {
thread_local dim3 t_grid, t_block;
thread_local size_t t_shm = 0;
thread_local hipStream_t t_stream = nullptr;
}  // namespace
hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t shm, hipStream_t s) {
  t_grid = g; t_block = b; t_shm = shm; t_stream = s;
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* shm, hipStream_t* s) {
  *g = t_grid; *b = t_block; *shm = t_shm; *s = t_stream;
  return hipSuccess;
}
hipError_t hipLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t shm, hipStream_t s) {
  if (!f || !args) fail("kernel launch without a function or arguments");
  if (g.x == 0 || g.y == 0 || g.z == 0) fail("kernel launch with an empty grid");
  if (g.y > 65535 || g.z > 65535) fail("grid y / z above 65535");
  const unsigned long threads = (unsigned long)b.x * b.y * b.z;
  if (threads == 0 || threads > 1024) fail("block of 0 or more than 1024 threads");
  if ((unsigned long)g.x * b.x >= (1ul << 32)) fail("grid x times block x reaches 2^32");
  if (shm > 163840) fail("dynamic LDS beyond 160 KiB");
  enqueue(s);
  g_launches++;
  return hipSuccess;
}

extern "C" void** __hipRegisterFatBinary(const void*) {
  static void* handle = nullptr;
  return &handle;
}
extern "C" void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int,
                                      uint3*, uint3*, dim3*, dim3*, int*) {}
extern "C" void __hipRegisterVar(void**, void*, char*, char*, int, size_t, int, int) {}
extern "C" void __hipUnregisterFatBinary(void**) {}
