// HIP runtime layer: device selection, a caching device allocator, copies, streams,
// events and fill kernels.  All device work of a context is ordered on its stream and the
// host does not wait for it before releasing buffers, so a freed block is only handed to
// later allocations bound to the same (device, stream): work queued after the release on that
// stream runs after every earlier use of the block.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace tdmps {
namespace {

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(TDMPS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Key {
  int device;
  void* stream;
  bool operator<(const Key& o) const { return device != o.device ? device < o.device : stream < o.stream; }
};
struct Block {
  size_t size;
  Key key;
};
std::mutex g_mu;
std::map<Key, std::multimap<size_t, void*>> g_free;
std::unordered_map<void*, Block> g_block;
thread_local Key tl_key{0, nullptr};  // set by dev_bind

// Sizes below 1 MiB round to 512 bytes, below 64 MiB to 2 MiB; larger ones to quarter-octave
// buckets (at most 25% over the request), so that the large per-bond intermediates, whose
// sizes drift from bond to bond, keep hitting the blocks released by earlier bonds.
size_t round_size(size_t b) {
  if (b < (1u << 20)) return (b + 511) & ~size_t(511);
  if (b < (size_t(64) << 20)) return (b + (2u << 20) - 1) & ~((size_t(2) << 20) - 1);
  size_t oct = size_t(64) << 20;
  while (oct * 2 <= b) oct *= 2;
  const size_t step = oct / 4;
  return (b + step - 1) / step * step;
}

void release_cache() {
  for (auto& lst : g_free)
    for (auto& kv : lst.second) {
      g_block.erase(kv.second);
      (void)hipFree(kv.second);
    }
  g_free.clear();
}

__global__ void fill_zero(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = i; k < n16; k += stride) p[k] = make_uint4(0, 0, 0, 0);
  if (i < ntail) tail[i] = 0;
}

__global__ void scale_kernel(double2* x, int64_t n, double ar, double ai) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) {
    double2 v = x[k];
    x[k] = make_double2(v.x * ar - v.y * ai, v.x * ai + v.y * ar);
  }
}

// FP64 complex -> FP32 complex (round to nearest), the storage of the mixed precisions' operands
__global__ void to_f32_kernel(const double2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n; k += stride) {
    const double2 v = src[k];
    dst[k] = make_float2((float)v.x, (float)v.y);
  }
}

}  // namespace

void dev_set_device(int device) { check(hipSetDevice(device), "hipSetDevice"); }

void dev_bind(int device, void* stream) {
  tl_key = Key{device, stream};
  dev_set_device(device);
}

static int64_t g_nmalloc = 0;
static double g_tmalloc = 0;

void dev_alloc_stats(double* count, double* seconds) {
  std::lock_guard<std::mutex> lk(g_mu);
  *count = (double)g_nmalloc;
  *seconds = g_tmalloc;
}

void* dev_alloc(size_t bytes) {
  size_t b = round_size(bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  auto& lst = g_free[tl_key];
  auto it = lst.lower_bound(b);
  if (it != lst.end() && it->first <= b + b / 4 + (4u << 20)) {
    void* p = it->second;
    lst.erase(it);
    return p;
  }
  void* p = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  ++g_nmalloc;
  const hipError_t e = hipMalloc(&p, b);
  g_tmalloc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_cache();
    p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  g_block[p] = Block{b, tl_key};
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_block.find(p);
  if (it == g_block.end()) return;
  g_free[it->second.key].emplace(it->second.size, p);
}

// Uploads go through pinned staging blocks so that they are truly asynchronous: a copy from
// pageable memory makes the host wait for the stream, which serialised host planning with
// device work.  A staging block is reused once the event recorded behind its last copy has
// completed; per (device, stream) at most PIN_CAP bytes are staged, beyond which the host
// waits for the oldest copy.
namespace {
struct PinBlock {
  char* p;
  size_t size;
  hipEvent_t ev;
  uint64_t stamp;  // order of last use
};
std::mutex g_pin_mu;
std::map<Key, std::vector<PinBlock>> g_pin;
uint64_t g_pin_clock = 0;
constexpr size_t PIN_MIN = (size_t)64 << 10, PIN_CAP = (size_t)1 << 30;
}  // namespace

void dev_h2d(void* dst, const void* src, size_t bytes, void* stream) {
  if (!bytes) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  int device = 0;
  check(hipGetDevice(&device), "hipGetDevice");
  auto& blocks = g_pin[Key{device, stream}];
  PinBlock* use = nullptr;
  size_t total = 0;
  for (auto& b : blocks) {
    total += b.size;
    if (b.size < bytes || (use && use->size <= b.size)) continue;
    if (hipEventQuery(b.ev) == hipSuccess) use = &b;
  }
  if (!use) {
    if (total + bytes > PIN_CAP && !blocks.empty()) {
      // wait for the least recently used block that is large enough, else grow anyway
      PinBlock* old = nullptr;
      for (auto& b : blocks)
        if (b.size >= bytes && (!old || b.stamp < old->stamp)) old = &b;
      if (old) {
        check(hipEventSynchronize(old->ev), "hipEventSynchronize");
        use = old;
      }
    }
    if (!use) {
      size_t sz = PIN_MIN;
      while (sz < bytes) sz <<= 1;
      PinBlock b{nullptr, sz, nullptr, 0};
      check(hipHostMalloc((void**)&b.p, sz, hipHostMallocDefault), "hipHostMalloc");
      check(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming), "hipEventCreate");
      blocks.push_back(b);
      use = &blocks.back();
    }
  }
  std::memcpy(use->p, src, bytes);
  check(hipMemcpyAsync(dst, use->p, bytes, hipMemcpyHostToDevice, (hipStream_t)stream), "hipMemcpyAsync H2D");
  check(hipEventRecord(use->ev, (hipStream_t)stream), "hipEventRecord");
  use->stamp = ++g_pin_clock;
}

void dev_h2d_wait(void* dst, const void* src, size_t bytes, void* stream) {
  if (!bytes) return;
  check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, (hipStream_t)stream), "hipMemcpyAsync H2D");
  check(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
}

// Readbacks land in a pinned bounce buffer per (device, stream): a copy into pageable memory
// is staged by the runtime and costs far more latency than the copy itself, and the host
// waits for every readback (singular values, convergence counters, scalar results).
namespace {
std::map<Key, std::pair<char*, size_t>> g_bounce;
constexpr size_t BOUNCE_MAX = (size_t)64 << 20;
}  // namespace

void dev_d2h(void* dst, const void* src, size_t bytes, void* stream) {
  if (!bytes) return;
  if (bytes > BOUNCE_MAX) {
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
    return;
  }
  char* buf = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    int device = 0;
    check(hipGetDevice(&device), "hipGetDevice");
    auto& b = g_bounce[Key{device, stream}];
    if (b.second < bytes) {
      if (b.first) check(hipHostFree(b.first), "hipHostFree");
      b.first = nullptr;
      b.second = 0;
      size_t sz = (size_t)64 << 10;
      while (sz < bytes) sz <<= 1;
      check(hipHostMalloc((void**)&b.first, sz, hipHostMallocDefault), "hipHostMalloc");
      b.second = sz;
    }
    buf = b.first;
  }
  check(hipMemcpyAsync(buf, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream), "hipMemcpyAsync D2H");
  check(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  std::memcpy(dst, buf, bytes);
}

void dev_d2d(void* dst, const void* src, size_t bytes, void* stream) {
  if (!bytes) return;
  check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream), "hipMemcpyAsync D2D");
}

void dev_zero(void* dst, size_t bytes, void* stream) {
  if (!bytes) return;
  size_t n16 = bytes / 16, ntail = bytes % 16;
  int threads = 256;
  size_t blocks = (n16 + threads - 1) / threads;
  if (blocks < 1) blocks = 1;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_zero, dim3((unsigned)blocks), dim3(threads), 0, (hipStream_t)stream, (uint4*)dst, n16,
                     (unsigned char*)dst + n16 * 16, ntail);
  check(hipGetLastError(), "fill_zero launch");
}

void launch_scale(cplx* x, int64_t n, cplx alpha, void* stream) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (double2*)x, n, alpha.x,
                     alpha.y);
  check(hipGetLastError(), "scale launch");
}

void launch_to_f32(const cplx* src, void* dst, int64_t n, void* stream) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (const double2*)src,
                     (float2*)dst, n);
  check(hipGetLastError(), "to_f32 launch");
}

void dev_sync(void* stream) { check(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize"); }

void* dev_stream_create() {
  hipStream_t s;
  check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
  return s;
}

void dev_stream_destroy(void* s) { (void)hipStreamDestroy((hipStream_t)s); }

// HIP graphs: a launch sequence recorded once on a (non-default) stream and replayed.
void graph_begin(void* stream) {
  check(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
}

void* graph_end(void* stream) {
  hipGraph_t g = nullptr;
  check(hipStreamEndCapture((hipStream_t)stream, &g), "hipStreamEndCapture");
  hipGraphExec_t e = nullptr;
  const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  check(r, "hipGraphInstantiate");
  return e;
}

void graph_abort(void* stream) {
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture((hipStream_t)stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
}

void graph_launch(void* exec, void* stream) {
  check(hipGraphLaunch((hipGraphExec_t)exec, (hipStream_t)stream), "hipGraphLaunch");
}

void graph_destroy(void* exec) {
  if (exec) (void)hipGraphExecDestroy((hipGraphExec_t)exec);
}

void* dev_event_create() {
  hipEvent_t e;
  check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

void dev_event_destroy(void* e) { (void)hipEventDestroy((hipEvent_t)e); }

void dev_event_record(void* e, void* stream) {
  check(hipEventRecord((hipEvent_t)e, (hipStream_t)stream), "hipEventRecord");
}

float dev_event_elapsed_ms(void* a, void* b) {
  check(hipEventSynchronize((hipEvent_t)b), "hipEventSynchronize");
  float ms = 0;
  check(hipEventElapsedTime(&ms, (hipEvent_t)a, (hipEvent_t)b), "hipEventElapsedTime");
  return ms;
}

}  // namespace tdmps
