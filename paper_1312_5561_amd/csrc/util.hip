// Device utilities: the device block cache, exclusive scan and sums used
// across the library.
#include <map>
#include <mutex>

#include "common.hpp"

namespace hfsi {

thread_local hipStream_t tls_stream = nullptr;
thread_local bool tls_idle = false;

namespace {

struct Block {
  void* p;
  hipStream_t stream;  // stream of its last use
  bool idle;           // released after that stream was synchronised
};

struct BlockCache {
  std::mutex m;
  std::map<int, std::multimap<size_t, Block>> free;  // device -> size -> block
};

BlockCache& cache() {
  static BlockCache* c = new BlockCache();  // outlives every static destructor
  return *c;
}

// take a cached block of [bytes, 2 bytes] that the current stream may use
void* take(int dev, size_t bytes, size_t* cap) {
  std::lock_guard<std::mutex> g(cache().m);
  auto& mm = cache().free[dev];
  for (auto it = mm.lower_bound(bytes); it != mm.end() && it->first <= 2 * bytes; ++it) {
    if (it->second.idle || it->second.stream == tls_stream) {
      void* p = it->second.p;
      *cap = it->first;
      mm.erase(it);
      return p;
    }
  }
  return nullptr;
}

// hipFree the idle blocks of one device (and, after synchronising it, the
// current stream's own)
void free_blocks(int dev, bool own_stream) {
  if (own_stream) (void)hipStreamSynchronize(tls_stream);
  std::lock_guard<std::mutex> g(cache().m);
  auto& mm = cache().free[dev];
  for (auto it = mm.begin(); it != mm.end();) {
    if (it->second.idle || (own_stream && it->second.stream == tls_stream)) {
      (void)hipFree(it->second.p);
      it = mm.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace

void* dev_alloc(size_t bytes, size_t* cap, int* dev) {
  bytes = (bytes + 255) & ~(size_t)255;
  HIP_CHECK(hipGetDevice(dev));
  if (void* p = take(*dev, bytes, cap)) return p;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    free_blocks(*dev, true);
    e = hipMalloc(&p, bytes);
  }
  if (e != hipSuccess)
    fail(e == hipErrorOutOfMemory ? HFSI_E_OOM : HFSI_E_HIP,
         std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
  *cap = bytes;
  return p;
}

void dev_release(void* p, size_t cap, int dev) {
  std::lock_guard<std::mutex> g(cache().m);
  cache().free[dev].insert({cap, Block{p, tls_stream, tls_idle}});
}

void dev_cache_trim() {
  std::lock_guard<std::mutex> g(cache().m);
  for (auto& kv : cache().free) {
    for (auto it = kv.second.begin(); it != kv.second.end();) {
      if (it->second.idle) {
        (void)hipSetDevice(kv.first);
        (void)hipFree(it->second.p);
        it = kv.second.erase(it);
      } else {
        ++it;
      }
    }
  }
}

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Per-tile exclusive scan; writes tile totals to block_sums.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_tiles(const int* __restrict__ in, int* __restrict__ out, int n, int* __restrict__ block_sums) {
  __shared__ int warp_tot[SCAN_THREADS / 64];
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int run = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int x = (base + k < n) ? in[base + k] : 0;
    v[k] = run;
    run += x;
  }
  // inclusive scan of per-thread totals inside the wavefront
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int inc = run;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) warp_tot[wid] = inc;
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wid; ++w) woff += warp_tot[w];
  const int excl = woff + inc - run;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) out[base + k] = v[k] + excl;
  if (threadIdx.x == SCAN_THREADS - 1) {
    int tot = 0;
    for (int w = 0; w < SCAN_THREADS / 64; ++w) tot += warp_tot[w];
    block_sums[blockIdx.x] = tot;
  }
}

__global__ void k_add_offsets(int* __restrict__ out, int n, const int* __restrict__ offs) {
  int i = blockIdx.x * SCAN_TILE + threadIdx.x;
  int o = offs[blockIdx.x];
  for (int k = 0; k < SCAN_ITEMS; ++k, i += SCAN_THREADS)
    if (i < n) out[i] += o;
}

void scan_rec(const int* in, int* out, int n, hipStream_t s) {
  if (n <= 0) return;
  int nb = div_up(n, SCAN_TILE);
  int* sums = nullptr;
  HIP_CHECK(hipMallocAsync(&sums, sizeof(int) * nb, s));
  k_scan_tiles<<<nb, SCAN_THREADS, 0, s>>>(in, out, n, sums);
  HIP_LAUNCH_CHECK();
  if (nb > 1) {
    scan_rec(sums, sums, nb, s);
    k_add_offsets<<<nb, SCAN_THREADS, 0, s>>>(out, n, sums);
    HIP_LAUNCH_CHECK();
  }
  HIP_CHECK(hipFreeAsync(sums, s));
}

__global__ void k_sum_partial(const double* __restrict__ x, int n, double* __restrict__ part) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) a += x[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// second stage: one block folds the partials and writes the total
__global__ void k_sum_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += part[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

}  // namespace

void exclusive_scan_async(const int* in, int* out, int n, hipStream_t s) { scan_rec(in, out, n, s); }

namespace {
constexpr int SCAN_EXTRA_MAX = 8;
thread_local int* g_scan_pinned = nullptr;  // [2 + SCAN_EXTRA_MAX], held until the process ends
}  // namespace

int64_t exclusive_scan(const int* in, int* out, int n, hipStream_t s, const int* extra, int n_extra,
                       int* extra_host) {
  if (n_extra < 0 || n_extra > SCAN_EXTRA_MAX) fail(HFSI_E_ARG, "exclusive_scan: too many extra values");
  if (!g_scan_pinned) HIP_CHECK(hipHostMalloc((void**)&g_scan_pinned, sizeof(int) * (2 + SCAN_EXTRA_MAX)));
  int* p = g_scan_pinned;
  p[0] = p[1] = 0;
  // the last input is read before an in-place scan overwrites it; the extra
  // values and the last output come back in the same wait
  if (n > 0) HIP_CHECK(hipMemcpyAsync(p, in + n - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  if (n_extra > 0) HIP_CHECK(hipMemcpyAsync(p + 2, extra, sizeof(int) * n_extra, hipMemcpyDeviceToHost, s));
  if (n > 0) {
    scan_rec(in, out, n, s);
    HIP_CHECK(hipMemcpyAsync(p + 1, out + n - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  HIP_CHECK(hipStreamSynchronize(s));
  for (int k = 0; k < n_extra; ++k) extra_host[k] = p[2 + k];
  return n > 0 ? (int64_t)p[1] + p[0] : 0;
}

double device_sum(hfsi_ctx* c, const double* x, int n) {
  const int nb = 256;
  c->kred.ensure(nb);
  c->scal.ensure(16);
  k_sum_partial<<<nb, 256, 0, c->stream>>>(x, n, c->kred.p);
  HIP_LAUNCH_CHECK();
  k_sum_final<<<1, 256, 0, c->stream>>>(c->kred.p, nb, c->scal.p + 15);
  HIP_LAUNCH_CHECK();
  double s = 0.0;
  HIP_CHECK(hipMemcpyAsync(&s, c->scal.p + 15, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(hipStreamSynchronize(c->stream));
  return s;
}

float elapsed_ms(hfsi_ctx* c) {
  HIP_CHECK(hipEventSynchronize(c->ev1));
  float ms = 0.f;
  HIP_CHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  return ms;
}

void require_stage(hfsi_ctx* c, int st, const char* what) {
  if (c->stage < st) fail(HFSI_E_ORDER, std::string(what) + ": called before its prerequisites");
}

}  // namespace hfsi
