// Ceiling probes: the vector FMA rate and the device copy bandwidth the
// chip sustains, measured on the box that runs the solver so that the
// kernels' roofline fractions can be read against measured ceilings as well
// as against the datasheet figures.  Instrumentation only; nothing on the
// solver's path calls them.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qb.h"

namespace {

constexpr int kChains = 8;       // independent FMA chains per thread
constexpr int kProbeBlocks = 4096;
constexpr int kProbeThreads = 256;

// kChains dependent FMA chains per thread, unrolled, iters rounds; the
// result is stored only if it equals a value it never takes, so the work
// is kept without memory traffic.
template <typename T>
__global__ __launch_bounds__(kProbeThreads) void k_fma_probe(T* __restrict__ out, int iters) {
  T a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (T)(threadIdx.x + k) * (T)1e-3;
  const T x = (T)0.9999999, y = (T)1e-7;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], x, y);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  if (s == (T)-1) out[blockIdx.x] = s;
}

// 16-byte grid-stride copy, four vectors in flight per thread, streaming
// (non-temporal) loads and stores
typedef unsigned int vec4u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_probe(const vec4u* __restrict__ src, vec4u* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const vec4u a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + stride),
                c = __builtin_nontemporal_load(src + i + 2 * stride), d = __builtin_nontemporal_load(src + i + 3 * stride);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + stride);
    __builtin_nontemporal_store(c, dst + i + 2 * stride);
    __builtin_nontemporal_store(d, dst + i + 3 * stride);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

bool ok(hipError_t e) { return e == hipSuccess; }

// milliseconds of `launch` run `reps` times between two events on stream s
template <typename F>
bool timed(hipStream_t s, int reps, F launch, float* ms) {
  hipEvent_t a, b;
  if (!ok(hipEventCreate(&a))) return false;
  if (!ok(hipEventCreate(&b))) {
    (void)hipEventDestroy(a);
    return false;
  }
  launch();  // warm-up
  bool good = ok(hipEventRecord(a, s));
  for (int r = 0; r < reps && good; ++r) launch();
  good = good && ok(hipGetLastError()) && ok(hipEventRecord(b, s)) && ok(hipEventSynchronize(b)) &&
         ok(hipEventElapsedTime(ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return good;
}

}  // namespace

extern "C" {

qb_status qb_probe_fma(int32_t precision, int32_t iters, void* scratch, double* tflops, void* stream) {
  if (!scratch || !tflops || iters < 1 || (precision != QB_F64 && precision != QB_F32)) return QB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  float ms = 0.f;
  const int reps = 3;
  bool good;
  if (precision == QB_F64)
    good = timed(s, reps, [&] { hipLaunchKernelGGL(k_fma_probe<double>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s,
                                                   (double*)scratch, iters); }, &ms);
  else
    good = timed(s, reps, [&] { hipLaunchKernelGGL(k_fma_probe<float>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s,
                                                   (float*)scratch, iters); }, &ms);
  if (!good) return QB_EHIP;
  const double flop = 2.0 * kChains * 8.0 * (double)iters * kProbeBlocks * kProbeThreads * reps;
  *tflops = flop / (ms * 1e-3) / 1e12;
  return QB_OK;
}

qb_status qb_probe_copy(const void* src, void* dst, size_t bytes, int32_t reps, double* gbps, void* stream) {
  if (!src || !dst || !gbps || reps < 1 || bytes < 16 || bytes % 16 != 0) return QB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const size_t n = bytes / 16;
  float ms = 0.f;
  const bool good = timed(s, reps, [&] { hipLaunchKernelGGL(k_copy_probe, dim3(4096), dim3(256), 0, s,
                                                            (const vec4u*)src, (vec4u*)dst, n); }, &ms);
  if (!good) return QB_EHIP;
  *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
  return QB_OK;
}

}  // extern "C"
