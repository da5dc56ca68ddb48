// Peak-rate probes (diagnostics): the MFMA issue rates and HBM copy bandwidth
// this device reaches, measured with HIP events, so measured kernel rates can
// be set against what the chip delivers as well as against its datasheet.
//
// MFMA probes: every wave runs a loop of independent accumulator chains on
// register operands (no memory traffic in the loop) and stores its
// accumulators once at the end.  The copy probe streams one buffer into
// another with 16-byte loads and stores.
#include <algorithm>
#include <vector>

#include "gwc_internal.h"

namespace gwc {

typedef double pd4 __attribute__((ext_vector_type(4)));
typedef float pf4 __attribute__((ext_vector_type(4)));
typedef __bf16 pbf8 __attribute__((ext_vector_type(8)));
typedef _Float16 ph8 __attribute__((ext_vector_type(8)));

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_CHAINS = 4;

__global__ void __launch_bounds__(PROBE_THREADS)
probe_mfma_f64_kernel(int iters, double seed, double *__restrict__ out) {
  const double a = seed + 1e-3 * threadIdx.x, b = seed - 1e-3 * threadIdx.x;
  pd4 acc[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = pd4{0.0, 0.0, 0.0, 0.0};
  // iters is a multiple of 32: the unrolled body keeps the accumulators in
  // place across many MFMAs
  for (int it = 0; it < iters; it += 32) {
#pragma unroll
    for (int u = 0; u < 32; ++u)
#pragma unroll
      for (int c = 0; c < PROBE_CHAINS; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

template <class T, class V>
__device__ __forceinline__ pf4 probe_mfma16(V a, V b, pf4 c);
template <>
__device__ __forceinline__ pf4 probe_mfma16<__bf16, pbf8>(pbf8 a, pbf8 b, pf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ pf4 probe_mfma16<_Float16, ph8>(ph8 a, ph8 b, pf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

template <class T, class V>
__global__ void __launch_bounds__(PROBE_THREADS)
probe_mfma16_kernel(int iters, float seed, float *__restrict__ out) {
  V a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (T)(seed + 1e-3f * (threadIdx.x + e));
    b[e] = (T)(seed - 1e-3f * (threadIdx.x + e));
  }
  pf4 acc[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = pf4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; it += 32) {
#pragma unroll
    for (int u = 0; u < 32; ++u)
#pragma unroll
      for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = probe_mfma16<T, V>(a, b, acc[c]);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

// FP8 (E4M3) MFMA: K = 32 (v_mfma_f32_16x16x32_fp8_fp8, 8 bytes per lane and
// operand) or K = 128 (v_mfma_f32_16x16x128_f8f6f4 without block scales, 32
// bytes per lane and operand).  The operand bytes are small normal E4M3
// values (no NaN codes).
typedef int pi8 __attribute__((ext_vector_type(8)));
template <int K>
__global__ void __launch_bounds__(PROBE_THREADS)
probe_mfma_fp8_kernel(int iters, int seed, float *__restrict__ out) {
  pi8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (seed + (int)threadIdx.x + e) & 0x37373737;
    b[e] = (seed + 3 * (int)threadIdx.x + e) & 0x37373737;
  }
  pf4 acc[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = pf4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; it += 32) {
#pragma unroll
    for (int u = 0; u < 32; ++u)
#pragma unroll
      for (int c = 0; c < PROBE_CHAINS; ++c) {
        if constexpr (K == 128) {
          acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[c], 0, 0, 0, 0, 0, 0);
        } else {
          const long a2 = ((long)(unsigned)a[1] << 32) | (unsigned)a[0];
          const long b2 = ((long)(unsigned)b[1] << 32) | (unsigned)b[0];
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a2, b2, acc[c], 0, 0, 0);
        }
      }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

// Four independent 16-byte loads in flight per thread and iteration; n is a
// multiple of 4 * gridDim.x * PROBE_THREADS (the host sizes it so).
__global__ void __launch_bounds__(PROBE_THREADS)
probe_copy_kernel(const double2 *__restrict__ src, double2 *__restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * PROBE_THREADS;
  for (size_t i = (size_t)blockIdx.x * PROBE_THREADS + threadIdx.x; i < n; i += 4 * stride) {
    const double2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
}

namespace {

struct ProbeError {
  hipError_t e;
};
#define PROBECHECK(x)                   \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) throw ProbeError{e_}; \
  } while (0)

// Median of `reps` timed launches (ms) of `launch`, after one untimed launch.
template <class Launch>
double time_launches(hipStream_t s, int reps, Launch &&launch) {
  hipEvent_t a, b;
  PROBECHECK(hipEventCreate(&a));
  PROBECHECK(hipEventCreate(&b));
  launch();
  PROBECHECK(hipGetLastError());
  std::vector<float> ms(reps);
  for (int r = 0; r < reps; ++r) {
    PROBECHECK(hipEventRecord(a, s));
    launch();
    PROBECHECK(hipEventRecord(b, s));
    PROBECHECK(hipEventSynchronize(b));
    PROBECHECK(hipEventElapsedTime(&ms[r], a, b));
  }
  PROBECHECK(hipEventDestroy(a));
  PROBECHECK(hipEventDestroy(b));
  std::sort(ms.begin(), ms.end());
  return ms[reps / 2];
}

}  // namespace

// kind 0: FP64 MFMA TFLOP/s; 1: BF16 MFMA TFLOP/s; 2: FP16 MFMA TFLOP/s;
// 3: HBM copy GB/s (bytes read + written); 4: FP8 MFMA K = 32 TFLOP/s;
// 5: FP8 MFMA K = 128 TFLOP/s.  Returns hipSuccess or the error.
hipError_t probe_peak(int kind, hipStream_t s, double *value) {
  try {
    int dev = 0, n_cu = 0;
    PROBECHECK(hipGetDevice(&dev));
    PROBECHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = n_cu * 8;
    if (kind <= 2 || kind == 4 || kind == 5) {
      const int iters = 16384;  // 10-20 ms per launch at the datasheet rates
      void *out = nullptr;
      PROBECHECK(hipMallocAsync(&out, (size_t)blocks * PROBE_THREADS * sizeof(double), s));
      double ms;
      if (kind == 0) {
        ms = time_launches(s, 5, [&] {
          probe_mfma_f64_kernel<<<blocks, PROBE_THREADS, 0, s>>>(iters, 0.5, (double *)out);
        });
      } else if (kind == 1) {
        ms = time_launches(s, 5, [&] {
          probe_mfma16_kernel<__bf16, pbf8><<<blocks, PROBE_THREADS, 0, s>>>(iters, 0.5f, (float *)out);
        });
      } else if (kind == 2) {
        ms = time_launches(s, 5, [&] {
          probe_mfma16_kernel<_Float16, ph8><<<blocks, PROBE_THREADS, 0, s>>>(iters, 0.5f, (float *)out);
        });
      } else if (kind == 4) {
        ms = time_launches(s, 5, [&] {
          probe_mfma_fp8_kernel<32><<<blocks, PROBE_THREADS, 0, s>>>(iters, 0x01020304, (float *)out);
        });
      } else {
        ms = time_launches(s, 5, [&] {
          probe_mfma_fp8_kernel<128><<<blocks, PROBE_THREADS, 0, s>>>(iters, 0x01020304, (float *)out);
        });
      }
      PROBECHECK(hipFreeAsync(out, s));
      PROBECHECK(hipStreamSynchronize(s));
      const double per_mfma = kind == 0 ? 2.0 * 16 * 16 * 4 : kind == 5 ? 2.0 * 16 * 16 * 128 : 2.0 * 16 * 16 * 32;
      const double waves = (double)blocks * (PROBE_THREADS / 64);
      *value = waves * iters * PROBE_CHAINS * per_mfma / (ms * 1e-3) / 1e12;
      return hipSuccess;
    }
    if (kind == 3) {
      const size_t bytes = (size_t)4 << 30;
      const size_t n = bytes / sizeof(double2);
      const int cblocks = n_cu * 16;
      if (n % (4 * (size_t)cblocks * PROBE_THREADS) != 0) throw ProbeError{hipErrorInvalidValue};
      void *src = nullptr, *dst = nullptr;
      PROBECHECK(hipMallocAsync(&src, bytes, s));
      PROBECHECK(hipMallocAsync(&dst, bytes, s));
      PROBECHECK(hipMemsetAsync(src, 0, bytes, s));
      const double ms = time_launches(s, 5, [&] {
        probe_copy_kernel<<<cblocks, PROBE_THREADS, 0, s>>>((const double2 *)src, (double2 *)dst, n);
      });
      PROBECHECK(hipFreeAsync(src, s));
      PROBECHECK(hipFreeAsync(dst, s));
      PROBECHECK(hipStreamSynchronize(s));
      *value = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
      return hipSuccess;
    }
  } catch (const ProbeError &pe) {
    return pe.e;
  }
  return hipErrorInvalidValue;
}

}  // namespace gwc
