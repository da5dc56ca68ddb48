// Mixed-precision polarisability: Pi(z) = L diag(chi(z)) L^T with 16-bit MFMA
// inputs and FP32 accumulation (precision form of the Pi build).
//
// Each operand x is split into two 16-bit values, x ~ hi + lo with
// hi = round16(x), lo = round16(x - hi), and the product is formed from three
// MFMA passes, hi*hi + hi*lo + lo*hi (the lo*lo term, relative size 2^-2p, is
// dropped).  B = L is split once per call; the A operand L_Pk chi_k is formed
// per frequency in FP32 from an FP32 copy of L and FP32-rounded chi (chi itself
// is computed in FP64) and split in registers.
//
//   BF16X3: bf16 (8-bit significand) -> ~2^-16 relative per product
//   FP16X3: fp16 (11-bit significand) with power-of-two scaling: columns of B
//           are scaled by 2^e_k (undone in A), and each frequency's A operand
//           by 2^g_f (undone on the FP32 result), keeping hi and lo parts in the
//           fp16 normal range -> ~2^-22 relative per product
//   FP8X3:  fp8 e4m3 (4-bit significand, largest 448) with the same scaling
//           aimed one binade higher -> ~2^-7 relative per product
//
// Tile: one 128 x 256 block of Pi per workgroup and frequency for the 16-bit
// forms (8 waves of 32 x 128, v_mfma_f32_16x16x32_{bf16,f16}; every B chunk
// staged in LDS serves 128 rows), 64 x 256 with 4 waves for FP8 (whose B chunk
// is half the bytes, so occupancy pays more than reuse); upper-triangle blocks
// only, the result written as 1 - Pi (FP64) into the bordered matrix with its
// mirror.
#include "gwc_internal.h"

namespace gwc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef unsigned char uc8 __attribute__((ext_vector_type(8)));

// fp8 e4m3 (the MFMA's fp8 operand format on this target)
struct e4m3 {};

constexpr int MX_TC = MX_TILE_COLS;  // tile columns
constexpr int MX_NB = MX_TC / 32;      // 16-column blocks per wave (a wave covers MX_TC / 2)
constexpr int MX_KC = 32;    // K per LDS stage

// 16-bit splits (round to nearest even)
__device__ __forceinline__ unsigned short to_bits(__bf16 x) { return __builtin_bit_cast(unsigned short, x); }
__device__ __forceinline__ unsigned short to_bits(_Float16 x) { return __builtin_bit_cast(unsigned short, x); }

template <class T>
__device__ __forceinline__ void split16(float x, unsigned short &hi, unsigned short &lo) {
  const T h = (T)x;
  const float r = x - (float)h;
  hi = to_bits(h);
  lo = to_bits((T)r);
}

// Per-form operand traits: storage element E, MFMA operand V (8 elements of
// one lane), the hi/lo split, the product, and the binade the scaling aims the
// largest |value| at (0: no scaling).
template <class T>
struct Mix;
template <>
struct Mix<__bf16> {
  using E = unsigned short;
  using V = us8;
  static constexpr int TARGET = 0;
  static __device__ __forceinline__ void split(float x, E &h, E &l) { split16<__bf16>(x, h, l); }
  static __device__ __forceinline__ f4 mfma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
  }
};
template <>
struct Mix<_Float16> {
  using E = unsigned short;
  using V = us8;
  static constexpr int TARGET = 7;  // max |x| in [2^6, 2^7)
  static __device__ __forceinline__ void split(float x, E &h, E &l) { split16<_Float16>(x, h, l); }
  static __device__ __forceinline__ f4 mfma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
  }
};
template <>
struct Mix<e4m3> {
  using E = unsigned char;
  using V = uc8;
  static constexpr int TARGET = 8;  // max |x| in [2^7, 2^8), below the e4m3 limit 448
  static __device__ __forceinline__ void split(float x, E &h, E &l) {
    const int hp = __builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false);  // round to nearest even
    const float r = x - __builtin_amdgcn_cvt_f32_fp8(hp, 0);
    const int lp = __builtin_amdgcn_cvt_pk_fp8_f32(r, 0.0f, 0, false);
    h = (E)(hp & 0xff);
    l = (E)(lp & 0xff);
  }
  static __device__ __forceinline__ f4 mfma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c, 0, 0, 0);
  }
};

// ---------------------------------------------------------------------------
// Tile rows per form (threads = 4 x rows: one wave per 16 rows).
template <class T>
constexpr int mx_rows() { return 128; }
template <>
constexpr int mx_rows<e4m3>() { return 64; }

// Per-call preparation: FP32 copy of L (A source) and the split B operand,
// all [rows_pad][ldl] with rows beyond n_aux_pad zero.  For FP16 and FP8 each
// column k carries the scale 2^e_k (max_P |L_Pk| 2^e_k in the form's target
// binade); A is formed with 2^-e_k.  For BF16 colscale is NULL (no scaling).
template <class T>
__global__ void mixed_prep_kernel(const double *__restrict__ Lp, int n_aux_pad, int rows_pad,
                                  int ldl, const float *__restrict__ colscale,
                                  float *__restrict__ Lf, typename Mix<T>::E *__restrict__ Bhi,
                                  typename Mix<T>::E *__restrict__ Blo) {
  const long long total = (long long)rows_pad * ldl;
  const long long valid = (long long)n_aux_pad * ldl;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(idx % ldl);
    const double v = idx < valid ? Lp[idx] : 0.0;
    Lf[idx] = (float)v;
    typename Mix<T>::E h, l;
    Mix<T>::split((float)(colscale ? v * (double)colscale[k] : v), h, l);
    Bhi[idx] = h;
    Blo[idx] = l;
  }
}

// Column scales: scale = 2^e_k with max_P |L_Pk| 2^e_k in [2^(target-1),
// 2^target), inv = 2^-e_k, acol = max_P |L_Pk| 2^-e_k (the largest |A| of
// column k per unit |chi|).  One thread per column.
__global__ void colscale_kernel(const double *__restrict__ Lp, int n_aux_pad, int ldl, int target,
                                float *__restrict__ scale, float *__restrict__ inv_scale,
                                float *__restrict__ acol) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ldl) return;
  double m = 0.0;
  for (int P = 0; P < n_aux_pad; ++P) m = fmax(m, fabs(Lp[(long long)P * ldl + k]));
  int e = 0;
  if (m > 0.0) {
    int ex;
    frexp(m, &ex);  // m = f 2^ex, f in [0.5, 1)
    e = target - ex;
  }
  scale[k] = ldexpf(1.0f, e);
  inv_scale[k] = ldexpf(1.0f, -e);
  acol[k] = (float)ldexp(m, -e);
}

// Per-frequency scale 2^g with max_k |chi_k| acol_k 2^g in [2^(target-1), 2^target).
__global__ void taskscale_kernel(const double *__restrict__ chi_re, const double *__restrict__ chi_im,
                                 int ldl, int target, const float *__restrict__ acol,
                                 float *__restrict__ tscale) {
  __shared__ double sh[256];
  const int f = blockIdx.x;
  double m = 0.0;
  for (int k = threadIdx.x; k < ldl; k += 256) {
    const double a = fmax(fabs(chi_re[(long long)f * ldl + k]), fabs(chi_im[(long long)f * ldl + k]));
    m = fmax(m, a * (double)acol[k]);
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int g = 0;
    if (sh[0] > 0.0) {
      int ex;
      frexp(sh[0], &ex);
      g = target - ex;
    }
    tscale[f] = ldexpf(1.0f, g);
  }
}

// Grid: (n_tiles, F).  Wave w: rows 32*(w/2) .. +32, columns (MX_TC/2)*(w%2)
// .. +MX_TC/2, i.e. 2 x MX_NB blocks of 16 x 16, Re and Im accumulators (FP32).
// MFMA layout (16x16x32): lane l supplies A[l%16][8(l/16)+e], B[8(l/16)+e][l%16];
// output element r of lane l is D[4(l/16)+r][l%16].
template <class T>
__global__ void __launch_bounds__(4 * mx_rows<T>(), 512 / (4 * mx_rows<T>()))
pi_build_mixed_kernel(const float *__restrict__ Lf, const typename Mix<T>::E *__restrict__ Bhi,
                      const typename Mix<T>::E *__restrict__ Blo, int ldl, int n_aux,
                      const double *__restrict__ chi_re, const double *__restrict__ chi_im,
                      const float *__restrict__ inv_colscale, const float *__restrict__ tscale,
                      const int2 *__restrict__ tiles, double2 *__restrict__ G, long long g_stride,
                      int ldg) {
  using E = typename Mix<T>::E;
  using V = typename Mix<T>::V;
  constexpr int EP = 16 / (int)sizeof(E);  // elements per 16-byte load
  // B rows padded by 16 bytes (rows stay 16-byte aligned)
  constexpr int KC = MX_KC, LA = KC + 4, LB = KC + EP;
  constexpr int TR = mx_rows<T>(), NT = 4 * TR;
  __shared__ float As[TR * LA];
  __shared__ E Bh[MX_TC * LB];
  __shared__ E Bl[MX_TC * LB];
  __shared__ float Cr[KC], Ci[KC];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int2 tb = tiles[blockIdx.x];
  const int P0 = tb.x * TR, Q0 = tb.y * MX_TC;
  const int f = blockIdx.y;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * (MX_TC / 2);
  const float gsc = tscale ? tscale[f] : 1.0f;

  f4 accr[2][MX_NB], acci[2][MX_NB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < MX_NB; ++b) {
      accr[a][b] = f4{0.f, 0.f, 0.f, 0.f};
      acci[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    }

  const double *cr_g = chi_re + (long long)f * ldl;
  const double *ci_g = chi_im + (long long)f * ldl;
  for (int kc = 0; kc < ldl; kc += KC) {
    // A source: TR rows x 32 floats (8 per thread as two float4)
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int idx = it * NT + tid;       // 0 .. 8 TR - 1
      const int row = idx >> 3, kq = (idx & 7) * 4;
      const float4 v = *reinterpret_cast<const float4 *>(Lf + (long long)(P0 + row) * ldl + kc + kq);
      float *dst = As + row * LA + kq;
      dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
    }
    // B: MX_TC rows x 32 elements, hi and lo (16 B per thread and pass)
#pragma unroll
    for (int it = 0; it < MX_TC * KC / (EP * NT); ++it) {
      const int idx = it * NT + tid;
      const int row = idx / (KC / EP), kq = (idx % (KC / EP)) * EP;
      const long long off = (long long)(Q0 + row) * ldl + kc + kq;
      const uint4 vh = *reinterpret_cast<const uint4 *>(Bhi + off);
      const uint4 vl = *reinterpret_cast<const uint4 *>(Blo + off);
      *reinterpret_cast<uint4 *>(Bh + row * LB + kq) = vh;
      *reinterpret_cast<uint4 *>(Bl + row * LB + kq) = vl;
    }
    if (tid < KC) {
      const float s = inv_colscale ? inv_colscale[kc + tid] : 1.0f;
      Cr[tid] = (float)cr_g[kc + tid] * s * gsc;
      Ci[tid] = (float)ci_g[kc + tid] * s * gsc;
    }
    __syncthreads();

    // A operands: this wave's two row blocks, Re and Im, split hi/lo
    V arh[2], arl[2], aih[2], ail[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const float *src = As + (wr + 16 * a + li) * LA + 8 * lq;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float lv = src[e];
        E h, l;
        Mix<T>::split(lv * Cr[8 * lq + e], h, l);
        arh[a][e] = h;
        arl[a][e] = l;
        Mix<T>::split(lv * Ci[8 * lq + e], h, l);
        aih[a][e] = h;
        ail[a][e] = l;
      }
    }
#pragma unroll
    for (int b = 0; b < MX_NB; ++b) {
      const int col = wc + 16 * b + li;
      const V bh = *reinterpret_cast<const V *>(Bh + col * LB + 8 * lq);
      const V bl = *reinterpret_cast<const V *>(Bl + col * LB + 8 * lq);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        accr[a][b] = Mix<T>::mfma(arh[a], bh, accr[a][b]);
        accr[a][b] = Mix<T>::mfma(arh[a], bl, accr[a][b]);
        accr[a][b] = Mix<T>::mfma(arl[a], bh, accr[a][b]);
        acci[a][b] = Mix<T>::mfma(aih[a], bh, acci[a][b]);
        acci[a][b] = Mix<T>::mfma(aih[a], bl, acci[a][b]);
        acci[a][b] = Mix<T>::mfma(ail[a], bh, acci[a][b]);
      }
    }
    __syncthreads();
  }

  // upper triangle (col >= row) written with its mirror, as 1 - Pi
  const double unscale = 1.0 / (double)gsc;
  double2 *Gf = G + (long long)f * g_stride;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < MX_NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = P0 + wr + 16 * a + 4 * lq + r;
        const int col = Q0 + wc + 16 * b + li;
        if (row < n_aux && col < n_aux && col >= row) {
          const double pr = (double)accr[a][b][r] * unscale, pi = (double)acci[a][b][r] * unscale;
          const double2 v = make_double2((row == col ? 1.0 : 0.0) - pr, -pi);
          Gf[(long long)row * ldg + col] = v;
          if (col != row) Gf[(long long)col * ldg + row] = v;
        }
      }
}

// ---------------------------------------------------------------------------
void launch_mixed_prep(int prec, const double *Lp, int n_aux_pad, int rows_pad, int ldl, float *Lf,
                       void *Bhi, void *Blo, float *colscale, float *inv_colscale, float *acol,
                       hipStream_t stream) {
  long long blocks = ((long long)rows_pad * ldl + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (prec == 2) {
    colscale_kernel<<<(ldl + 255) / 256, 256, 0, stream>>>(Lp, n_aux_pad, ldl, Mix<_Float16>::TARGET,
                                                            colscale, inv_colscale, acol);
    mixed_prep_kernel<_Float16><<<(unsigned)blocks, 256, 0, stream>>>(
        Lp, n_aux_pad, rows_pad, ldl, colscale, Lf, static_cast<unsigned short *>(Bhi),
        static_cast<unsigned short *>(Blo));
  } else if (prec == 3) {
    colscale_kernel<<<(ldl + 255) / 256, 256, 0, stream>>>(Lp, n_aux_pad, ldl, Mix<e4m3>::TARGET,
                                                            colscale, inv_colscale, acol);
    mixed_prep_kernel<e4m3><<<(unsigned)blocks, 256, 0, stream>>>(
        Lp, n_aux_pad, rows_pad, ldl, colscale, Lf, static_cast<unsigned char *>(Bhi),
        static_cast<unsigned char *>(Blo));
  } else {
    mixed_prep_kernel<__bf16><<<(unsigned)blocks, 256, 0, stream>>>(
        Lp, n_aux_pad, rows_pad, ldl, nullptr, Lf, static_cast<unsigned short *>(Bhi),
        static_cast<unsigned short *>(Blo));
  }
}

void launch_pi_build_mixed(int prec, const float *Lf, const void *Bhi, const void *Blo, int ldl,
                           int n_aux, const double *chi_re, const double *chi_im,
                           const float *inv_colscale, const float *acol, float *tscale, int F,
                           const int2 *tiles, int n_tiles, double2 *G, long long g_stride, int ldg,
                           hipStream_t stream) {
  dim3 grid(n_tiles, F);
  if (prec == 2) {
    taskscale_kernel<<<F, 256, 0, stream>>>(chi_re, chi_im, ldl, Mix<_Float16>::TARGET, acol, tscale);
    pi_build_mixed_kernel<_Float16><<<grid, 4 * mx_rows<_Float16>(), 0, stream>>>(
        Lf, static_cast<const unsigned short *>(Bhi), static_cast<const unsigned short *>(Blo), ldl,
        n_aux, chi_re, chi_im, inv_colscale, tscale, tiles, G, g_stride, ldg);
  } else if (prec == 3) {
    taskscale_kernel<<<F, 256, 0, stream>>>(chi_re, chi_im, ldl, Mix<e4m3>::TARGET, acol, tscale);
    pi_build_mixed_kernel<e4m3><<<grid, 4 * mx_rows<e4m3>(), 0, stream>>>(
        Lf, static_cast<const unsigned char *>(Bhi), static_cast<const unsigned char *>(Blo), ldl,
        n_aux, chi_re, chi_im, inv_colscale, tscale, tiles, G, g_stride, ldg);
  } else {
    pi_build_mixed_kernel<__bf16><<<grid, 4 * mx_rows<__bf16>(), 0, stream>>>(
        Lf, static_cast<const unsigned short *>(Bhi), static_cast<const unsigned short *>(Blo), ldl,
        n_aux, chi_re, chi_im, nullptr, nullptr, tiles, G, g_stride, ldg);
  }
}

}  // namespace gwc
