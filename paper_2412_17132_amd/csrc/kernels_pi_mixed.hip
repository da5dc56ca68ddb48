// Mixed-precision polarisability: Pi(z) = L diag(chi(z)) L^T with 16-bit or
// 8-bit MFMA inputs and FP32 accumulation (precision form of the Pi build).
//
// Each operand x is split into two values of the form's type, x ~ hi + lo
// with hi = round(x), lo = round(x - hi), and the product is formed from three
// MFMA passes, hi*hi + hi*lo + lo*hi (the lo*lo term, relative size 2^-2p, is
// dropped).  B = L is split once per call; the A operand L_Pk chi_k is formed
// per frequency in FP32 from a copy of L (FP32; FP16 with the column scales
// applied for FP8) and FP32-rounded chi (chi itself is computed in FP64) and
// split in registers.
//
//   BF16X3: bf16 (8-bit significand) -> ~2^-16 relative per product
//   FP16X3: fp16 (11-bit significand) with power-of-two scaling: columns of B
//           are scaled by 2^e_k (undone in A), and each frequency's A operand
//           by 2^g_f (undone on the FP32 result), keeping hi and lo parts in the
//           fp16 normal range -> ~2^-22 relative per product
//   FP8X3:  fp8 e4m3 (4-bit significand, largest 448) with the same scaling
//           aimed one binade higher -> ~2^-7 relative per product
//
// Tile: one 128 x 256 block of Pi per workgroup and frequency (8 waves of
// 16 x 256, v_mfma_f32_16x16x32_{bf16,f16} or, for FP8, two K chunks per
// v_mfma_f32_16x16x128_f8f6f4; every B chunk staged in LDS serves 128 rows);
// upper-triangle blocks only, the result written as 1 - Pi (FP64) into the
// bordered matrix with its mirror.
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
constexpr int MX_KSTEP = 32;  // K of one MFMA step (chi is laid out per step)
typedef float f8v __attribute__((ext_vector_type(8)));

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
  // (products: mix_mfma128, two K chunks at a time)
};

// ---------------------------------------------------------------------------
// K per chunk of the Pi build: one MFMA K step (32) for the 16-bit forms, two
// for FP8, so that a lane's 16-byte load holds 8 one-byte values of each step.
// FP8 takes its chunks in pairs (one K = 128 product per pair), so its
// operands span a whole number of pairs (KPAD columns).
template <class T>
struct MixK {
  static constexpr int KC = 32, STEPS = 1, KPAD = 32;
};
template <>
struct MixK<e4m3> {
  static constexpr int KC = 64, STEPS = 2, KPAD = 128;
};

// Source of the A operand L chi: FP32 L for the 16-bit forms (their split
// keeps about 16 or 22 bits of A); for FP8, whose split keeps about 8, FP16
// L with the column scales 2^e_k applied (the largest |value| of a column in
// [2^7, 2^8), so that 11 significant bits hold down to 2^-21 of it), half the
// bytes per chunk.  AP: 1 KB pieces per 16-row block and chunk.
template <class T>
struct MixA {
  using E = float;
  static constexpr int AP = 2 * MixK<T>::STEPS;
};
template <>
struct MixA<e4m3> {
  using E = _Float16;
  static constexpr int AP = MixK<e4m3>::STEPS;
};

// Per-call preparation: FP32 copy of L (A source) and the split B operand,
// rows beyond n_aux_pad and columns beyond ldl zero (the operands span ldlk
// columns, a multiple of the form's chunk).  For FP16 and FP8 each column k
// carries the scale 2^e_k (max_P |L_Pk| 2^e_k in the form's target binade);
// A is formed with 2^-e_k.  For BF16 colscale is NULL (no scaling).
//
// Both are stored in MFMA operand-fragment order, so that the Pi build
// fetches each 1 KB piece of a tile with one fully contiguous 16-byte-per-lane
// load and finds it in the order its products read it: per 16-row block rb
// and K chunk c (nch chunks of KC), with step s = (k mod KC) / 32 and
// q = k mod 32,
//   B: 64 lanes x 16 bytes; lane li + 16 (q / 8) holds row 16 rb + li, as
//      element 8 s + q mod 8 of its 16 bytes;
//   A (FP32): 2 STEPS pieces of 64 lanes x 4 floats; lane li + 16 (q / 8) of
//      piece 2 s + (q mod 8) / 4 holds row 16 rb + li, as float q mod 4;
//   A (FP16, FP8 form): STEPS pieces of 64 lanes x 8 halves; lane
//      li + 16 (q / 8) of piece s holds row 16 rb + li, as half q mod 8.
template <class T>
__device__ __forceinline__ long long mix_frag_b(int r, int k, int nch) {
  constexpr int KC = MixK<T>::KC, EPL = 16 / (int)sizeof(typename Mix<T>::E);
  const int rb = r >> 4, li = r & 15, c = k / KC, kk = k % KC, st = kk >> 5, q = kk & 31;
  return (((long long)rb * nch + c) * 64 + li + 16 * (q >> 3)) * EPL + 8 * st + (q & 7);
}
template <class T>
__device__ __forceinline__ long long mix_frag_a(int r, int k, int nch) {
  constexpr int KC = MixK<T>::KC, AP = MixA<T>::AP;
  const int rb = r >> 4, li = r & 15, c = k / KC, kk = k % KC, st = kk >> 5, q = kk & 31;
  if constexpr (sizeof(typename MixA<T>::E) == 2)
    return ((((long long)rb * nch + c) * AP + st) * 64 + li + 16 * (q >> 3)) * 8 + (q & 7);
  else
    return ((((long long)rb * nch + c) * AP + 2 * st + ((q >> 2) & 1)) * 64 + li + 16 * (q >> 3)) * 4 +
           (q & 3);
}

template <class T>
__global__ void mixed_prep_kernel(const double *__restrict__ Lp, int n_aux_pad, int rows_pad,
                                  int ldl, int ldlk, const float *__restrict__ colscale,
                                  typename MixA<T>::E *__restrict__ Lf,
                                  typename Mix<T>::E *__restrict__ Bhi,
                                  typename Mix<T>::E *__restrict__ Blo) {
  const long long total = (long long)rows_pad * ldlk;
  const int nch = ldlk / MixK<T>::KC;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / ldlk), k = (int)(idx % ldlk);
    const bool in = r < n_aux_pad && k < ldl;
    const double v = in ? Lp[(long long)r * ldl + k] : 0.0;
    const double vs = colscale && in ? v * (double)colscale[k] : v;
    if constexpr (sizeof(typename MixA<T>::E) == 2)
      Lf[mix_frag_a<T>(r, k, nch)] = (typename MixA<T>::E)(float)vs;  // the scaled value
    else
      Lf[mix_frag_a<T>(r, k, nch)] = (float)v;
    typename Mix<T>::E h, l;
    Mix<T>::split((float)vs, h, l);
    const long long ib = mix_frag_b<T>(r, k, nch);
    Bhi[ib] = h;
    Blo[ib] = l;
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

// Per-frequency FP32 chi with the column scales 2^-e_k and the frequency scale
// 2^g folded in (the same float operations as the A operand needs), per K
// chunk of 32 the 32 Re values then the 32 Im values: cf[f][k / 32][2][32].
// With an A source that already carries 2^e_k (FP8), the column factor is
// 2^-2 e_k, so that A = L chi 2^-e_k 2^g either way.
__global__ void __launch_bounds__(256)
mixed_chi_kernel(const double *__restrict__ chi_re, const double *__restrict__ chi_im, int ldl,
                 const float *__restrict__ inv_colscale, int scaled_source,
                 const float *__restrict__ tscale, float *__restrict__ cf) {
  const int k = blockIdx.x * 256 + threadIdx.x, f = blockIdx.y;
  if (k >= ldl) return;
  float s = inv_colscale ? inv_colscale[k] : 1.0f;
  if (scaled_source) s *= s;
  const float g = tscale ? tscale[f] : 1.0f;
  float *o = cf + (long long)f * 2 * ldl + (k / MX_KSTEP) * 2 * MX_KSTEP + k % MX_KSTEP;
  o[0] = (float)chi_re[(long long)f * ldl + k] * s * g;
  o[MX_KSTEP] = (float)chi_im[(long long)f * ldl + k] * s * g;
}

// The Pi build of every mixed form, with the K chunks in a four-stage LDS
// ring and one barrier per two chunks.  One workgroup of 8 waves per
// 128 x 256 tile and frequency; wave w covers rows 16 w and all 256 columns:
// 16 blocks of 16 x 16, Re and Im accumulators.  Each K chunk (32 for the
// 16-bit forms, 64 for FP8) is fetched two chunks ahead of its multiply: per
// wave two 1 KB pieces of each split B operand (hi, lo) straight into LDS
// (buffer_load ... lds, 16 bytes per lane at piece base + 16 lane: no
// registers, no padding) with the chunk's FP32 chi, and the wave's own A rows
// into registers, all in operand-fragment order.  The stages are separate
// __shared__ objects and the loop is unrolled by four, so each multiply names
// its stages and each fetch others, and the compiler inserts no waits between
// them.
// Raw buffer resources (base, no stride, size in bytes; the gfx9 format word):
// the hardware returns zeros past the size instead of faulting.
constexpr int BUF_FORMAT_WORD = 0x00020000;

// The A rows of one chunk for one lane: 8 values per MFMA K step (FP32, or
// FP16 for the FP8 form).
template <class T>
struct MixAReg {
  f8v v[MixK<T>::STEPS];
};
template <>
struct MixAReg<e4m3> {
  h8 v[MixK<e4m3>::STEPS];
};

// The loads of one K chunk (columns kc .. kc + KC), issued in three parts
// spread over the products of the chunk before (a burst of all of them at
// once holds the waves at the memory issue queue while the MFMA pipes idle).
// The chunk offset goes into the per-lane offset, which the hardware checks
// against the buffer's size (a load past it reads zeros), not into the scalar
// offset.
template <class T>
struct MixFetch {
  using E = typename Mix<T>::E;
  static constexpr int KC = MixK<T>::KC, AP = MixA<T>::AP;
  static constexpr int LOADS = 1 + AP + 4;  // loads of one fetch per wave
  static constexpr int A_CHUNK = AP * 1024 / KC;  // A bytes per K column of a 16-row block
  __amdgpu_buffer_rsrc_t rA, rBh, rBl, rC;
  int voA[AP], voB[2], wave, lane;

  // part 0: the chunk's chi (2 KC floats) into the stage's 1 KB of C, by every
  // wave (the same bytes, so that each wave's own wait covers them; the lanes
  // past the chunk read what follows, or zeros: unused), and the wave's own A
  // rows straight into registers (its lane's 8 floats per K step)
  __device__ __forceinline__ void part0(MixAReg<T> &areg, float *C, int kc) const {
    typedef float f4v __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rC, C, 16, 16 * lane + kc * 8, 0, 0, 0);
#pragma unroll
    for (int st = 0; st < MixK<T>::STEPS; ++st) {
      if constexpr (sizeof(typename MixA<T>::E) == 2) {
        areg.v[st] = __builtin_bit_cast(h8, __builtin_amdgcn_raw_buffer_load_b128(rA, voA[st] + kc * A_CHUNK, 0, 0));
      } else {
        const f4v a0 = __builtin_bit_cast(
            f4v, __builtin_amdgcn_raw_buffer_load_b128(rA, voA[2 * st] + kc * A_CHUNK, 0, 0));
        const f4v a1 = __builtin_bit_cast(
            f4v, __builtin_amdgcn_raw_buffer_load_b128(rA, voA[2 * st + 1] + kc * A_CHUNK, 0, 0));
        areg.v[st] = f8v{a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
      }
    }
  }
  // parts 1 and 2: the wave's B pieces 2 wave + j (hi and lo) into the stage
  __device__ __forceinline__ void partB(int j, E *Bh, E *Bl, int kc) const {
    constexpr int PIECE = 1024 / (int)sizeof(E);  // elements of a 1 KB piece
    const int q = 2 * wave + j;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rBh, Bh + PIECE * q, 16, voB[j] + kc * (1024 / KC), 0, 0, 0);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rBl, Bl + PIECE * q, 16, voB[j] + kc * (1024 / KC), 0, 0, 0);
  }
  __device__ __forceinline__ void all(MixAReg<T> &areg, E *Bh, E *Bl, float *C, int kc) const {
    part0(areg, C, kc);
    partB(0, Bh, Bl, kc);
    partB(1, Bh, Bl, kc);
  }
};

// Waits until at most one fetch (its LOADS loads) of this wave is in flight:
// s_waitcnt vmcnt(LOADS), the other counters unconstrained (expcnt 7,
// lgkmcnt 15).
template <class T>
__device__ __forceinline__ void mix_wait_one_fetch() {
  static_assert(MixFetch<T>::LOADS < 16, "vmcnt's low field holds 0 .. 15");
  __builtin_amdgcn_s_waitcnt(0x0F70 | MixFetch<T>::LOADS);
}

// The workgroup barrier of the K loop, without the memory fence that
// __syncthreads adds: that fence waits for every load of the wave, the
// fetch still in flight included.  The empty asm statements keep the
// compiler from moving LDS accesses across the barrier; each wave has
// already waited for its own part of the chunk (mix_wait_one_fetch), and its
// LDS reads of the chunk before were consumed by its products.
__device__ __forceinline__ void mix_barrier() {
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// x = hi + lo for 8 values at once (vector conversions, round to nearest
// even, packed in pairs by the hardware): the same values as Mix<T>::split.
__device__ __forceinline__ f8v ld8(const float *p) {
  const float4 a = reinterpret_cast<const float4 *>(p)[0];
  const float4 b = reinterpret_cast<const float4 *>(p)[1];
  return f8v{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

template <class T>
__device__ __forceinline__ void split8(f8v x, typename Mix<T>::V &hi, typename Mix<T>::V &lo) {
  typedef T t8 __attribute__((ext_vector_type(8)));
  const t8 h = __builtin_convertvector(x, t8);
  const f8v r = x - __builtin_convertvector(h, f8v);
  hi = __builtin_bit_cast(us8, h);
  lo = __builtin_bit_cast(us8, __builtin_convertvector(r, t8));
}
// bf16: hi back in FP32 straight from its packed bits (a bf16 is the top half
// of an FP32), instead of converting each value again
template <>
__device__ __forceinline__ void split8<__bf16>(f8v x, us8 &hi, us8 &lo) {
  typedef __bf16 t8 __attribute__((ext_vector_type(8)));
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const t8 h = __builtin_convertvector(x, t8);
  const u4 p = __builtin_bit_cast(u4, h);  // element 2 i in the low half of word i
  const u4 e = p << 16, o = p & 0xFFFF0000u;
  // (subscripts: .y/.z/.w inside __builtin_bit_cast were seen to read lane 0)
  const f8v hf = f8v{__builtin_bit_cast(float, (unsigned)e[0]), __builtin_bit_cast(float, (unsigned)o[0]),
                     __builtin_bit_cast(float, (unsigned)e[1]), __builtin_bit_cast(float, (unsigned)o[1]),
                     __builtin_bit_cast(float, (unsigned)e[2]), __builtin_bit_cast(float, (unsigned)o[2]),
                     __builtin_bit_cast(float, (unsigned)e[3]), __builtin_bit_cast(float, (unsigned)o[3])};
  hi = __builtin_bit_cast(us8, h);
  lo = __builtin_bit_cast(us8, __builtin_convertvector(x - hf, t8));
}
// e4m3: pairs converted into the halves of a word (round to nearest even, the
// same conversions as Mix<e4m3>::split), hi read back per pair
template <>
__device__ __forceinline__ void split8<e4m3>(f8v x, uc8 &hi, uc8 &lo) {
  typedef int i2 __attribute__((ext_vector_type(2)));
  int h0 = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
  h0 = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], h0, true);
  int h1 = __builtin_amdgcn_cvt_pk_fp8_f32(x[4], x[5], 0, false);
  h1 = __builtin_amdgcn_cvt_pk_fp8_f32(x[6], x[7], h1, true);
  typedef float f2 __attribute__((ext_vector_type(2)));
  // hi back in FP32 two values per conversion (the low, then the high word)
  const f2 p0 = __builtin_amdgcn_cvt_pk_f32_fp8(h0, false), p1 = __builtin_amdgcn_cvt_pk_f32_fp8(h0, true);
  const f2 p2 = __builtin_amdgcn_cvt_pk_f32_fp8(h1, false), p3 = __builtin_amdgcn_cvt_pk_f32_fp8(h1, true);
  const f8v hf = f8v{p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
  const f8v r = x - hf;
  int l0 = __builtin_amdgcn_cvt_pk_fp8_f32(r[0], r[1], 0, false);
  l0 = __builtin_amdgcn_cvt_pk_fp8_f32(r[2], r[3], l0, true);
  int l1 = __builtin_amdgcn_cvt_pk_fp8_f32(r[4], r[5], 0, false);
  l1 = __builtin_amdgcn_cvt_pk_fp8_f32(r[6], r[7], l1, true);
  hi = __builtin_bit_cast(uc8, i2{h0, h1});
  lo = __builtin_bit_cast(uc8, i2{l0, l1});
}

// A lane's 16 bytes of a B piece as the operand of K step st.
template <class T>
__device__ __forceinline__ typename Mix<T>::V mix_bstep(const uint4 &w, int st) {
  if constexpr (sizeof(typename Mix<T>::E) == 2) {
    return __builtin_bit_cast(typename Mix<T>::V, w);
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(typename Mix<T>::V, st == 0 ? u2{w.x, w.y} : u2{w.z, w.w});
  }
}

// Column blocks per skip group of the 16-bit forms.
constexpr int MX_BGROUP = 4;

// One wave's 16 rows against the 16 column blocks of a stage, in groups of
// MX_BGROUP blocks: a group is skipped when none of its blocks is in [b0, b1)
// (wave-uniform bounds: blocks wholly below the diagonal or past n_aux produce
// nothing that is stored, and the two waves of a SIMD share its MFMA pipe, so
// skipping them shortens the tiles that cross the diagonal).
template <class T>
__device__ __forceinline__ void mix_multiply(const MixAReg<T> &lv, const typename Mix<T>::E *Bh,
                                             const typename Mix<T>::E *Bl, const float *C, int lane,
                                             int lq, int b0, int b1, f4 (&accr)[16], f4 (&acci)[16],
                                             const MixFetch<T> &fetch, MixAReg<T> &areg_next,
                                             typename Mix<T>::E *Bh_next, typename Mix<T>::E *Bl_next,
                                             float *C_next, int kc_next) {
  using E = typename Mix<T>::E;
  using V = typename Mix<T>::V;
  constexpr int STEPS = MixK<T>::STEPS, PIECE = 1024 / (int)sizeof(E), EPL = 16 / (int)sizeof(E);
  fetch.part0(areg_next, C_next, kc_next);
  V arh[STEPS], arl[STEPS], aih[STEPS], ail[STEPS];
#pragma unroll
  for (int st = 0; st < STEPS; ++st) {
    // 16-byte LDS reads only (a 32-byte read is split by the compiler into
    // accesses it cannot tell apart from the fetch into the other stage, and
    // it would then wait for that fetch); the chunk's chi is [K step][Re, Im][32]
    const f8v cr = ld8(C + 64 * st + 8 * lq), ci = ld8(C + 64 * st + 32 + 8 * lq);
    split8<T>(lv.v[st] * cr, arh[st], arl[st]);
    split8<T>(lv.v[st] * ci, aih[st], ail[st]);
  }
  const E *bh_p = Bh + EPL * lane;
  const E *bl_p = Bl + EPL * lane;
  // groups of NG column blocks: one uniform branch per group, and a group's
  // 2 NG LDS reads are issued together ahead of its products (2 NG
  // independent accumulator chains)
  constexpr int NG = MX_BGROUP, NGR = 16 / NG;
#pragma unroll
  for (int g = 0; g < NGR; ++g) {
    if (g == NGR / 4 || g == NGR / 2) fetch.partB(g == NGR / 4 ? 0 : 1, Bh_next, Bl_next, kc_next);
    if (NG * g + NG - 1 >= b0 && NG * g < b1) {
      uint4 bh[NG], bl[NG];
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        bh[j] = *reinterpret_cast<const uint4 *>(bh_p + PIECE * (NG * g + j));
        bl[j] = *reinterpret_cast<const uint4 *>(bl_p + PIECE * (NG * g + j));
      }
#pragma unroll
      for (int st = 0; st < STEPS; ++st) {
#pragma unroll
        for (int j = 0; j < NG; ++j) {
          const V h = mix_bstep<T>(bh[j], st);
          accr[NG * g + j] = Mix<T>::mfma(arh[st], h, accr[NG * g + j]);
          acci[NG * g + j] = Mix<T>::mfma(aih[st], h, acci[NG * g + j]);
        }
#pragma unroll
        for (int j = 0; j < NG; ++j) {
          const V h = mix_bstep<T>(bh[j], st);
          accr[NG * g + j] = Mix<T>::mfma(arl[st], h, accr[NG * g + j]);
          acci[NG * g + j] = Mix<T>::mfma(ail[st], h, acci[NG * g + j]);
        }
#pragma unroll
        for (int j = 0; j < NG; ++j) {
          const V l = mix_bstep<T>(bl[j], st);
          accr[NG * g + j] = Mix<T>::mfma(arh[st], l, accr[NG * g + j]);
          acci[NG * g + j] = Mix<T>::mfma(aih[st], l, acci[NG * g + j]);
        }
      }
    }
  }
}

// FP8: two K chunks (a, b) at once, each lane's 32 bytes of A and of B being
// chunk a's 16 then chunk b's 16, so that one v_mfma_f32_16x16x128_f8f6f4
// (E4M3 operands, no block scales) replaces four K = 32 products; it issues
// at twice the rate of the K = 32 FP8 form.  A lane's 16 bytes of a chunk
// hold the same 16 K indices in A (8 per step, split from its FP32 rows) as
// in B (the fragment order above), and the instruction pairs byte i of an A
// lane with byte i of the B lane of the same K group, so the 128-term sums
// are the chunks' dot products.  Column blocks in groups of two (the K = 128
// operands take twice the registers of the K = 64 ones).
typedef int i8v __attribute__((ext_vector_type(8)));
__device__ __forceinline__ i8v mix_cat(uc8 a0, uc8 a1, uc8 b0, uc8 b1) {
  typedef int i2 __attribute__((ext_vector_type(2)));
  const i2 w = __builtin_bit_cast(i2, a0), x = __builtin_bit_cast(i2, a1);
  const i2 y = __builtin_bit_cast(i2, b0), z = __builtin_bit_cast(i2, b1);
  return i8v{w[0], w[1], x[0], x[1], y[0], y[1], z[0], z[1]};
}
__device__ __forceinline__ i8v mix_cat(const uint4 &a, const uint4 &b) {
  return i8v{(int)a.x, (int)a.y, (int)a.z, (int)a.w, (int)b.x, (int)b.y, (int)b.z, (int)b.w};
}
__device__ __forceinline__ f4 mix_mfma128(const i8v &a, const i8v &b, f4 c) {
  // format 0 (E4M3) for both operands; zero scale operands select the
  // unscaled instruction
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

__device__ __forceinline__ void mix_multiply_pair(
    const MixAReg<e4m3> &la, const MixAReg<e4m3> &lb, const unsigned char *Bh_a,
    const unsigned char *Bl_a, const float *C_a, const unsigned char *Bh_b, const unsigned char *Bl_b,
    const float *C_b, int lane, int lq, int b0, int b1, f4 (&accr)[16], f4 (&acci)[16],
    const MixFetch<e4m3> &fetch, MixAReg<e4m3> &an_a, MixAReg<e4m3> &an_b, unsigned char *Bhn_a,
    unsigned char *Bln_a, float *Cn_a, unsigned char *Bhn_b, unsigned char *Bln_b, float *Cn_b,
    int kc_next) {
  constexpr int KC = MixK<e4m3>::KC;
  fetch.part0(an_a, Cn_a, kc_next);
  fetch.part0(an_b, Cn_b, kc_next + KC);
  uc8 rh[4], rl[4], ih[4], il[4];  // [chunk a step 0, a 1, b 0, b 1]
#pragma unroll
  for (int st = 0; st < 2; ++st) {
    const f8v xa = __builtin_convertvector(la.v[st], f8v), xb = __builtin_convertvector(lb.v[st], f8v);
    split8<e4m3>(xa * ld8(C_a + 64 * st + 8 * lq), rh[st], rl[st]);
    split8<e4m3>(xa * ld8(C_a + 64 * st + 32 + 8 * lq), ih[st], il[st]);
    split8<e4m3>(xb * ld8(C_b + 64 * st + 8 * lq), rh[2 + st], rl[2 + st]);
    split8<e4m3>(xb * ld8(C_b + 64 * st + 32 + 8 * lq), ih[2 + st], il[2 + st]);
  }
  const i8v AH = mix_cat(rh[0], rh[1], rh[2], rh[3]), AL = mix_cat(rl[0], rl[1], rl[2], rl[3]);
  const i8v IH = mix_cat(ih[0], ih[1], ih[2], ih[3]), IL = mix_cat(il[0], il[1], il[2], il[3]);
  const int lo = 16 * lane;
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    if (g == 1) fetch.partB(0, Bhn_a, Bln_a, kc_next);
    if (g == 2) fetch.partB(1, Bhn_a, Bln_a, kc_next);
    if (g == 3) fetch.partB(0, Bhn_b, Bln_b, kc_next + KC);
    if (g == 4) fetch.partB(1, Bhn_b, Bln_b, kc_next + KC);
    if (2 * g + 1 >= b0 && 2 * g < b1) {
      i8v bh[2], bl[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int o = 1024 * (2 * g + j) + lo;
        bh[j] = mix_cat(*reinterpret_cast<const uint4 *>(Bh_a + o), *reinterpret_cast<const uint4 *>(Bh_b + o));
        bl[j] = mix_cat(*reinterpret_cast<const uint4 *>(Bl_a + o), *reinterpret_cast<const uint4 *>(Bl_b + o));
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        accr[2 * g + j] = mix_mfma128(AH, bh[j], accr[2 * g + j]);
        acci[2 * g + j] = mix_mfma128(IH, bh[j], acci[2 * g + j]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        accr[2 * g + j] = mix_mfma128(AL, bh[j], accr[2 * g + j]);
        acci[2 * g + j] = mix_mfma128(IL, bh[j], acci[2 * g + j]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        accr[2 * g + j] = mix_mfma128(AH, bl[j], accr[2 * g + j]);
        acci[2 * g + j] = mix_mfma128(IH, bl[j], acci[2 * g + j]);
      }
    }
  }
}

// Workgroup -> (tile, frequency) so that the workgroups one XCD holds at a
// time share a tile: workgroups are dispatched round-robin over the 8 XCDs,
// and each XCD's consecutive workgroups take one tile for `group` consecutive
// frequencies (group = 32, one per CU of the XCD, or F when smaller).  They
// then read the same A and B rows chunk by chunk, from the XCD's L2.  Blocks
// of (tile, frequency group) go to the XCDs in turn, so that each XCD gets a
// mix of diagonal and full tiles.
constexpr int MX_NXCD = 8;
__device__ __forceinline__ bool mx_item(int wg, int n_tiles, int F, int group, int &tile, int &f) {
  const int x = wg % MX_NXCD, j = wg / MX_NXCD;
  const int blk = (j / group) * MX_NXCD + x;
  const int g = blk / n_tiles;
  tile = blk - g * n_tiles;
  f = g * group + j % group;
  return g * group < F && f < F;
}

template <class T>
__global__ void __launch_bounds__(512, 1)
pi_build_mixed_async_kernel(const typename MixA<T>::E *__restrict__ Lf,
                            const typename Mix<T>::E *__restrict__ Bhi,
                            const typename Mix<T>::E *__restrict__ Blo, int ldl, int n_aux,
                            const float *__restrict__ cf_all, const float *__restrict__ tscale,
                            const int2 *__restrict__ tiles, int n_tiles, int F, int group,
                            double2 *__restrict__ G, long long g_stride, int ldg) {
  using E = typename Mix<T>::E;
  constexpr int KC = MixK<T>::KC, AP = MixA<T>::AP;
  // four stages as separate objects (the compiler then needs no wait between
  // a fetch into one and the reads of another); a stage's B pieces are 16 KB
  // of each split part in every form
  struct Stage {
    E Bh[MX_TC * KC], Bl[MX_TC * KC];
    float C[256];
  };
  __shared__ Stage S0, S1, S2, S3;
  MixAReg<T> R0, R1, R2, R3;  // the A rows of the chunk in each stage (registers)
  // the wave index is uniform: in a scalar register, the LDS bases of the
  // fetches can go to M0
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lq = lane >> 4;
  int tile, f;
  if (!mx_item(blockIdx.x, n_tiles, F, group, tile, f)) return;  // uniform: the whole workgroup
  const int2 tb = tiles[tile];
  const int P0 = tb.x * 128, Q0 = tb.y * MX_TC;
  const int wr = 16 * wave;
  const float *cf = cf_all + (long long)f * 2 * ldl;
  // column blocks this wave needs: some column >= its first row, and < n_aux;
  // none when its rows are all padding
  const int r_first = P0 + wr;
  int b0 = (r_first - Q0 - 15 + 15) / 16;  // ceil((r_first - Q0 - 15) / 16) for r_first >= Q0
  if (r_first - Q0 - 15 <= 0) b0 = 0;
  const int b1 = r_first < n_aux ? min(16, (n_aux - Q0 + 15) / 16) : 0;
  // This tile's operands in fragment order (mixed_prep_kernel): A from row
  // block P0 / 16 on (8 blocks of AP 1 KB pieces per chunk), B from row block
  // Q0 / 16 on (16 blocks of one 1 KB piece per chunk), as buffer resources.
  // Wave w fetches A block w (its own 16 rows) and B blocks 2 w, 2 w + 1; lane
  // l of a piece loads its bytes 16 l .. 16 l + 15 and lands at 16 l of the
  // piece in LDS, where the products' lane l reads them (consecutive lanes,
  // consecutive bytes: coalesced, and no LDS bank conflicts).
  constexpr int KPAD = MixK<T>::KPAD;
  const int nch = (ldl + KPAD - 1) / KPAD * (KPAD / KC);  // the operands span nch KC columns
  constexpr int PIECE = 1024 / (int)sizeof(E);
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(reinterpret_cast<const char *>(Lf) + (long long)(P0 / 16) * nch * AP * 1024), 0,
      8 * nch * AP * 1024, BUF_FORMAT_WORD);
  const __amdgpu_buffer_rsrc_t rBh = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(Bhi + (long long)(Q0 / 16) * nch * PIECE), 0, 16 * nch * 1024, BUF_FORMAT_WORD);
  const __amdgpu_buffer_rsrc_t rBl = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(Blo + (long long)(Q0 / 16) * nch * PIECE), 0, 16 * nch * 1024, BUF_FORMAT_WORD);
  const __amdgpu_buffer_rsrc_t rC = __builtin_amdgcn_make_buffer_rsrc((void *)cf, 0, 2 * ldl * 4,
                                                                      BUF_FORMAT_WORD);
  MixFetch<T> fetch;
  fetch.rA = rA;
  fetch.rBh = rBh;
  fetch.rBl = rBl;
  fetch.rC = rC;
  fetch.wave = wave;
  fetch.lane = lane;
#pragma unroll
  for (int j = 0; j < AP; ++j) fetch.voA[j] = (wave * nch * AP + j) * 1024 + 16 * lane;
#pragma unroll
  for (int j = 0; j < 2; ++j) fetch.voB[j] = (2 * wave + j) * nch * 1024 + 16 * lane;

  f4 accr[16], acci[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    accr[b] = f4{0.f, 0.f, 0.f, 0.f};
    acci[b] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // Four stages, two chunks per barrier: chunk c is in stage c % 4.  A
  // double step waits for all of this wave's loads (chunks c and c + 1),
  // meets the other waves at the barrier (every wave's part of both has
  // landed, and every wave has multiplied chunks c - 2 and c - 1, so their
  // stages are free) and multiplies c and c + 1, issuing the fetches of
  // c + 2 and c + 3 into those stages between their column groups.  Every
  // step fetches (the compiler then tells the stages apart and adds no waits
  // of its own): the fetches past the last chunk read the rows' next bytes or
  // zeros into stages that are not multiplied.
#define MX_MUL(S, R, N, RN, kn, bend) \
  mix_multiply<T>(R, S.Bh, S.Bl, S.C, lane, lq, b0, bend, accr, acci, fetch, RN, N.Bh, N.Bl, N.C, kn)
  fetch.all(R0, S0.Bh, S0.Bl, S0.C, 0);
  fetch.all(R1, S1.Bh, S1.Bl, S1.C, KC);
#define MX_MUL2(SA, SB, RA, RB, NA, NB, RNA, RNB, kn, bend)                                     \
  mix_multiply_pair(RA, RB, SA.Bh, SA.Bl, SA.C, SB.Bh, SB.Bl, SB.C, lane, lq, b0, bend, accr, acci, \
                    fetch, RNA, RNB, NA.Bh, NA.Bl, NA.C, NB.Bh, NB.Bl, NB.C, kn)
  for (int c = 0; c < nch; c += 4) {
    // a step past the last chunk multiplies nothing (no column block below
    // 0) but still fetches, so that no fetch sits in a branch
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's chunks c, c + 1
    mix_barrier();
    if constexpr (MixK<T>::KPAD == 2 * KC) {  // FP8: nch is even, a pair at a time
      MX_MUL2(S0, S1, R0, R1, S2, S3, R2, R3, (c + 2) * KC, b1);
    } else {
      MX_MUL(S0, R0, S2, R2, (c + 2) * KC, b1);
      MX_MUL(S1, R1, S3, R3, (c + 3) * KC, c + 1 < nch ? b1 : 0);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);
    mix_barrier();
    if constexpr (MixK<T>::KPAD == 2 * KC) {
      MX_MUL2(S2, S3, R2, R3, S0, S1, R0, R1, (c + 4) * KC, c + 2 < nch ? b1 : 0);
    } else {
      MX_MUL(S2, R2, S0, R0, (c + 4) * KC, c + 2 < nch ? b1 : 0);
      MX_MUL(S3, R3, S1, R1, (c + 5) * KC, c + 3 < nch ? b1 : 0);
    }
  }
#undef MX_MUL2
  __builtin_amdgcn_s_waitcnt(0);  // no fetch lands after the workgroup's end
#undef MX_MUL

  // upper triangle (col >= row) written with its mirror, as 1 - Pi
  const double unscale = 1.0 / (double)(tscale ? tscale[f] : 1.0f);
  double2 *Gf = G + (long long)f * g_stride;
#pragma unroll
  for (int b = 0; b < 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = P0 + wr + 4 * lq + r;
      const int col = Q0 + 16 * b + li;
      if (row < n_aux && col < n_aux && col >= row) {
        const double pr = (double)accr[b][r] * unscale, pi = (double)acci[b][r] * unscale;
        const double2 v = make_double2((row == col ? 1.0 : 0.0) - pr, -pi);
        Gf[(long long)row * ldg + col] = v;
        if (col != row) Gf[(long long)col * ldg + row] = v;
      }
    }
}

// ---------------------------------------------------------------------------
void launch_mixed_prep(int prec, const double *Lp, int n_aux_pad, int rows_pad, int ldl, int ldlk,
                       void *Lf, void *Bhi, void *Blo, float *colscale, float *inv_colscale,
                       float *acol, hipStream_t stream) {
  long long blocks = ((long long)rows_pad * ldlk + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (prec == 2) {
    colscale_kernel<<<(ldl + 255) / 256, 256, 0, stream>>>(Lp, n_aux_pad, ldl, Mix<_Float16>::TARGET,
                                                            colscale, inv_colscale, acol);
    mixed_prep_kernel<_Float16><<<(unsigned)blocks, 256, 0, stream>>>(
        Lp, n_aux_pad, rows_pad, ldl, ldlk, colscale, static_cast<float *>(Lf),
        static_cast<unsigned short *>(Bhi), static_cast<unsigned short *>(Blo));
  } else if (prec == 3) {
    colscale_kernel<<<(ldl + 255) / 256, 256, 0, stream>>>(Lp, n_aux_pad, ldl, Mix<e4m3>::TARGET,
                                                            colscale, inv_colscale, acol);
    mixed_prep_kernel<e4m3><<<(unsigned)blocks, 256, 0, stream>>>(
        Lp, n_aux_pad, rows_pad, ldl, ldlk, colscale, static_cast<_Float16 *>(Lf),
        static_cast<unsigned char *>(Bhi), static_cast<unsigned char *>(Blo));
  } else {
    mixed_prep_kernel<__bf16><<<(unsigned)blocks, 256, 0, stream>>>(
        Lp, n_aux_pad, rows_pad, ldl, ldlk, nullptr, static_cast<float *>(Lf),
        static_cast<unsigned short *>(Bhi), static_cast<unsigned short *>(Blo));
  }
}

void launch_pi_build_mixed(int prec, const void *Lf, const void *Bhi, const void *Blo, int ldl,
                           int n_aux, const double *chi_re, const double *chi_im,
                           const float *inv_colscale, const float *acol, float *tscale, float *chi_f32,
                           int F, const int2 *tiles, int n_tiles, double2 *G, long long g_stride,
                           int ldg, hipStream_t stream) {
  // FP16 and FP8 scale each frequency's A operand by a power of two (undone on
  // the result) and fold the column scales into chi; BF16 needs neither
  const bool scaled = prec == 2 || prec == 3;
  if (scaled)
    taskscale_kernel<<<F, 256, 0, stream>>>(chi_re, chi_im, ldl,
                                            prec == 3 ? Mix<e4m3>::TARGET : Mix<_Float16>::TARGET, acol,
                                            tscale);
  mixed_chi_kernel<<<dim3((ldl + 255) / 256, F), 256, 0, stream>>>(
      chi_re, chi_im, ldl, scaled ? inv_colscale : nullptr, prec == 3, scaled ? tscale : nullptr,
      chi_f32);
  // (tile, frequency-group) blocks, rounded up to a whole turn of the XCDs
  const int group = F < 32 ? F : 32;
  const long long blocks = (long long)n_tiles * ((F + group - 1) / group);
  const long long wgs = (blocks + MX_NXCD - 1) / MX_NXCD * MX_NXCD * group;
  if (prec == 3)
    pi_build_mixed_async_kernel<e4m3><<<(unsigned)wgs, 512, 0, stream>>>(
        static_cast<const _Float16 *>(Lf), static_cast<const unsigned char *>(Bhi), static_cast<const unsigned char *>(Blo), ldl,
        n_aux, chi_f32, tscale, tiles, n_tiles, F, group, G, g_stride, ldg);
  else if (prec == 2)
    pi_build_mixed_async_kernel<_Float16><<<(unsigned)wgs, 512, 0, stream>>>(
        static_cast<const float *>(Lf), static_cast<const unsigned short *>(Bhi), static_cast<const unsigned short *>(Blo), ldl,
        n_aux, chi_f32, tscale, tiles, n_tiles, F, group, G, g_stride, ldg);
  else
    pi_build_mixed_async_kernel<__bf16><<<(unsigned)wgs, 512, 0, stream>>>(
        static_cast<const float *>(Lf), static_cast<const unsigned short *>(Bhi), static_cast<const unsigned short *>(Blo), ldl,
        n_aux, chi_f32, nullptr, tiles, n_tiles, F, group, G, g_stride, ldg);
}

}  // namespace gwc
