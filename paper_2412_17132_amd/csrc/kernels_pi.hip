// RPA polarisability in the RI basis (FP64), CDNA4 MFMA.
//
//   Pi_PQ(z) = sum_ia M^P_ia M^Q_ia chi_ia(z),  chi_ia(z) = 4 Delta_ia / (z^2 - Delta_ia^2)
//
// (closed-shell response of each occupied-virtual pair; Delta_ia = eps_a - eps_i).
// The same formula covers the imaginary axis (z = i w, chi real and negative)
// and the residue frequencies (z = |eps_m - w| + i eta, chi complex).
//
// The build is L diag(chi) L^T with L = M_ov as an N_aux x N_ov matrix: a
// symmetric contraction over the long pair index, computed on FP64 MFMA
// (v_mfma_f64_16x16x4f64).  Each workgroup owns one 64 x 64 tile of the upper
// triangle for PI_FB frequencies, so every L tile staged in LDS feeds 2*PI_FB
// real products (Re chi and Im chi of each frequency); the output is written as
// 1 - Pi into the top-left block of the bordered matrix that the LU consumes.
#include "gwc_internal.h"

namespace gwc {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// L = M_ov reshaped to N_aux x N_ov, copied into a zero-padded buffer
// [n_aux_pad][ldl] (rows padded to 64, columns to PI_KC) so tile loads need no
// bounds checks.
__global__ void pack_l_kernel(const double *__restrict__ M_ov, int n_aux, int n_ov,
                              double *__restrict__ Lp, int n_aux_pad, int ldl) {
  const long long total = (long long)n_aux_pad * ldl;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int row = (int)(idx / ldl);
    const int col = (int)(idx - (long long)row * ldl);
    Lp[idx] = (row < n_aux && col < n_ov) ? M_ov[(long long)row * n_ov + col] : 0.0;
  }
}

void launch_pack_l(const double *M_ov, int n_aux, int n_ov, double *Lp, int n_aux_pad, int ldl,
                   hipStream_t stream) {
  const long long total = (long long)n_aux_pad * ldl;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  pack_l_kernel<<<(unsigned)blocks, 256, 0, stream>>>(M_ov, n_aux, n_ov, Lp, n_aux_pad, ldl);
}

// ---------------------------------------------------------------------------
// chi_ia(z_f) for every pair of every task of a batch, zero in the padding.
__global__ void chi_kernel(const double *__restrict__ eps, int n_occ, int n_virt,
                           const double2 *__restrict__ z, int ldl, double *__restrict__ chi_re,
                           double *__restrict__ chi_im) {
  const int f = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ldl) return;
  const int n_ov = n_occ * n_virt;
  double cr = 0.0, ci = 0.0;
  if (k < n_ov) {
    const int i = k / n_virt;
    const int a = k - i * n_virt;
    const double delta = eps[n_occ + a] - eps[i];
    const double x = z[f].x, y = z[f].y;
    // z^2 - Delta^2 = (x^2 - y^2 - Delta^2) + i (2 x y)
    const double dr = (x - y) * (x + y) - delta * delta;
    const double di = 2.0 * x * y;
    if (di == 0.0) {
      cr = 4.0 * delta / dr;
    } else {
      const double den = dr * dr + di * di;
      cr = 4.0 * delta * dr / den;
      ci = -4.0 * delta * di / den;
    }
  }
  chi_re[(long long)f * ldl + k] = cr;
  chi_im[(long long)f * ldl + k] = ci;
}

void launch_chi(const double *eps, int n_occ, int n_virt, const double2 *z, int F, int ldl,
                double *chi_re, double *chi_im, hipStream_t stream) {
  dim3 grid((ldl + 255) / 256, F);
  chi_kernel<<<grid, 256, 0, stream>>>(eps, n_occ, n_virt, z, ldl, chi_re, chi_im);
}

// ---------------------------------------------------------------------------
// Workgroup -> (tile, frequency pair) so that the workgroups one XCD holds at
// a time share a tile: workgroups go round-robin over the 8 XCDs, and each
// XCD's consecutive workgroups take one tile for `group` consecutive
// frequency pairs (two per CU of the XCD), so they read the same L rows,
// chunk by chunk, from the XCD's L2.  Blocks of (tile, pair group) go to the
// XCDs in turn.  False for the workgroups past the last pair.
constexpr int PI_NXCD = 8;
__device__ __forceinline__ bool pi_item(int wg, int n_tiles, int P, int group, int &tile, int &p) {
  const int x = wg % PI_NXCD, j = wg / PI_NXCD;
  const int blk = (j / group) * PI_NXCD + x;
  const int g = blk / n_tiles;
  tile = blk - g * n_tiles;
  p = g * group + j % group;
  return g * group < P && p < P;
}

// Pi build.  Grid: one workgroup per (tile, frequency pair), ordered by
// pi_item.  Wave w of the workgroup owns
// rows 32*(w/2) .. +32 and columns 32*(w%2) .. +32 of the 64 x 64 tile, i.e. a
// 2 x 2 block of 16 x 16 MFMA outputs, for PI_FB frequencies, real and
// imaginary parts: 16 accumulators of 4 doubles per lane.
//
// MFMA operand layout (v_mfma_f64_16x16x4f64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; output element r of lane l is D[4r + l/16][l%16].
__global__ void __launch_bounds__(PI_THREADS, 2)
pi_build_f64_kernel(const double *__restrict__ Lp, int ldl, int n_aux,
                    const double *__restrict__ chi_re, const double *__restrict__ chi_im, int F,
                    const int2 *__restrict__ tiles, int n_tiles, int group, double2 *__restrict__ G,
                    long long g_stride, int ldg) {
  constexpr int T = PI_TILE, KC = PI_KC, FB = PI_FB, LDA = KC + 1;
  __shared__ double As[T * LDA];
  __shared__ double Bs[T * LDA];
  __shared__ double Cs[FB][2][KC];

  int tile, pair;
  if (!pi_item(blockIdx.x, n_tiles, (F + FB - 1) / FB, group, tile, pair)) return;  // the whole workgroup
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int2 tb = tiles[tile];
  const int P0 = tb.x * T, Q0 = tb.y * T;
  const int f0 = pair * FB;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // on a diagonal tile the lower-left quadrant is the mirror of the upper-right
  // one: its wave stages operands with the others but forms no products, and
  // the upper-right wave writes both
  const bool idle = tb.x == tb.y && wr > wc;

  d4 acc[FB][2][2][2];
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[f][p][a][b] = d4{0.0, 0.0, 0.0, 0.0};

  const double *Arow = Lp + (long long)P0 * ldl;
  const double *Brow = Lp + (long long)Q0 * ldl;

  for (int kc = 0; kc < ldl; kc += KC) {
    // stage the two 64 x KC tiles of L (row-major, padded stride) and chi
#pragma unroll
    for (int it = 0; it < (T * KC / 2) / PI_THREADS; ++it) {
      const int idx = it * PI_THREADS + tid;
      const int row = idx / (KC / 2);
      const int kp = (idx - row * (KC / 2)) * 2;
      const double2 va = *reinterpret_cast<const double2 *>(Arow + (long long)row * ldl + kc + kp);
      const double2 vb = *reinterpret_cast<const double2 *>(Brow + (long long)row * ldl + kc + kp);
      As[row * LDA + kp] = va.x;
      As[row * LDA + kp + 1] = va.y;
      Bs[row * LDA + kp] = vb.x;
      Bs[row * LDA + kp + 1] = vb.y;
    }
    if (tid < FB * KC) {
      const int f = tid / KC, k = tid - (tid / KC) * KC;
      const int fg = f0 + f;
      double cr = 0.0, ci = 0.0;
      if (fg < F) {
        cr = chi_re[(long long)fg * ldl + kc + k];
        ci = chi_im[(long long)fg * ldl + kc + k];
      }
      Cs[f][0][k] = cr;
      Cs[f][1][k] = ci;
    }
    __syncthreads();

#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      if (idle) continue;  // uniform: the whole wave
      const int k = kk + lk;
      const double a0 = As[(wr + li) * LDA + k];
      const double a1 = As[(wr + 16 + li) * LDA + k];
      const double b0 = Bs[(wc + li) * LDA + k];
      const double b1 = Bs[(wc + 16 + li) * LDA + k];
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const double cr = Cs[f][0][k], ci = Cs[f][1][k];
        const double ar0 = a0 * cr, ar1 = a1 * cr, ai0 = a0 * ci, ai1 = a1 * ci;
        acc[f][0][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar0, b0, acc[f][0][0][0], 0, 0, 0);
        acc[f][0][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar0, b1, acc[f][0][0][1], 0, 0, 0);
        acc[f][0][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar1, b0, acc[f][0][1][0], 0, 0, 0);
        acc[f][0][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar1, b1, acc[f][0][1][1], 0, 0, 0);
        acc[f][1][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai0, b0, acc[f][1][0][0], 0, 0, 0);
        acc[f][1][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai0, b1, acc[f][1][0][1], 0, 0, 0);
        acc[f][1][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai1, b0, acc[f][1][1][0], 0, 0, 0);
        acc[f][1][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai1, b1, acc[f][1][1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // store 1 - Pi (and its mirror for off-diagonal tiles and the upper-right
  // quadrant of a diagonal tile)
  if (idle) return;
  const bool mirror = tb.x != tb.y || wr < wc;
#pragma unroll
  for (int f = 0; f < FB; ++f) {
    const int fg = f0 + f;
    if (fg >= F) break;
    double2 *Gf = G + (long long)fg * g_stride;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = P0 + wr + 16 * a + 4 * r + lk;
          const int col = Q0 + wc + 16 * b + li;
          if (row < n_aux && col < n_aux) {
            const double pr = acc[f][0][a][b][r], pi = acc[f][1][a][b][r];
            const double2 v = make_double2((row == col ? 1.0 : 0.0) - pr, -pi);
            Gf[(long long)row * ldg + col] = v;
            if (mirror) Gf[(long long)col * ldg + row] = v;
          }
        }
  }
}

void launch_pi_build_f64(const double *Lp, int ldl, int n_aux, const double *chi_re,
                         const double *chi_im, int F, const int2 *tiles, int n_tiles,
                         double2 *G, long long g_stride, int ldg, hipStream_t stream) {
  // (tile, pair-group) blocks, rounded up to a whole turn of the XCDs
  const int P = (F + PI_FB - 1) / PI_FB;
  const int group = P < 64 ? P : 64;
  const long long blocks = (long long)n_tiles * ((P + group - 1) / group);
  const long long wgs = (blocks + PI_NXCD - 1) / PI_NXCD * PI_NXCD * group;
  pi_build_f64_kernel<<<(unsigned)wgs, PI_THREADS, 0, stream>>>(Lp, ldl, n_aux, chi_re, chi_im, F, tiles,
                                                                n_tiles, group, G, g_stride, ldg);
}

}  // namespace gwc
