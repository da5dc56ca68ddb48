// Screened-interaction elements from a bordered LU factorisation (FP64 complex).
//
// For one frequency z and border vectors b_r (r < R) the workgroup factors
//
//        [ 1 - Pi(z)   B ]          B = [b_0 ... b_{R-1}]   (N x R)
//   M =  [ B^T         0 ]          n = N + R
//
// by Gaussian elimination of the first N columns with partial pivoting among
// the first N rows (the border rows never pivot).  The trailing diagonal then
// holds the Schur complement  -b_r^T (1 - Pi)^-1 b_r, so
//
//   W^c(z) = b^T [(1 - Pi(z))^-1 - 1] b = -S_rr - b^T b
//
// without any back substitution: the solve is folded into the elimination.
// Only the diagonal of the R x R border block is needed, so border-border
// tiles away from the diagonal are skipped.
//
// Right-looking blocked LU, panel width LU_NB: the panel is factored column
// by column, its row swaps are applied to the trailing columns, the U12 block
// is a unit-lower triangular solve, and the rank-LU_NB trailing update runs on
// FP64 MFMA (complex product as four real products).
#include "gwc_internal.h"

namespace gwc {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cinv(double2 d) {
  // 1/d with scaling by the larger component (Smith)
  if (fabs(d.x) >= fabs(d.y)) {
    const double r = d.y / d.x, den = d.x + d.y * r;
    return make_double2(1.0 / den, -r / den);
  }
  const double r = d.x / d.y, den = d.x * r + d.y;
  return make_double2(r / den, -1.0 / den);
}

constexpr int GT = 64;  // trailing-update tile

__global__ void __launch_bounds__(LU_THREADS)
lu_bordered_kernel(double2 *__restrict__ G, long long g_stride, int ldg, int N, int R,
                   const double *__restrict__ bb, const long long *__restrict__ out_base,
                   const int *__restrict__ out_stride, double2 *__restrict__ W_out,
                   int *__restrict__ status) {
  constexpr int NB = LU_NB, NT = LU_THREADS, NW = LU_THREADS / 64;
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ int piv[NB];
  __shared__ double2 prow[NB];
  __shared__ double2 L11[NB][NB];
  __shared__ double2 Ls[GT][NB + 1];
  __shared__ double2 Us[NB][GT + 1];
  __shared__ int singular;

  const int f = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int n = N + R;
  double2 *A = G + (long long)f * g_stride;
  if (tid == 0) singular = 0;

  for (int k0 = 0; k0 < N; k0 += NB) {
    const int kb = min(NB, N - k0);
    const int kend = k0 + kb;

    // ---- panel: columns [k0, kend), rows [k0, n)
    for (int c = k0; c < kend; ++c) {
      double best = -1.0;
      int bi = c;
      for (int r = c + tid; r < N; r += NT) {
        const double2 v = A[(long long)r * ldg + c];
        const double m = fabs(v.x) + fabs(v.y);
        if (m > best) { best = m; bi = r; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) { red_v[wave] = best; red_i[wave] = bi; }
      __syncthreads();
      if (tid == 0) {
        double b = red_v[0];
        int p = red_i[0];
        for (int w = 1; w < NW; ++w)
          if (red_v[w] > b || (red_v[w] == b && red_i[w] < p)) { b = red_v[w]; p = red_i[w]; }
        piv[c - k0] = p;
      }
      __syncthreads();
      const int p = piv[c - k0];
      if (p != c && tid < kb) {
        double2 *rc = A + (long long)c * ldg + k0 + tid;
        double2 *rp = A + (long long)p * ldg + k0 + tid;
        const double2 t = *rc;
        *rc = *rp;
        *rp = t;
      }
      __syncthreads();
      if (tid < kb) prow[tid] = A[(long long)c * ldg + k0 + tid];
      __syncthreads();
      const double2 d = prow[c - k0];
      double2 inv;
      if (d.x == 0.0 && d.y == 0.0) {
        if (tid == 0) singular = 1;
        inv = make_double2(0.0, 0.0);
      } else {
        inv = cinv(d);
      }
      for (int r = c + 1 + tid; r < n; r += NT) {
        double2 *row = A + (long long)r * ldg;
        const double2 l = cmul(row[c], inv);
        row[c] = l;
        for (int j = c + 1; j < kend; ++j) row[j] = csub(row[j], cmul(l, prow[j - k0]));
      }
      __syncthreads();
    }

    // ---- row swaps of this panel on the trailing columns [kend, n)
    for (int j = kend + tid; j < n; j += NT) {
      for (int t = 0; t < kb; ++t) {
        const int c = k0 + t, p = piv[t];
        if (p != c) {
          double2 *ec = A + (long long)c * ldg + j;
          double2 *ep = A + (long long)p * ldg + j;
          const double2 tmp = *ec;
          *ec = *ep;
          *ep = tmp;
        }
      }
    }
    // ---- U12 = L11^-1 A12 (unit lower triangular, kb x kb)
    for (int idx = tid; idx < NB * NB; idx += NT) {
      const int i = idx / NB, t = idx - i * NB;
      L11[i][t] = (i < kb && t < kb) ? A[(long long)(k0 + i) * ldg + k0 + t] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int j = kend + tid; j < n; j += NT) {
      // forward substitution down one column; earlier rows are re-read from
      // the cache (this thread wrote them) to keep register use low
      for (int i = 1; i < kb; ++i) {
        double2 acc = A[(long long)(k0 + i) * ldg + j];
        for (int t = 0; t < i; ++t) acc = csub(acc, cmul(L11[i][t], A[(long long)(k0 + t) * ldg + j]));
        A[(long long)(k0 + i) * ldg + j] = acc;
      }
    }
    __syncthreads();

    // ---- trailing update A22 -= L21 U12 on rows/cols [kend, n)
    const int rem = n - kend;
    if (rem <= 0) continue;
    const int mt = (rem + GT - 1) / GT;
    for (int tile = 0; tile < mt * mt; ++tile) {
      const int ti = tile / mt, tj = tile - ti * mt;
      const int ra = kend + ti * GT, ca = kend + tj * GT;
      // border-border tiles off the diagonal are never read
      if (ra >= N && ca >= N && (ra + GT <= ca || ca + GT <= ra)) continue;
      for (int idx = tid; idx < GT * NB; idx += NT) {
        const int r = idx / NB, t = idx - r * NB;
        Ls[r][t] = (ra + r < n && t < kb) ? A[(long long)(ra + r) * ldg + k0 + t]
                                          : make_double2(0.0, 0.0);
      }
      for (int idx = tid; idx < NB * GT; idx += NT) {
        const int t = idx / GT, j = idx - t * GT;
        Us[t][j] = (t < kb && ca + j < n) ? A[(long long)(k0 + t) * ldg + ca + j]
                                          : make_double2(0.0, 0.0);
      }
      __syncthreads();
#pragma unroll
      for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int row0 = ra + wr + 16 * a, col0 = ca + wc + 16 * b;
          const int col = col0 + li;
          d4 cre, cim;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = row0 + 4 * r + lk;
            double2 v = make_double2(0.0, 0.0);
            if (row < n && col < n) v = A[(long long)row * ldg + col];
            cre[r] = v.x;
            cim[r] = v.y;
          }
#pragma unroll
          for (int kk = 0; kk < NB; kk += 4) {
            const double2 lv = Ls[wr + 16 * a + li][kk + lk];
            const double2 uv = Us[kk + lk][wc + 16 * b + li];
            const double ar = -lv.x, ai = -lv.y;
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, uv.x, cre, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.y, uv.y, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, uv.y, cim, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, uv.x, cim, 0, 0, 0);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = row0 + 4 * r + lk;
            if (row < n && col < n) A[(long long)row * ldg + col] = make_double2(cre[r], cim[r]);
          }
        }
      }
      __syncthreads();
    }
  }

  // ---- W_r = -S_rr - b_r^T b_r
  for (int r = tid; r < R; r += NT) {
    const double2 s = A[(long long)(N + r) * ldg + N + r];
    W_out[out_base[f] + (long long)r * out_stride[f]] =
        make_double2(-s.x - bb[(long long)f * R + r], -s.y);
  }
  __syncthreads();
  if (tid == 0) status[f] = singular;
}

void launch_lu_bordered(double2 *G, long long g_stride, int ldg, int N, int R, int F,
                        const double *bb, const long long *out_base, const int *out_stride,
                        double2 *W_out, int *status, hipStream_t stream) {
  lu_bordered_kernel<<<F, LU_THREADS, 0, stream>>>(G, g_stride, ldg, N, R, bb, out_base,
                                                   out_stride, W_out, status);
}

}  // namespace gwc
