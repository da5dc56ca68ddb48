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
// Blocking (one workgroup per matrix, matrices private to a CU, so HBM
// traffic of the trailing update is what bounds it):
//   outer panels of LU_NBO = 64 columns, each factored as LU_NB = 16-wide inner
//   blocks (column-by-column pivoting, rank-16 updates inside the panel only);
//   then the panel's row swaps on the trailing columns, the 64 rows of U12 by
//   a blocked unit-lower solve, and one rank-64 trailing update whose 64 x 64
//   output tiles stay in registers across K = 64 (FP64 MFMA, the complex
//   product as four real products).  The trailing matrix is read and written
//   once per 64 eliminated columns.
#include "gwc_internal.h"

namespace gwc {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NBO = 64;  // outer panel width
constexpr int GT = 64;   // update tile
constexpr int KCH = 16;  // K chunk staged in LDS

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

struct LuShared {
  double red_v[LU_THREADS / 64];
  int red_i[LU_THREADS / 64];
  int piv[NBO];           // absolute pivot rows of the current outer panel
  double2 prow[LU_NB];
  double2 L11[LU_NB][LU_NB];
  double2 Ls[GT][KCH + 1];
  double2 Us[KCH][GT + 1];
  int singular;
};

// A[r0:r1, c0:c1] -= A[r0:r1, kA:kA+K] * A[kA:kA+K, c0:c1].  Tiles entirely
// inside the border-border block and off its diagonal are skipped.
__device__ void gemm_update(double2 *__restrict__ A, int ldg, int N, int r0, int r1, int c0,
                            int c1, int kA, int K, LuShared &sh) {
  if (r1 <= r0 || c1 <= c0 || K <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int mt = (r1 - r0 + GT - 1) / GT, nt = (c1 - c0 + GT - 1) / GT;
  for (int tile = 0; tile < mt * nt; ++tile) {
    const int ti = tile / nt, tj = tile - ti * nt;
    const int ra = r0 + ti * GT, ca = c0 + tj * GT;
    if (ra >= N && ca >= N && (ra + GT <= ca || ca + GT <= ra)) continue;
    d4 cre[2][2], cim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int col = ca + wc + 16 * b + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = ra + wr + 16 * a + 4 * r + lk;
          double2 v = make_double2(0.0, 0.0);
          if (row < r1 && col < c1) v = A[(long long)row * ldg + col];
          cre[a][b][r] = v.x;
          cim[a][b][r] = v.y;
        }
      }
    for (int kc = 0; kc < K; kc += KCH) {
      const int kw = min(KCH, K - kc);
      for (int idx = tid; idx < GT * KCH; idx += LU_THREADS) {
        const int r = idx / KCH, t = idx - r * KCH;
        sh.Ls[r][t] = (ra + r < r1 && t < kw) ? A[(long long)(ra + r) * ldg + kA + kc + t]
                                              : make_double2(0.0, 0.0);
      }
      for (int idx = tid; idx < KCH * GT; idx += LU_THREADS) {
        const int t = idx / GT, j = idx - t * GT;
        sh.Us[t][j] = (t < kw && ca + j < c1) ? A[(long long)(kA + kc + t) * ldg + ca + j]
                                              : make_double2(0.0, 0.0);
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KCH; kk += 4) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const double2 lv = sh.Ls[wr + 16 * a + li][kk + lk];
          const double ar = -lv.x, ai = -lv.y;
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const double2 uv = sh.Us[kk + lk][wc + 16 * b + li];
            cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, uv.x, cre[a][b], 0, 0, 0);
            cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.y, uv.y, cre[a][b], 0, 0, 0);
            cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, uv.y, cim[a][b], 0, 0, 0);
            cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, uv.x, cim[a][b], 0, 0, 0);
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int col = ca + wc + 16 * b + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = ra + wr + 16 * a + 4 * r + lk;
          if (row < r1 && col < c1)
            A[(long long)row * ldg + col] = make_double2(cre[a][b][r], cim[a][b][r]);
        }
      }
  }
}

// Rows [k0, k0+kb) of columns [c0, c1): unit-lower solve with the kb x kb
// diagonal block A[k0.., k0..].
__device__ void trsm_block(double2 *__restrict__ A, int ldg, int k0, int kb, int c0, int c1,
                           LuShared &sh) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < LU_NB * LU_NB; idx += LU_THREADS) {
    const int i = idx / LU_NB, t = idx - i * LU_NB;
    sh.L11[i][t] = (i < kb && t < kb) ? A[(long long)(k0 + i) * ldg + k0 + t] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int j = c0 + tid; j < c1; j += LU_THREADS) {
    // earlier rows are re-read from the cache (this thread wrote them)
    for (int i = 1; i < kb; ++i) {
      double2 acc = A[(long long)(k0 + i) * ldg + j];
      for (int t = 0; t < i; ++t) acc = csub(acc, cmul(sh.L11[i][t], A[(long long)(k0 + t) * ldg + j]));
      A[(long long)(k0 + i) * ldg + j] = acc;
    }
  }
  __syncthreads();
}

// Row interchanges (row_base + t) <-> piv[t0 + t] for t < cnt, in order, on
// columns [c0, c1).  Each thread owns whole columns, so no barrier is needed
// between interchanges.
__device__ void apply_swaps(double2 *__restrict__ A, int ldg, int row_base, int t0, int cnt,
                            int c0, int c1, const LuShared &sh) {
  for (int j = c0 + threadIdx.x; j < c1; j += LU_THREADS) {
    for (int t = 0; t < cnt; ++t) {
      const int c = row_base + t, p = sh.piv[t0 + t];
      if (p != c) {
        double2 *ec = A + (long long)c * ldg + j;
        double2 *ep = A + (long long)p * ldg + j;
        const double2 tmp = *ec;
        *ec = *ep;
        *ep = tmp;
      }
    }
  }
}

__global__ void __launch_bounds__(LU_THREADS, 4)
lu_bordered_kernel(double2 *__restrict__ G, long long g_stride, int ldg, int N, int R,
                   const double *__restrict__ bb, const long long *__restrict__ out_base,
                   const int *__restrict__ out_stride, double2 *__restrict__ W_out,
                   int *__restrict__ status) {
  constexpr int NT = LU_THREADS, NW = LU_THREADS / 64;
  __shared__ LuShared sh;
  const int f = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = N + R;
  double2 *A = G + (long long)f * g_stride;
  if (tid == 0) sh.singular = 0;

  for (int K0 = 0; K0 < N; K0 += NBO) {
    const int kbo = min(NBO, N - K0);
    const int kend = K0 + kbo;

    // ---- outer panel: inner blocks of LU_NB columns
    for (int k0 = K0; k0 < kend; k0 += LU_NB) {
      const int kb = min(LU_NB, kend - k0);
      const int ke = k0 + kb;
      for (int c = k0; c < ke; ++c) {
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
        if (lane == 0) { sh.red_v[wave] = best; sh.red_i[wave] = bi; }
        __syncthreads();
        if (tid == 0) {
          double b = sh.red_v[0];
          int p = sh.red_i[0];
          for (int w = 1; w < NW; ++w)
            if (sh.red_v[w] > b || (sh.red_v[w] == b && sh.red_i[w] < p)) { b = sh.red_v[w]; p = sh.red_i[w]; }
          sh.piv[c - K0] = p;
        }
        __syncthreads();
        const int p = sh.piv[c - K0];
        if (p != c && tid < kb) {
          double2 *rc = A + (long long)c * ldg + k0 + tid;
          double2 *rp = A + (long long)p * ldg + k0 + tid;
          const double2 t = *rc;
          *rc = *rp;
          *rp = t;
        }
        __syncthreads();
        if (tid < kb) sh.prow[tid] = A[(long long)c * ldg + k0 + tid];
        __syncthreads();
        const double2 d = sh.prow[c - k0];
        double2 inv;
        if (d.x == 0.0 && d.y == 0.0) {
          if (tid == 0) sh.singular = 1;
          inv = make_double2(0.0, 0.0);
        } else {
          inv = cinv(d);
        }
        for (int r = c + 1 + tid; r < n; r += NT) {
          double2 *row = A + (long long)r * ldg;
          const double2 l = cmul(row[c], inv);
          row[c] = l;
          for (int j = c + 1; j < ke; ++j) row[j] = csub(row[j], cmul(l, sh.prow[j - k0]));
        }
        __syncthreads();
      }
      // this block's interchanges on the rest of the outer panel
      apply_swaps(A, ldg, k0, k0 - K0, kb, K0, k0, sh);
      apply_swaps(A, ldg, k0, k0 - K0, kb, ke, kend, sh);
      __syncthreads();
      if (ke < kend) {
        trsm_block(A, ldg, k0, kb, ke, kend, sh);
        gemm_update(A, ldg, N, ke, n, ke, kend, k0, kb, sh);
      }
      __syncthreads();
    }
    if (kend >= n) continue;

    // ---- the panel's interchanges on the trailing columns
    apply_swaps(A, ldg, K0, 0, kbo, kend, n, sh);
    __syncthreads();
    // ---- U12 rows [K0, kend): blocked unit-lower solve
    for (int k0 = K0; k0 < kend; k0 += LU_NB) {
      const int kb = min(LU_NB, kend - k0);
      gemm_update(A, ldg, N, k0, k0 + kb, kend, n, K0, k0 - K0, sh);
      __syncthreads();
      trsm_block(A, ldg, k0, kb, kend, n, sh);
    }
    // ---- rank-kbo trailing update
    gemm_update(A, ldg, N, kend, n, kend, n, K0, kbo, sh);
    __syncthreads();
  }

  // ---- W_r = -S_rr - b_r^T b_r
  for (int r = tid; r < R; r += NT) {
    const double2 s = A[(long long)(N + r) * ldg + N + r];
    W_out[out_base[f] + (long long)r * out_stride[f]] =
        make_double2(-s.x - bb[(long long)f * R + r], -s.y);
  }
  __syncthreads();
  if (tid == 0) status[f] = sh.singular;
}

void launch_lu_bordered(double2 *G, long long g_stride, int ldg, int N, int R, int F,
                        const double *bb, const long long *out_base, const int *out_stride,
                        double2 *W_out, int *status, hipStream_t stream) {
  lu_bordered_kernel<<<F, LU_THREADS, 0, stream>>>(G, g_stride, ldg, N, R, bb, out_base,
                                                   out_stride, W_out, status);
}

}  // namespace gwc
