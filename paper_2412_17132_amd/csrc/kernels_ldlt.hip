// Screened-interaction elements from a bordered LDL^T factorisation without
// pivoting (FP64 complex symmetric).
//
// 1 - Pi(z) is complex symmetric (Pi = L diag(chi) L^T).  On the real axis,
// z = x + i eta with x > 0, every Im chi_ia < 0, so Im(1 - Pi) = L |Im chi| L^T
// is positive semidefinite; on the imaginary axis 1 - Pi is real symmetric
// positive definite.  Then v^T (1 - Pi) v has a positive imaginary (or real)
// part for every real nonzero v restricted to a leading block, so every
// leading principal minor is nonsingular and the elimination needs no
// pivoting.  The bordered matrix
//
//        [ 1 - Pi(z)   B ]
//   M =  [ B^T         0 ]      (symmetric, order n = N + R)
//
// is factored L D L^T over its first N columns; the border block then holds
// the Schur complement -B^T (1 - Pi)^-1 B, and W^c = -S_rr - b^T b as for the
// LU (launch_bordered_finish).  Only the lower triangle is read.
//
// Right-looking, 64-column steps, per step and batch of matrices:
//   D  one workgroup per matrix: the 64 x 64 diagonal block A11 = L11 D1 L11^T
//      in LDS (64 dependent rank-1 steps), then L11^-1 (unit lower) to the
//      scratch and D1^-1 to the matrix's row of pivots' inverses;
//   T  one workgroup per (matrix, 64-row block below the panel): W = A21 L11^-T
//      on MFMA from the block staged in LDS, stored transposed in the row part
//      (the upper triangle, otherwise unused): W^T = D1 L21^T, so that
//   G  the trailing update A22 -= L21 (W^T) = L21 D1 L21^T is the LU's
//      trailing kernel restricted to the tiles on or below the diagonal
//      (half the tiles; border-border tiles off the diagonal skipped), both
//      operands read from the row part (L21[r][k] = W^T[k][r] / D[k]: the
//      left operand's loads are coalesced along r and no column part is
//      written).
// Up to LDLT_GROUP panels share one trailing update (K = 64 LDLT_GROUP), a
// later panel of a group first receiving the group's earlier panels on its own
// 64 columns.  Against the partial-pivoting LU this halves the trailing flops
// and removes the pivot searches, interchanges and row moves.
#include "gwc_internal.h"

namespace gwc {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NB = 64;
constexpr int NXCD = 8;
constexpr int LDLT_GROUP = 4;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zsub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 zinv(double2 d) {
  // 1/d with scaling by the larger component (Smith)
  if (fabs(d.x) >= fabs(d.y)) {
    const double r = d.y / d.x, den = d.x + d.y * r;
    return make_double2(1.0 / den, -r / den);
  }
  const double r = d.x / d.y, den = d.x * r + d.y;
  return make_double2(r / den, -1.0 / den);
}

// Workgroup -> (matrix, item), all items of a matrix on one XCD.
__device__ __forceinline__ bool xcd_item(int wg, int items, int F, int &f, int &item) {
  const int x = wg % NXCD, j = wg / NXCD;
  f = (j / items) * NXCD + x;
  item = j - (j / items) * items;
  return f < F;
}

// D: one workgroup (256 threads) per matrix.  X = the lower triangle of the
// kb x kb diagonal block (identity beyond kb), stored packed in LDS.  Step t: every row i > t takes
// X[i][j] -= (X[i][t] / d_t) X[j][t] for t < j <= i; the columns are scaled
// by 1/d_t after the last step (a step reads column t and writes only the
// columns right of it, so one barrier per step suffices).  Thread tid owns
// row tid / 4 and the columns j = tid % 4 (mod 4); the four threads of a row
// are in one wave.  Afterwards X holds L11 (unit, strictly lower) and D1
// (diagonal); D1^-1 goes to dinv_g[f N + K0 + t] and L11^-1 (the LU's
// right-looking in-place inversion, one barrier per step as well: step t
// reads row t and writes only rows below it, and a row's multiplier is read
// by the row's own wave before one of its threads overwrites it) to the
// scratch, zero-padded beyond kb.
__global__ void __launch_bounds__(256)
ldlt_diag_kernel(const double2 *__restrict__ G, long long gs, int ldg, int N, int K0,
                 double2 *__restrict__ linv_g, double2 *__restrict__ dinv_g, int *__restrict__ status) {
  // the lower triangle only, row by row (33 KB: four workgroups per CU)
  __shared__ double2 Xp[NB * (NB + 1) / 2];
  __shared__ double2 Dinv[NB];
  __shared__ int zero;
  auto X = [&](int r, int c) -> double2 & { return Xp[(r * (r + 1) >> 1) + c]; };
  const int f = blockIdx.x, tid = threadIdx.x;
  const double2 *A = G + (long long)f * gs;
  const int kb = min(NB, N - K0);
  if (tid == 0) zero = 0;
  {
    // all of a thread's loads in flight before its first LDS store
    constexpr int PER = NB * NB / 256;
    double2 v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      // every load unconditional, from an element inside the block (a load
      // under a branch would be waited for before the other branch's write)
      const int idx = q * 256 + tid, i = idx / NB, j = idx - i * NB;
      const int ic = min(i, kb - 1), jc = min(j, ic);
      const double2 a = A[(long long)(K0 + ic) * ldg + K0 + jc];
      v[q] = (i < kb && j <= i) ? a : make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = q * 256 + tid, i = idx / NB, j = idx - i * NB;
      if (j <= i) X(i, j) = v[q];
    }
  }
  __syncthreads();
  const int i = tid >> 2, j0 = tid & 3;
  for (int t = 0; t < kb; ++t) {
    const double2 d = X(t, t);
    const bool dz = d.x == 0.0 && d.y == 0.0;
    const double2 inv = dz ? make_double2(0.0, 0.0) : zinv(d);
    if (tid == 0) {
      if (dz) zero = 1;
      Dinv[t] = inv;
    }
    if (i > t) {
      const double2 l = zmul(X(i, t), inv);
      int j = t + 1 + ((j0 - (t + 1)) & 3);
      for (; j <= i; j += 4) X(i, j) = zsub(X(i, j), zmul(l, X(j, t)));
    }
    __syncthreads();
  }
  // L11: column t scaled by 1/d_t (the multipliers the steps used); D1^-1
  for (int t = j0; t < i && t < kb; t += 4) X(i, t) = zmul(X(i, t), Dinv[t]);
  if (tid < kb) dinv_g[(long long)f * N + K0 + tid] = Dinv[tid];
  __syncthreads();
  if (tid < NB) X(tid, tid) = make_double2(1.0, 0.0);
  __syncthreads();
  // L11^-1 in place: at step t every row i > t takes X[i][j] -= L[i][t] X[t][j]
  // for j < t and X[i][t] = -L[i][t] (row t of X is final by then)
  for (int t = 0; t < NB - 1; ++t) {
    if (i > t) {
      const double2 l = X(i, t);
      for (int j = j0; j < t; j += 4) X(i, j) = zsub(X(i, j), zmul(l, X(t, j)));
      if ((t & 3) == j0) X(i, t) = make_double2(-l.x, -l.y);
    }
    __syncthreads();
  }
  // L11^-1 is unit lower triangular: zeros above the diagonal and beyond kb
  double2 *Li = linv_g + (long long)f * NB * NB;
#pragma unroll
  for (int q = 0; q < NB * NB / 256; ++q) {
    const int idx = q * 256 + tid, r = idx / NB, c = idx - r * NB;
    Li[idx] = (r < kb && c <= r) ? X(r, c) : make_double2(0.0, 0.0);
  }
  if (tid == 0 && zero) status[f] = 1;
}

// T: one workgroup (4 waves) per (matrix, 64-row block of rows r0.. below the
// panel).  The A21 block is staged through LDS (coalesced rows); each wave
// forms 16 rows of W = A21 L11^-T on MFMA (L11^-1 from L2, shared by the
// matrix's workgroups on its XCD); W goes back to LDS and is stored
// transposed into the row part, A[K0 + k][r] = W[r][k], along contiguous
// rows.  Columns >= kb of the block are zero in LDS, rows >= n are not
// stored.  MFMA layouts: A[l%16][l/16], B[l/16][l%16], D[4r + l/16][l%16].
__global__ void __launch_bounds__(256)
ldlt_trsm_kernel(double2 *__restrict__ G, long long gs, int ldg, int N, int R, int K0, int F,
                 int nblk, const double2 *__restrict__ linv_g) {
  __shared__ double2 S[NB][NB + 1];
  int f, blk;
  if (!xcd_item(blockIdx.x, nblk, F, f, blk)) return;
  const int n = N + R;
  const int kb = min(NB, N - K0);
  const int r0 = K0 + kb + NB * blk;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double2 *A = G + (long long)f * gs;
  const double2 *Li = linv_g + (long long)f * NB * NB;
  // all of a thread's loads in flight before its first LDS store
  constexpr int PER = NB * NB / 256;
  double2 v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = q * 256 + tid, r = idx / NB, k = idx - r * NB;
    v[q] = (r0 + r < n && k < kb) ? A[(long long)(r0 + r) * ldg + K0 + k] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = q * 256 + tid;
    S[idx / NB][idx % NB] = v[q];
  }
  __syncthreads();
  d4 re[4], im[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    re[b] = d4{0.0, 0.0, 0.0, 0.0};
    im[b] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const int wr = 16 * wave;
  // the whole K of 64 unrolled (S and L11^-1 are zero beyond kb), so that the
  // L11^-1 loads of later steps are issued ahead of the products
#pragma unroll
  for (int kk = 0; kk < NB; kk += 4) {
    const int k = kk + lk;
    // A operand: rows wr + li of the block, column k; B operand:
    // L11^-T [k][c] = L11^-1 [c][k] (zero for k >= kb), c = 16 b + li.
    // Column block b needs k <= 16 b + 15 only: L11^-1 is lower triangular.
    const double2 av = S[wr + li][k];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (kk < 16 * b + 16) {
        const double2 bv = Li[(16 * b + li) * NB + k];
        re[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, re[b], 0, 0, 0);
        re[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.y, re[b], 0, 0, 0);
        im[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, im[b], 0, 0, 0);
        im[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, im[b], 0, 0, 0);
      }
    }
  }
  __syncthreads();  // every wave has read its A21 rows
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[wr + 4 * r + lk][16 * b + li] = make_double2(re[b][r], im[b][r]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = q * 256 + tid, k = idx / NB, r = idx - k * NB;
    if (k < kb && r0 + r < n) A[(long long)(K0 + k) * ldg + r0 + r] = S[r][k];
  }
}

struct LdltLaunch {
  double2 *G;
  long long gs;
  int ldg, N, R, F, fgroups;
  double2 *linv, *dinv;
  int *status;
  hipStream_t s;

  void diag_trsm(int K0) const {
    const int n = N + R;
    const int kb = min(NB, N - K0);
    ldlt_diag_kernel<<<F, 256, 0, s>>>(G, gs, ldg, N, K0, linv, dinv, status);
    const int nblk = (n - K0 - kb + NB - 1) / NB;
    if (nblk > 0)
      ldlt_trsm_kernel<<<NXCD * fgroups * nblk, 256, 0, s>>>(G, gs, ldg, N, R, K0, F, nblk, linv);
  }
  // rows [r0, n) x columns [c0, c1) -= L[.., K range] W^T[K range, ..]
  void trailing(int r0, int c0, int c1, int kstart, int klen, bool lower) const {
    launch_trailing_update_sym(G, gs, ldg, N, R, F, r0, c0, c1, kstart, klen, lower, dinv, N, s);
  }
};

}  // namespace

// L11^-1 of the current panel per matrix, then every pivot's D^-1 per matrix.
size_t ldlt_scratch_bytes(int F, int N) {
  return (size_t)F * ((size_t)NB * NB + (size_t)N) * sizeof(double2) + 256;
}

hipError_t launch_ldlt_bordered(double2 *G, long long g_stride, int ldg, int N, int R, int F,
                                const double *bb, const long long *out_base, const int *out_stride,
                                double2 *W_out, int *status, void *scratch, hipStream_t stream) {
  const int n = N + R;
  double2 *linv = static_cast<double2 *>(scratch);
  double2 *dinv = linv + (size_t)F * NB * NB;
  launch_zero_status(status, F, stream);
  const LdltLaunch L{G, g_stride, ldg, N, R, F, (F + NXCD - 1) / NXCD, linv, dinv, status, stream};
  int K0 = 0;
  while (K0 < N) {
    const int g = min(LDLT_GROUP, (N - K0) / NB);
    if (g >= 2) {
      const int a = K0, e = K0 + g * NB;
      for (int p = 0; p < g; ++p) {
        const int b = a + p * NB;
        if (p > 0) L.trailing(b, b, b + NB, a, p * NB, false);
        L.diag_trsm(b);
      }
      L.trailing(e, e, n, a, g * NB, true);
      K0 = e;
    } else {
      const int kend = min(K0 + NB, N);
      L.diag_trsm(K0);
      L.trailing(kend, kend, n, K0, kend - K0, true);
      K0 = kend;
    }
  }
  launch_bordered_finish(G, g_stride, ldg, N, R, F, bb, out_base, out_stride, W_out, stream);
  return hipGetLastError();
}

}  // namespace gwc
