// Screened-interaction elements from a bordered LU factorisation (FP64 complex).
//
// For one frequency z and border vectors b_r (r < R) the batch factors
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
// Batched right-looking LU over all matrices of a batch, in 64-column panels:
//   P  one workgroup per matrix: the 64-wide panel (rows K0..n) is factored in
//      register-resident column blocks of width W (partial pivoting, rank-1
//      updates in registers, pivot row broadcast through LDS), with the block
//      updates inside the panel on MFMA; then the permutation of the step as a
//      list of row moves;
//   L  L11^-1 (64 x 64 unit lower) of the panel, for the next launch;
//   S  one workgroup per (matrix, 16 columns): applies the row moves and forms
//      U12 = L11^-1 A12 on MFMA;
//   G  one workgroup per (matrix, 64 x 64 tile): A22 -= L21 U12 on MFMA (the
//      complex product as three real products), tiles of a matrix kept on one
//      XCD so its L21 / U12 panels stay in that L2.
// Up to LU_GROUP panels share one trailing update (K = 64 LU_GROUP) while at
// least two whole panels remain.
#include "gwc_internal.h"

namespace gwc {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NBO = 64;                     // columns per step
constexpr int PT = 512;                     // panel threads
constexpr int PNW = PT / 64;
constexpr int MAX_MOVES = 2 * NBO;
constexpr int SW = 16;                      // trailing columns per swap/U12 workgroup
constexpr int NXCD = 8;
constexpr int LU_GROUP = 3;                 // panels per wide trailing update

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

// Workgroup -> (matrix, item) with all items of a matrix on one XCD
// (workgroups are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ bool xcd_map(int wg, int items, int F, int &f, int &item) {
  const int x = wg % NXCD, j = wg / NXCD;
  f = (j / items) * NXCD + x;
  item = j - (j / items) * items;
  return f < F;
}

// ===========================================================================
// P: panel factorisation
constexpr int WMAX = 16;  // widest register column block of the panel

struct PanelShared {
  double red_v[PNW];
  int red_i[PNW];
  int piv[NBO];
  int mrow[MAX_MOVES], mcont[MAX_MOVES];
  int flags;
  int bcnt;
  int brow[2 * WMAX], bcont[2 * WMAX];  // one block's interchanges as net row moves
  int bdst[2 * WMAX], bsrc[2 * WMAX];
  double2 prow[WMAX];
  double2 xbuf[WMAX];
  double2 lbb[WMAX][WMAX + 1];
  double2 lpre[WMAX][WMAX + 1];  // an odd block's rows of the even block's L
  int pslot[NBO];
  struct {
    struct {
      double2 stage[2 * WMAX][NBO];  // moved rows of the panel columns outside the block
      double2 U[WMAX][NBO];          // U rows of the block on the columns to its right
    } blk;
  } u;
};

// One workgroup per matrix.  Thread tid owns rows K0 + tid + s PT (s < RPT) for
// the whole panel.  The panel is factored in column blocks of width W:
//   1. the block's rows >= k0 are loaded into registers (v) and its W columns
//      are eliminated there: pivot search among rows < N (border rows never
//      pivot), the pivot row broadcast through LDS, rank-1 updates in registers;
//   2. the block is stored, and its interchanges are applied to the panel
//      columns left and right of it in one pass through LDS (net row moves);
//   3. the block's U rows on the columns to its right are solved with its unit
//      lower diagonal block (one thread per column, U rows kept in LDS);
//   4. the rows below are updated on MFMA stripes.  Blocks go in pairs: an
//      even block updates only the next block's columns, the odd block then
//      applies both blocks' rank-2W update to every column to its right, so
//      the rest of the panel is read and written once per pair instead of
//      once per block.
template <int RPT, int W, int WPE>
__global__ void __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(WPE)))
lu_panel_kernel(double2 *__restrict__ G, long long gs, int ldg, int N, int R, int K0,
                int *__restrict__ piv_g, int *__restrict__ moves_g, int *__restrict__ status) {
  static_assert(2 * W <= WMAX, "a pair of column blocks wider than the shared buffers");
  __shared__ PanelShared sh;
  const int f = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = N + R;
  double2 *A = G + (long long)f * gs;
  const int kbo = min(NBO, N - K0), kend = K0 + kbo;
  if (tid == 0) sh.flags = 0;
  __syncthreads();

  for (int k0 = K0; k0 < kend; k0 += W) {
    const int kb = min(W, kend - k0), ke = k0 + kb;
    double2 v[RPT][W];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = K0 + tid + s * PT;
#pragma unroll
      for (int j = 0; j < W; ++j)
        v[s][j] = (r >= k0 && r < n && j < kb) ? A[(long long)r * ldg + k0 + j]
                                               : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < W; ++c) {
      if (c < kb) {
        const int rc = k0 + c;
        double best = -1.0;
        int bi = rc;
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = K0 + tid + s * PT;
          if (r >= rc && r < N) {
            const double m = fabs(v[s][c].x) + fabs(v[s][c].y);
            if (m > best) { best = m; bi = r; }
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off);
          const int oi = __shfl_xor(bi, off);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (lane == 0) { sh.red_v[wave] = best; sh.red_i[wave] = bi; }
        __syncthreads();
        // every thread reduces the wave maxima itself (same order, same result)
        double bv = sh.red_v[0];
        int p = sh.red_i[0];
#pragma unroll
        for (int w = 1; w < PNW; ++w)
          if (sh.red_v[w] > bv || (sh.red_v[w] == bv && sh.red_i[w] < p)) { bv = sh.red_v[w]; p = sh.red_i[w]; }
        if (tid == 0) sh.piv[rc - K0] = p;
        // row rc is slot 0 of thread rc - K0 (rc - K0 < NBO <= PT); row p is
        // slot sp of thread tp: the owner of p publishes the pivot row, the
        // owner of rc its old content
        const int tc = rc - K0;
        const int tp = (p - K0) % PT, sp = (p - K0) / PT;
        if (tid == tp) {
#pragma unroll
          for (int s = 0; s < RPT; ++s)
            if (s == sp) {
#pragma unroll
              for (int j = 0; j < W; ++j) sh.prow[j] = v[s][j];
            }
        }
        if (p != rc && tid == tc) {
#pragma unroll
          for (int j = 0; j < W; ++j) sh.xbuf[j] = v[0][j];
        }
        __syncthreads();
        if (tid == tc) {
#pragma unroll
          for (int j = 0; j < W; ++j) v[0][j] = sh.prow[j];
        }
        if (p != rc && tid == tp) {
#pragma unroll
          for (int s = 0; s < RPT; ++s)
            if (s == sp) {
#pragma unroll
              for (int j = 0; j < W; ++j) v[s][j] = sh.xbuf[j];
            }
        }
        const double2 d = sh.prow[c];
        double2 inv;
        if (d.x == 0.0 && d.y == 0.0) {
          if (tid == 0) sh.flags = 1;
          inv = make_double2(0.0, 0.0);
        } else {
          inv = cinv(d);
        }
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = K0 + tid + s * PT;
          if (r > rc && r < n) {
            const double2 l = cmul(v[s][c], inv);
            v[s][c] = l;
#pragma unroll
            for (int j = c + 1; j < W; ++j)
              if (j < kb) v[s][j] = csub(v[s][j], cmul(l, sh.prow[j]));
          }
        }
      }  // c < kb
    }
    // 2. store the block; its interchanges as net row moves (content of row
    //    bsrc goes to row bdst) over the panel columns outside the block
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = K0 + tid + s * PT;
      if (r >= k0 && r < n) {
#pragma unroll
        for (int j = 0; j < W; ++j)
          if (j < kb) A[(long long)r * ldg + k0 + j] = v[s][j];
      }
    }
    if (tid == 0) {
      int cnt = 0;
      for (int t = 0; t < kb; ++t) {
        const int a = k0 + t, b = sh.piv[a - K0];
        int ia = -1, ib = -1;
        for (int i = 0; i < cnt; ++i) {
          if (sh.brow[i] == a) ia = i;
          if (sh.brow[i] == b) ib = i;
        }
        if (ia < 0) { sh.brow[cnt] = a; sh.bcont[cnt] = a; ia = cnt++; }
        if (ib < 0) { sh.brow[cnt] = b; sh.bcont[cnt] = b; ib = cnt++; }
        const int tmp = sh.bcont[ia];
        sh.bcont[ia] = sh.bcont[ib];
        sh.bcont[ib] = tmp;
      }
      int m = 0;
      for (int i = 0; i < cnt; ++i)
        if (sh.bcont[i] != sh.brow[i]) {
          sh.bdst[m] = sh.brow[i];
          sh.bsrc[m] = sh.bcont[i];
          ++m;
        }
      sh.bcnt = m;
    }
    __syncthreads();
    {
      const int cnt = sh.bcnt, nl = k0 - K0, nc = nl + (kend - ke);
      if (cnt > 0 && nc > 0) {
        for (int idx = tid; idx < cnt * nc; idx += PT) {
          const int i = idx / nc, cc = idx - i * nc;
          const int col = cc < nl ? K0 + cc : ke + (cc - nl);
          sh.u.blk.stage[i][cc] = A[(long long)sh.bsrc[i] * ldg + col];
        }
        __syncthreads();
        for (int idx = tid; idx < cnt * nc; idx += PT) {
          const int i = idx / nc, cc = idx - i * nc;
          const int col = cc < nl ? K0 + cc : ke + (cc - nl);
          A[(long long)sh.bdst[i] * ldg + col] = sh.u.blk.stage[i][cc];
        }
      }
    }
    __syncthreads();
    if (ke < kend) {
      // Blocks go in pairs (even, odd) by (k0 - K0) / W.  After an even block
      // only the next block's W columns are updated; after the odd block one
      // rank-(W + kb) update reaches every column to its right, so the rest of
      // the panel streams through memory once per pair.  The U rows of both
      // blocks stay in the U buffer, columns counted from the pair's base (the
      // even block's ke): the even block's in rows 0..W, the odd block's in
      // rows W..W+kb.
      const bool odd = (((k0 - K0) / W) & 1) != 0;
      const int base = odd ? k0 : ke, urow = odd ? W : 0;
      // 3. U rows k0..ke of columns ke..kend: unit lower solve with the
      //    diagonal block (rows k0..ke are slot 0 of threads k0-K0 .. ke-K0),
      //    for an odd block after subtracting the even block's contribution
      //    L[k0..ke, k0-W..k0] U_even (its update of these rows was deferred)
      if (tid >= k0 - K0 && tid < ke - K0) {
        const int i = tid - (k0 - K0);
#pragma unroll
        for (int t = 0; t < W; ++t) sh.lbb[i][t] = v[0][t];
      }
      if (odd)
        for (int idx = tid; idx < kb * W; idx += PT) {
          const int i = idx / W, t = idx - i * W;
          sh.lpre[i][t] = A[(long long)(k0 + i) * ldg + k0 - W + t];
        }
      __syncthreads();
      // one thread per column; the solved rows accumulate in the U buffer
      for (int c = ke + tid; c < kend; c += PT) {
        double2 *uc = &sh.u.blk.U[urow][c - base];
        for (int i = 0; i < kb; ++i) {
          double2 x = A[(long long)(k0 + i) * ldg + c];
          if (odd)
            for (int t = 0; t < W; ++t) x = csub(x, cmul(sh.lpre[i][t], sh.u.blk.U[t][c - base]));
          uc[i * NBO] = x;
        }
#pragma unroll 1
        for (int i = 1; i < kb; ++i) {
          double2 x = uc[i * NBO];
          for (int t = 0; t < i; ++t) x = csub(x, cmul(sh.lbb[i][t], uc[t * NBO]));
          uc[i * NBO] = x;
        }
        for (int i = 0; i < kb; ++i) A[(long long)(k0 + i) * ldg + c] = uc[i * NBO];
      }
      __syncthreads();
      // 4. update of rows ke..n on columns ke..cend (at most 4 tiles of 16
      //    columns) with the K range kbeg..kbeg+klen on MFMA, without
      //    barriers: each wave takes 16-row stripes; L from the stored
      //    blocks, U from LDS (columns past cend read a clamped U column and
      //    are not stored).  The MFMA layouts: A[l%16][l/16], B[l/16][l%16],
      //    D[4r + l/16][l%16].
      const int li = lane & 15, lk = lane >> 4;
      const int cend = odd ? kend : min(ke + W, kend);
      const int kbeg = odd ? k0 - W : k0, klen = odd ? W + kb : kb, uoff = ke - base;
      const int nct = (cend - ke + 15) / 16;
#pragma unroll 1
      for (int r0 = ke + 16 * wave; r0 < n; r0 += 16 * PNW) {
        d4 cre[4], cim[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const int col = ke + 16 * ct + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + 4 * r + lk;
            double2 x = make_double2(0.0, 0.0);
            if (ct < nct && row < n && col < cend) x = A[(long long)row * ldg + col];
            cre[ct][r] = x.x;
            cim[ct][r] = x.y;
          }
        }
#pragma unroll
        for (int kk = 0; kk < 2 * W; kk += 4) {
          if (kk < klen) {
            const int row = r0 + li, k = kk + lk;
            const double2 lv = (row < n && k < klen) ? A[(long long)row * ldg + kbeg + k]
                                                     : make_double2(0.0, 0.0);
            const double ar = -lv.x, ai = -lv.y;
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
              if (ct < nct) {
                const double2 uv = k < klen ? sh.u.blk.U[k][min(uoff + 16 * ct + li, NBO - 1)]
                                            : make_double2(0.0, 0.0);
                cre[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, uv.x, cre[ct], 0, 0, 0);
                cre[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.y, uv.y, cre[ct], 0, 0, 0);
                cim[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, uv.y, cim[ct], 0, 0, 0);
                cim[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, uv.x, cim[ct], 0, 0, 0);
              }
            }
          }
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const int col = ke + 16 * ct + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + 4 * r + lk;
            if (ct < nct && row < n && col < cend)
              A[(long long)row * ldg + col] = make_double2(cre[ct][r], cim[ct][r]);
          }
        }
      }
    }
    __syncthreads();
  }

  if (tid < kbo) piv_g[(long long)f * NBO + tid] = sh.piv[tid];
  // net row moves of the step: slot t < kbo holds row K0 + t, slot kbo + t the
  // pivot row piv[t] when it lies below the panel and t is its first use
  if (tid < kbo) {
    const int p = sh.piv[tid];
    int first = tid;
    if (p >= kend)
      for (int u = 0; u < tid; ++u)
        if (sh.piv[u] == p) { first = u; break; }
    sh.pslot[tid] = p < kend ? p - K0 : kbo + first;
    sh.mrow[tid] = K0 + tid;
    sh.mcont[tid] = K0 + tid;
    sh.mrow[kbo + tid] = p;
    sh.mcont[kbo + tid] = p;
  }
  __syncthreads();
  if (tid == 0) {
    for (int t = 0; t < kbo; ++t) {
      const int b = sh.pslot[t];
      const int tmp = sh.mcont[t];
      sh.mcont[t] = sh.mcont[b];
      sh.mcont[b] = tmp;
    }
    int m = 0;
    int *mv = moves_g + (long long)f * (1 + 2 * MAX_MOVES);
    for (int i = 0; i < 2 * kbo; ++i)
      if (sh.mcont[i] != sh.mrow[i]) {
        mv[1 + 2 * m] = sh.mrow[i];
        mv[2 + 2 * m] = sh.mcont[i];
        ++m;
      }
    mv[0] = m;
    if (sh.flags) status[f] = 1;
  }
}

// L11^-1 of the step's panel (unit lower, 64 x 64), one workgroup per matrix,
// in place in LDS, right-looking: X starts as L11 (identity on the diagonal);
// at step t every row i > t takes X[i][j] -= L[i][t] X[t][j] for j < t and
// X[i][t] = -L[i][t] (row t of X is final by then).  Thread tid owns row
// tid / 4 and the columns j = tid % 4 (mod 4); L[i][t] is read before the
// barrier that precedes its overwrite.
__global__ void __launch_bounds__(256)
lu_linv_kernel(const double2 *__restrict__ G, long long gs, int ldg, int N, int K0,
               double2 *__restrict__ linv_g) {
  __shared__ double2 X[NBO][NBO + 1];
  const int f = blockIdx.x, tid = threadIdx.x;
  const double2 *A = G + (long long)f * gs;
  const int kbo = min(NBO, N - K0);
  for (int idx = tid; idx < NBO * NBO; idx += 256) {
    const int i = idx / NBO, j = idx - i * NBO;
    X[i][j] = (i < kbo && j < i) ? A[(long long)(K0 + i) * ldg + K0 + j]
                                 : make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int i = tid >> 2, j0 = tid & 3;
  for (int t = 0; t < NBO - 1; ++t) {
    const double2 l = X[i][t];
    __syncthreads();
    if (i > t) {
      for (int j = j0; j < t; j += 4) X[i][j] = csub(X[i][j], cmul(l, X[t][j]));
      if ((t & 3) == j0) X[i][t] = make_double2(-l.x, -l.y);
    }
    __syncthreads();
  }
  double2 *Li = linv_g + (long long)f * NBO * NBO;
  for (int idx = tid; idx < NBO * NBO; idx += 256) {
    const int r = idx / NBO, c = idx - r * NBO;
    Li[idx] = (r < kbo && c < kbo) ? X[r][c] : make_double2(0.0, 0.0);
  }
}

// ===========================================================================
// S: row moves on columns [c_start, c_end) (16 per workgroup, 4 waves of 16
// rows each); with u12, then U12 = L11^-1 A12 for the panel rows K0..K0+64,
// after subtracting the contribution of the earlier panels of its group
// A[K0.., kpre..K0] A[kpre..K0, ..] when kpre >= 0 (a later panel of a
// grouped step, whose rows the wide trailing update skips).
__global__ void __launch_bounds__(256)
lu_swap_u12_kernel(double2 *__restrict__ G, long long gs, int ldg, int N, int K0, int F,
                   int nchunks, int c_start, int c_end, int kpre, int u12,
                   const int *__restrict__ moves_g, const double2 *__restrict__ linv_g) {
  __shared__ int mv[1 + 2 * MAX_MOVES];
  __shared__ double2 val[NBO][SW + 1];
  int f, chunk;
  if (!xcd_map(blockIdx.x, nchunks, F, f, chunk)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int kbo = min(NBO, N - K0);
  const int c0 = c_start + chunk * SW, cw = min(SW, c_end - c0);
  double2 *A = G + (long long)f * gs;
  const int *m = moves_g + (long long)f * (1 + 2 * MAX_MOVES);
  for (int i = tid; i < 1 + 2 * MAX_MOVES; i += 256) mv[i] = m[i];
  __syncthreads();
  // the moves go through registers: every source is read before any
  // destination is written (a row can be both)
  const int cnt = mv[0];
  constexpr int MPT = MAX_MOVES * SW / 256;
  double2 moved[MPT];
#pragma unroll
  for (int q = 0; q < MPT; ++q) {
    const int idx = tid + 256 * q, i = idx / SW, j = idx - i * SW;
    moved[q] = (i < cnt && j < cw) ? A[(long long)mv[2 + 2 * i] * ldg + c0 + j]
                                   : make_double2(0.0, 0.0);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MPT; ++q) {
    const int idx = tid + 256 * q, i = idx / SW, j = idx - i * SW;
    if (i < cnt && j < cw) A[(long long)mv[1 + 2 * i] * ldg + c0 + j] = moved[q];
  }
  if (!u12) return;
  __syncthreads();
  for (int idx = tid; idx < NBO * SW; idx += 256) {
    const int t = idx / SW, j = idx - t * SW;
    val[t][j] = (t < kbo && j < cw) ? A[(long long)(K0 + t) * ldg + c0 + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (kpre >= 0) {
    d4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
    const int arow = K0 + 16 * wave + li;
    const int kplen = K0 - kpre;
#pragma unroll 4
    for (int kk = 0; kk < kplen; kk += 4) {
      const int k = kpre + kk + lk;
      const double2 a = (16 * wave + li < kbo) ? A[(long long)arow * ldg + k] : make_double2(0.0, 0.0);
      const double2 b = (li < cw) ? A[(long long)k * ldg + c0 + li] : make_double2(0.0, 0.0);
      yr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, yr, 0, 0, 0);
      yr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, yi, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, yi, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = 16 * wave + 4 * r + lk;
      val[t][li] = make_double2(val[t][li].x - yr[r], val[t][li].y - yi[r]);
    }
    __syncthreads();
  }
  const double2 *Li = linv_g + (long long)f * NBO * NBO;
  d4 re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < NBO; kk += 4) {
    const double2 a = Li[(16 * wave + li) * NBO + kk + lk];
    const double2 b = val[kk + lk][li];
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, im, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * wave + 4 * r + lk;
    if (row < kbo && li < cw) A[(long long)(K0 + row) * ldg + c0 + li] = make_double2(re[r], im[r]);
  }
}

// ===========================================================================
// G: trailing update A[rows, cols] -= A[rows, K] A[K, cols] over the K range
// [kstart, kstart + klen) (a multiple of 64 up to 64 LU_GROUP, or the ragged
// last panel), one 64 x 64 tile
// per workgroup on an mt_r x mt_c grid from (row0, col0), columns below col_end
// only (a range may end inside a tile); the MFMA operands
// come straight from memory (the panels of one matrix are shared in its XCD's
// L2), so the K loop has no barriers.  The operands of the next k step are
// loaded into a second register set while the MFMAs of the current one run.
// LOWER: the grid holds only the tiles on or below the diagonal of a square
// range (row0 == col0, mt_r == mt_c), tile t -> (ti, tj) with
// t = ti (ti + 1) / 2 + tj, tj <= ti (the symmetric factorisation's update).
// SYM: the left operand comes from the row part as well, A[r][k] = A[k][r] d_k
// with d_k = dinv[f dinv_ld + k] (the symmetric factorisation keeps only
// W^T = D L^T in the rows of its panels: L[r][k] = W^T[k][r] / D[k]).
template <bool LOWER, bool SYM>
__global__ void __launch_bounds__(256, 3)
lu_trailing_kernel(double2 *__restrict__ G, long long gs, int ldg, int N, int R, int F, int row0,
                   int col0, int col_end, int mt_r, int mt_c, int kstart, int klen,
                   const double2 *__restrict__ dinv, int dinv_ld) {
  int f, tile;
  const int items = LOWER ? mt_r * (mt_r + 1) / 2 : mt_r * mt_c;
  if (!xcd_map(blockIdx.x, items, F, f, tile)) return;
  const int n = N + R;
  int ti, tj;
  if (LOWER) {
    ti = (int)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
    while (ti * (ti + 1) / 2 > tile) --ti;
    tj = tile - ti * (ti + 1) / 2;
  } else {
    ti = tile / mt_c;
    tj = tile - ti * mt_c;
  }
  const int ra = row0 + ti * 64, ca = col0 + tj * 64;
  if (ra >= N && ca >= N && (ra + 64 <= ca || ca + 64 <= ra)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  // the strictly upper quadrant of a diagonal tile is never read by the
  // symmetric factorisation (the kernel has no barriers: a wave may leave)
  if (LOWER && ra == ca && wr < wc) return;
  double2 *A = G + (long long)f * gs;

  // complex product in three real MFMA products (Gauss):
  //   P1 = L_r U_r, P2 = L_i U_i, P3 = (L_r + L_i)(U_r + U_i),
  //   (L U)_r = P1 - P2, (L U)_i = P3 - P1 - P2
  d4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      p1[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      p2[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      p3[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    }
  auto mfmas = [&](const double2 (&lv)[2], const double2 (&uv)[2]) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double ls = lv[a].x + lv[a].y;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double us = uv[b].x + uv[b].y;
        p1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv[a].x, uv[b].x, p1[a][b], 0, 0, 0);
        p2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv[a].y, uv[b].y, p2[a][b], 0, 0, 0);
        p3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ls, us, p3[a][b], 0, 0, 0);
      }
    }
  };

  // Whole steps of 4 k: rows >= n and columns >= col_end only feed outputs
  // that are never stored, so their operands come unmasked from a clamped,
  // in-bounds row or column.
  const double2 *lrow[2], *ucol[2];
  const double2 *dk = SYM ? dinv + (long long)f * dinv_ld + kstart + lk : nullptr;
#pragma unroll
  for (int a = 0; a < 2; ++a)
    lrow[a] = SYM ? A + (long long)(kstart + lk) * ldg + min(ra + wr + 16 * a + li, n - 1)
                  : A + (long long)min(ra + wr + 16 * a + li, n - 1) * ldg + kstart + lk;
#pragma unroll
  for (int b = 0; b < 2; ++b)
    ucol[b] = A + (long long)(kstart + lk) * ldg + min(ca + wc + 16 * b + li, col_end - 1);
  const long long ustep = 4LL * ldg;
  auto load_ops = [&](int kk, double2 (&lv)[2], double2 (&uv)[2]) {
    if (SYM) {
      const double2 d = dk[kk];
#pragma unroll
      for (int a = 0; a < 2; ++a) lv[a] = cmul(lrow[a][(kk >> 2) * ustep], d);
    } else {
#pragma unroll
      for (int a = 0; a < 2; ++a) lv[a] = lrow[a][kk];
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) uv[b] = ucol[b][(kk >> 2) * ustep];
  };
  const int klen4 = klen & ~3;
  if (klen4 > 0) {
    double2 la[2], ua[2], lb[2], ub[2];
    load_ops(0, la, ua);
    for (int kk = 0; kk < klen4; kk += 8) {
      load_ops(min(kk + 4, klen4 - 4), lb, ub);
      __builtin_amdgcn_sched_barrier(0);  // keep the next loads ahead of these MFMAs
      mfmas(la, ua);
      if (kk + 4 >= klen4) break;
      load_ops(min(kk + 8, klen4 - 4), la, ua);
      __builtin_amdgcn_sched_barrier(0);
      mfmas(lb, ub);
    }
  }
  if (klen4 < klen) {
    // ragged end of the K range: lanes with k >= klen contribute zero
    const int k = klen4 + lk;
    double2 lv[2], uv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int row = ra + wr + 16 * a + li;
      if (SYM)
        lv[a] = (k < klen && row < n)
                    ? cmul(A[(long long)(kstart + k) * ldg + row], dinv[(long long)f * dinv_ld + kstart + k])
                    : make_double2(0.0, 0.0);
      else
        lv[a] = (k < klen && row < n) ? A[(long long)row * ldg + kstart + k] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = ca + wc + 16 * b + li;
      uv[b] = (k < klen && col < col_end) ? A[(long long)(kstart + k) * ldg + col]
                                          : make_double2(0.0, 0.0);
    }
    mfmas(lv, uv);
  }

  // the tile's values, a row of 16 x 16 blocks at a time: the eight values per
  // lane loaded before any is stored (two memory round trips for the tile;
  // the compiler cannot move a block's loads above the stores of another, and
  // all sixteen at once would not fit beside the accumulators)
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    double2 x[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int colc = min(ca + wc + 16 * b + li, col_end - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        x[b][r] = A[(long long)min(ra + wr + 16 * a + 4 * r + lk, n - 1) * ldg + colc];
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = ca + wc + 16 * b + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ra + wr + 16 * a + 4 * r + lk;
        const double q1 = p1[a][b][r], q2 = p2[a][b][r];
        if (row < n && col < col_end)
          A[(long long)row * ldg + col] =
              make_double2(x[b][r].x - (q1 - q2), x[b][r].y - (p3[a][b][r] - q1 - q2));
      }
    }
  }
}

// ===========================================================================
__global__ void lu_finish_kernel(const double2 *__restrict__ G, long long gs, int ldg, int N,
                                 int R, const double *__restrict__ bb,
                                 const long long *__restrict__ out_base,
                                 const int *__restrict__ out_stride, double2 *__restrict__ W_out) {
  const int f = blockIdx.x;
  const double2 *A = G + (long long)f * gs;
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    const double2 s = A[(long long)(N + r) * ldg + N + r];
    W_out[out_base[f] + (long long)r * out_stride[f]] =
        make_double2(-s.x - bb[(long long)f * R + r], -s.y);
  }
}

__global__ void zero_int_kernel(int *__restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

size_t lu_scratch_bytes(int F) {
  return (size_t)F * (NBO * sizeof(int) + (1 + 2 * MAX_MOVES) * sizeof(int) +
                      NBO * NBO * sizeof(double2)) + 256;
}

int lu_max_order() { return 24 * PT; }

// WPE: waves per SIMD the register allocation must allow (4: two panel
// workgroups per CU, where that costs at most a small spill)
template <int RPT, int W, int WPE>
static void launch_panel(int F, double2 *G, long long gs, int ldg, int N, int R, int K0, int *piv,
                         int *moves, int *status, hipStream_t stream) {
  lu_panel_kernel<RPT, W, WPE><<<F, PT, 0, stream>>>(G, gs, ldg, N, R, K0, piv, moves, status);
}

namespace {

struct LuLaunch {
  double2 *G;
  long long gs;
  int ldg, N, R, F, fgroups;
  int *piv, *moves, *status;
  double2 *linv;
  hipStream_t s;

  void panel(int K0) const {
    const int rpt = (N + R + PT - 1) / PT;
    // register block v[RPT][W] kept at <= 128 VGPRs; up to 512 rows take the
    // two-row form too (the one-row form spills its update accumulators)
    if (rpt <= 2) launch_panel<2, 8, 4>(F, G, gs, ldg, N, R, K0, piv, moves, status, s);
    else if (rpt <= 3) launch_panel<3, 8, 4>(F, G, gs, ldg, N, R, K0, piv, moves, status, s);
    else if (rpt <= 4) launch_panel<4, 8, 1>(F, G, gs, ldg, N, R, K0, piv, moves, status, s);
    else if (rpt <= 6) launch_panel<6, 4, 1>(F, G, gs, ldg, N, R, K0, piv, moves, status, s);
    else if (rpt <= 8) launch_panel<8, 4, 1>(F, G, gs, ldg, N, R, K0, piv, moves, status, s);
    else if (rpt <= 12) launch_panel<12, 2, 1>(F, G, gs, ldg, N, R, K0, piv, moves, status, s);
    else if (rpt <= 16) launch_panel<16, 1, 1>(F, G, gs, ldg, N, R, K0, piv, moves, status, s);
    else launch_panel<24, 1, 1>(F, G, gs, ldg, N, R, K0, piv, moves, status, s);
    lu_linv_kernel<<<F, 256, 0, s>>>(G, gs, ldg, N, K0, linv);
  }
  // row moves of the panel at K0 on columns [c0, c1); with u12 also its U rows
  void swap_u12(int K0, int c0, int c1, int kpre, int u12) const {
    const int nch = (c1 - c0 + SW - 1) / SW;
    if (nch < 1) return;
    lu_swap_u12_kernel<<<NXCD * fgroups * nch, 256, 0, s>>>(G, gs, ldg, N, K0, F, nch, c0, c1, kpre,
                                                             u12, moves, linv);
  }
  // rows [r0, n) x columns [c0, c1) -= A[.., K range] A[K range, ..]
  void trailing(int r0, int c0, int c1, int kstart, int klen) const {
    const int n = N + R;
    const int mt_r = (n - r0 + 63) / 64, mt_c = (c1 - c0 + 63) / 64;
    if (mt_r < 1 || mt_c < 1) return;
    lu_trailing_kernel<false, false><<<NXCD * fgroups * mt_r * mt_c, 256, 0, s>>>(
        G, gs, ldg, N, R, F, r0, c0, c1, mt_r, mt_c, kstart, klen, nullptr, 0);
  }
};

}  // namespace

hipError_t launch_lu_bordered(double2 *G, long long g_stride, int ldg, int N, int R, int F,
                              const double *bb, const long long *out_base, const int *out_stride,
                              double2 *W_out, int *status, void *scratch, hipStream_t stream) {
  const int n = N + R;
  int *piv = static_cast<int *>(scratch);
  int *moves = piv + (size_t)F * NBO;
  double2 *linv = reinterpret_cast<double2 *>(
      (reinterpret_cast<uintptr_t>(moves + (size_t)F * (1 + 2 * MAX_MOVES)) + 255) & ~uintptr_t(255));
  zero_int_kernel<<<(F + 255) / 256, 256, 0, stream>>>(status, F);
  const LuLaunch L{G, g_stride, ldg, N, R, F, (F + NXCD - 1) / NXCD, piv, moves, status, linv, stream};
  int K0 = 0;
  while (K0 < N) {
    const int g = min(LU_GROUP, (N - K0) / NBO);
    if (g >= 2) {
      // g whole panels, then one trailing update with K = 64 g: the A22 block
      // streams through memory once per 64 g columns.  Panel p first receives
      // the updates of the group's earlier panels on its own columns; after
      // it is factored, its row moves reach the group's earlier L columns, and
      // its U rows (less the earlier panels' contribution) every column to its
      // right.
      const int a = K0, e = K0 + g * NBO;
      for (int p = 0; p < g; ++p) {
        const int b = a + p * NBO;
        if (p > 0) L.trailing(b, b, b + NBO, a, p * NBO);
        L.panel(b);
        if (p > 0) L.swap_u12(b, a, b, -1, 0);
        L.swap_u12(b, b + NBO, n, p > 0 ? a : -1, 1);
      }
      L.trailing(e, e, n, a, g * NBO);
      K0 = e;
    } else {
      const int kend = min(K0 + NBO, N);
      L.panel(K0);
      L.swap_u12(K0, kend, n, -1, 1);
      L.trailing(kend, kend, n, K0, kend - K0);
      K0 = kend;
    }
  }
  lu_finish_kernel<<<F, 64, 0, stream>>>(G, g_stride, ldg, N, R, bb, out_base, out_stride, W_out);
  return hipGetLastError();
}

void launch_trailing_update_sym(double2 *G, long long gs, int ldg, int N, int R, int F, int r0,
                                int c0, int c1, int kstart, int klen, bool lower,
                                const double2 *dinv, int dinv_ld, hipStream_t s) {
  const int n = N + R;
  const int mt_r = (n - r0 + 63) / 64, mt_c = (c1 - c0 + 63) / 64;
  if (mt_r < 1 || mt_c < 1) return;
  const int fgroups = (F + NXCD - 1) / NXCD;
  if (lower)
    lu_trailing_kernel<true, true><<<NXCD * fgroups * (mt_r * (mt_r + 1) / 2), 256, 0, s>>>(
        G, gs, ldg, N, R, F, r0, c0, c1, mt_r, mt_r, kstart, klen, dinv, dinv_ld);
  else
    lu_trailing_kernel<false, true><<<NXCD * fgroups * mt_r * mt_c, 256, 0, s>>>(
        G, gs, ldg, N, R, F, r0, c0, c1, mt_r, mt_c, kstart, klen, dinv, dinv_ld);
}

void launch_bordered_finish(const double2 *G, long long gs, int ldg, int N, int R, int F,
                            const double *bb, const long long *out_base, const int *out_stride,
                            double2 *W_out, hipStream_t s) {
  lu_finish_kernel<<<F, 64, 0, s>>>(G, gs, ldg, N, R, bb, out_base, out_stride, W_out);
}

void launch_zero_status(int *status, int F, hipStream_t s) {
  zero_int_kernel<<<(F + 255) / 256, 256, 0, s>>>(status, F);
}

}  // namespace gwc
