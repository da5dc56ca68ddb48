// Fully analytic G0W0 for core states (paper section "GW for core levels":
// Eqs. rpa_casida, rpa_matrices, density_shifts, sigma_spectral,
// A_explicit_real_imaginary, hedin_sigma_spectral).
//
// Closed-shell singlet RPA in the symmetric form C Z = Omega^2 Z with
//   C = Delta^2 + 4 Delta^1/2 K Delta^1/2 = Vt^T Vt + diag(Delta^2),
//   Vt[P][ia] = 2 Delta_ia^1/2 M^P_ia,   X + Y = Delta^1/2 Z Omega^-1/2.
// The eigenvectors are never formed: every Jacobi rotation applied to C is
// also applied to Y = Delta^1/2 L (Y[P][ia] = Delta_ia^1/2 M^P_ia), which ends
// as R = Y Z, so that rho^nu_nm = sqrt(2) sum_P M^P_nm R[P][nu] / Omega_nu^1/2.
//
// Eigensolver: cyclic block Jacobi.  Indices are grouped in blocks of JB = 32;
// a sweep has nb - 1 rounds (round-robin ordering of the nb blocks), each
// pairing all blocks disjointly.  Per round, jacobi_pair_kernel takes each
// pair's 64 x 64 principal submatrix through one cyclic Jacobi sweep in LDS
// (63 rounds of 32 disjoint plane rotations) and stores the accumulated
// orthogonal V_p as E_p = V_p - I (kept exactly: c - 1 = -s^2 / (1 + c));
// jacobi_apply_kernel then forms C <- V^T C V block by block (only pair-blocks
// P <= Q; C is kept as its upper triangle of 32 x 32 blocks) and Y <- Y V as
// corrections,
//   V_P^T C V_Q = C + (C E_Q + E_P^T (C + C E_Q)),   Y V_Q = Y + Y E_Q,
// so that an element is rounded once per round relative to its own size and
// not once per product term; a round without rotations leaves C exact.  A
// rotation is skipped when |c_pq| <= tol sqrt(|c_pp c_qq|); sweeps repeat until
// one skips them all.
#include <algorithm>

#include "gwc_internal.h"

namespace gwc {

namespace {

constexpr int JB = 32;          // Jacobi block size
constexpr int JP = 2 * JB;      // pair submatrix order
constexpr int JLD = JP + 1;     // LDS row stride (bank spread)
constexpr int GT = 64;          // gemm tile
constexpr int GK = 16;          // gemm K chunk
constexpr int JPT = 1024;       // threads of the pair-sweep kernel

// Round-robin (circle) pairing of m items: round r in [0, m-1), slot k in [0, m/2).
__device__ __forceinline__ int2 circle_pair(int m, int r, int k) {
  if (k == 0) return make_int2(r, m - 1);
  return make_int2((r + k) % (m - 1), (r - k + m - 1) % (m - 1));
}

// Global index of row/column t (< 64) of the submatrix of block pair (I, J).
__device__ __forceinline__ int pair_index(int2 IJ, int t) {
  return t < JB ? IJ.x * JB + t : IJ.y * JB + (t - JB);
}

// During the sweeps the symmetric C is kept as its upper triangle of 32 x 32
// blocks: block (X, Y) is stored when X <= Y and a lower block is read through
// its mirror.  The logical 64 x 64 tile with the rows of pair R and the
// columns of pair K is moved as four 32 x 32 sub-blocks; consecutive threads
// touch consecutive addresses in both orientations.
__device__ __forceinline__ void load_pair_tile(const double *__restrict__ C, long long ldc, int2 R,
                                               int2 K, double (*T)[JLD]) {
  for (int e = threadIdx.x; e < JP * JP; e += blockDim.x) {
    const int sub = e / (JB * JB), w = e % (JB * JB);
    const int sa = sub >> 1, sc = sub & 1;
    const int rb = sa ? R.y : R.x, cb = sc ? K.y : K.x;
    const int u = w / JB, v = w % JB;
    if (rb <= cb) T[sa * JB + u][sc * JB + v] = C[(long long)(rb * JB + u) * ldc + cb * JB + v];
    else T[sa * JB + v][sc * JB + u] = C[(long long)(cb * JB + u) * ldc + rb * JB + v];
  }
}

// Writes the logical tile T back into the stored triangle.  For a diagonal
// pair tile (same pair as rows and columns) the lower off-diagonal sub-block
// is left to its mirror and the two diagonal 32-blocks are written symmetrised.
__device__ __forceinline__ void store_pair_tile(double *__restrict__ C, long long ldc, int2 R,
                                                int2 K, bool same, const double (*T)[JLD]) {
  for (int e = threadIdx.x; e < JP * JP; e += blockDim.x) {
    const int sub = e / (JB * JB), w = e % (JB * JB);
    const int sa = sub >> 1, sc = sub & 1;
    const int rb = sa ? R.y : R.x, cb = sc ? K.y : K.x;
    const int u = w / JB, v = w % JB;
    if (rb == cb) {
      const int o = sa * JB;
      C[(long long)(rb * JB + u) * ldc + cb * JB + v] = u <= v ? T[o + u][o + v] : T[o + v][o + u];
    } else if (rb < cb) {
      C[(long long)(rb * JB + u) * ldc + cb * JB + v] = T[sa * JB + u][sc * JB + v];
    } else if (!same) {
      C[(long long)(cb * JB + u) * ldc + rb * JB + v] = T[sa * JB + v][sc * JB + u];
    }
  }
}

}  // namespace

// Column k of the (permuted) transition space is ia = perm[k]:
// Vt[P][k] = 2 sqrt(Delta_ia) M^P_ia and Y[P][k] = sqrt(Delta_ia) M^P_ia for
// k < n_ov, zero for n_ov <= k < ld (the padding).
__global__ void __launch_bounds__(256)
casida_operands_kernel(const double *__restrict__ M_ov, const double *__restrict__ eps,
                       const int *__restrict__ perm, int n_aux, int n_occ, int n_virt, int ld,
                       double *__restrict__ Vt, double *__restrict__ Y) {
  const long long total = (long long)n_aux * ld;
  const int n_ov = n_occ * n_virt;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int P = (int)(e / ld), k = (int)(e % ld);
    double v = 0.0, y = 0.0;
    if (k < n_ov) {
      const int ia = perm[k];
      const int i = ia / n_virt, a = ia % n_virt;
      const double sd = sqrt(eps[n_occ + a] - eps[i]);
      const double m = M_ov[(long long)P * n_ov + ia];
      y = sd * m;
      v = 2.0 * y;
    }
    Vt[e] = v;
    Y[e] = y;
  }
}

// out[i][j] = sum_k A[k][i] B[k][j] (+ diag[i] on the diagonal for i < n_diag
// when diag != NULL), i < M, j < N.  64 x 64 tiles, K in chunks of 16 through
// LDS, 4 x 4 outputs per thread.
__global__ void __launch_bounds__(256)
gemm_tn_kernel(const double *__restrict__ A, long long lda, const double *__restrict__ B,
               long long ldb, int M, int N, int K, double *__restrict__ out, long long ldo,
               const double *__restrict__ diag, int n_diag) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = tid; e < GK * GT; e += 256) {
      const int kk = e / GT, c = e % GT, k = k0 + kk;
      As[kk][c] = (k < K && i0 + c < M) ? A[(long long)k * lda + i0 + c] : 0.0;
      Bs[kk][c] = (k < K && j0 + c < N) ? B[(long long)k * ldb + j0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty + 16 * u];
        b[u] = Bs[kk][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + ty + 16 * u;
    if (i >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + tx + 16 * v;
      if (j >= N) continue;
      double x = acc[u][v];
      if (diag && i == j && i < n_diag) x += diag[i];
      out[(long long)i * ldo + j] = x;
    }
  }
}

// One cyclic Jacobi sweep on the 64 x 64 submatrix of each block pair of round
// r; E_out[pair] receives V - I for the accumulated rotation V (columns = new
// basis) and active[pair] whether any rotation was applied.  Each inner round
// rotates 32 disjoint index pairs: every 2 x 2 block (alpha, beta) of S becomes
// J_alpha^T S_ab J_beta with J = [[c, s], [-s, c]], and E's columns p, q follow
// V's (d = the identity's columns):
//   E_p <- c E_p - s E_q + (c - 1) d_p - s d_q,  E_q <- s E_p + c E_q + s d_p + (c - 1) d_q.
__global__ void __launch_bounds__(JPT)
jacobi_pair_kernel(const double *__restrict__ C, long long ldc, int nb, int r, double tol,
                   double *__restrict__ E_out, int *__restrict__ active, int *__restrict__ rotations) {
  __shared__ double S[JP][JLD];
  __shared__ double V[JP][JLD];  // E = V - I
  __shared__ double rc[JB], rs[JB], rcm1[JB];
  __shared__ int2 rpq[JB];
  __shared__ int nrot_block;
  const int tid = threadIdx.x;
  const int2 IJ = circle_pair(nb, r, blockIdx.x);
  load_pair_tile(C, ldc, IJ, IJ, S);
  for (int e = tid; e < JP * JP; e += JPT) V[e / JP][e % JP] = 0.0;
  if (tid == 0) nrot_block = 0;
  __syncthreads();
  // a submatrix already diagonal to the threshold needs no sweep: E = 0
  int big = 0;
  for (int e = tid; e < JP * JP; e += JPT) {
    const int a = e / JP, b = e % JP;
    const double x = S[a][b];
    big |= a < b && x != 0.0 && fabs(x) > tol * sqrt(fabs(S[a][a] * S[b][b]));
  }
  if (!__syncthreads_or(big)) {
    double *Eo = E_out + (long long)blockIdx.x * JP * JP;
    for (int e = tid; e < JP * JP; e += JPT) Eo[e] = 0.0;
    if (tid == 0) active[blockIdx.x] = 0;
    return;
  }
  int nrot = 0;
  for (int rr = 0; rr < JP - 1; ++rr) {
    if (tid < JB) {
      const int2 pq = circle_pair(JP, rr, tid);
      const double app = S[pq.x][pq.x], aqq = S[pq.y][pq.y], apq = S[pq.x][pq.y];
      double c = 1.0, s = 0.0, cm1 = 0.0;
      if (apq != 0.0 && fabs(apq) > tol * sqrt(fabs(app * aqq))) {
        const double th = (aqq - app) / (2.0 * apq);
        const double t = fabs(th) > 1e100 ? 0.5 / th
                                          : (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
        c = 1.0 / sqrt(1.0 + t * t);
        s = t * c;
        cm1 = -s * s / (1.0 + c);
        ++nrot;
      }
      rc[tid] = c;
      rs[tid] = s;
      rcm1[tid] = cm1;
      rpq[tid] = pq;
    }
    __syncthreads();
    // S: 2 x 2 blocks (alpha, beta), four per thread
    for (int e = tid; e < JB * JB; e += JPT) {
      const int al = e / JB, be = e % JB;
      const int2 pa = rpq[al], pb = rpq[be];
      const double ca = rc[al], sa = rs[al], cb = rc[be], sb = rs[be];
      const double b00 = S[pa.x][pb.x], b01 = S[pa.x][pb.y], b10 = S[pa.y][pb.x], b11 = S[pa.y][pb.y];
      // rows: J_a^T B
      const double r00 = ca * b00 - sa * b10, r01 = ca * b01 - sa * b11;
      const double r10 = sa * b00 + ca * b10, r11 = sa * b01 + ca * b11;
      // columns: (J_a^T B) J_b
      S[pa.x][pb.x] = cb * r00 - sb * r01;
      S[pa.x][pb.y] = sb * r00 + cb * r01;
      S[pa.y][pb.x] = cb * r10 - sb * r11;
      S[pa.y][pb.y] = sb * r10 + cb * r11;
    }
    // E: columns p, q of every row, eight per thread
    for (int e = tid; e < JB * JP; e += JPT) {
      const int be = e / JP, row = e % JP;
      const int2 pq = rpq[be];
      const double c = rc[be], s = rs[be], cm1 = rcm1[be];
      const double dp = row == pq.x ? 1.0 : 0.0, dq = row == pq.y ? 1.0 : 0.0;
      const double vx = V[row][pq.x], vy = V[row][pq.y];
      V[row][pq.x] = (c * vx - s * vy) + (cm1 * dp - s * dq);
      V[row][pq.y] = (s * vx + c * vy) + (s * dp + cm1 * dq);
    }
    __syncthreads();
  }
  if (tid < JB && nrot) atomicAdd(&nrot_block, nrot);
  double *Eo = E_out + (long long)blockIdx.x * JP * JP;
  for (int e = tid; e < JP * JP; e += JPT) Eo[e] = V[e / JP][e % JP];
  __syncthreads();
  if (tid == 0) {
    active[blockIdx.x] = nrot_block > 0;
    if (nrot_block) atomicAdd(rotations, nrot_block);
  }
}

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// 64 x 64 x 64 products on FP64 MFMA (v_mfma_f64_16x16x4f64) with one operand
// a 64 x 64 tile in LDS and the other a rotation correction E (row-major
// 64 x 64, read straight from L2: every tile of a round shares it):
//   prod_tile_e:  out = X E        (X in LDS)
//   prod_et_tile: out = E^T X      (X in LDS)
// Wave w owns the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 MFMA tiles.  Operand
// layout: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; element r of
// lane l's accumulator is D[4 r + l / 16][l % 16].
__device__ __forceinline__ void prod_tile_e(const double (*X)[JLD], const double *__restrict__ E,
                                            int wave, int lane, d4 acc[2][2]) {
  const int li = lane & 15, lk = lane >> 4;
  const int qr = (wave >> 1) * 32, qc = (wave & 1) * 32;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < JP; k0 += 4) {
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = X[qr + 16 * t + li][k0 + lk];
      b[t] = E[(k0 + lk) * JP + qc + 16 * t + li];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
  }
}

__device__ __forceinline__ void prod_et_tile(const double *__restrict__ E, const double (*X)[JLD],
                                             int wave, int lane, d4 acc[2][2]) {
  const int li = lane & 15, lk = lane >> 4;
  const int qr = (wave >> 1) * 32, qc = (wave & 1) * 32;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < JP; k0 += 4) {
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = E[(k0 + lk) * JP + qr + 16 * t + li];
      b[t] = X[k0 + lk][qc + 16 * t + li];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
  }
}

// Position of accumulator element (t, u, r) of this lane in the 64 x 64 tile.
__device__ __forceinline__ int acc_row(int wave, int lane, int t, int r) {
  return (wave >> 1) * 32 + 16 * t + 4 * r + (lane >> 4);
}
__device__ __forceinline__ int acc_col(int wave, int lane, int u) {
  return (wave & 1) * 32 + 16 * u + (lane & 15);
}

}  // namespace

// Round r's rotations applied to C (pair-blocks P <= Q, each 32-block written
// once into the stored triangle) and to Y (64-row tiles), from E = V - I:
//   C_PQ <- C_PQ + (T + E_P^T (C_PQ + T)),  T = C_PQ E_Q;   Y <- Y + Y E_Q.
// Blocks [0, np*np) handle C, the next n_ytiles * np handle Y; blocks whose
// pairs applied no rotation leave their tile untouched.
__global__ void __launch_bounds__(256)
jacobi_apply_kernel(double *__restrict__ C, long long ldc, int nb, int r,
                    const double *__restrict__ Ep, const int *__restrict__ active,
                    double *__restrict__ Y, long long ldy, int n_aux, int *__restrict__ work) {
  __shared__ double X[JP][JLD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int np = nb / 2;
  int b = blockIdx.x;
  d4 acc[2][2];
  if (b < np * np) {
    const int P = b / np, Q = b % np;
    // no rotation in either pair: V_P = V_Q = I exactly and C_PQ is unchanged
    if (P > Q || (!active[P] && !active[Q])) return;
    if (tid == 0) atomicAdd(&work[0], 1);
    const int2 IP = circle_pair(nb, r, P), IQ = circle_pair(nb, r, Q);
    const double *EQ = Ep + (long long)Q * JP * JP, *EP = Ep + (long long)P * JP * JP;
    load_pair_tile(C, ldc, IP, IQ, X);
    __syncthreads();
    prod_tile_e(X, EQ, wave, lane, acc);  // T = C_PQ E_Q
    double own[2][2][4], tpart[2][2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          own[t][u][q] = X[acc_row(wave, lane, t, q)][acc_col(wave, lane, u)];
          tpart[t][u][q] = acc[t][u][q];
        }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          X[acc_row(wave, lane, t, q)][acc_col(wave, lane, u)] = own[t][u][q] + tpart[t][u][q];
    __syncthreads();
    prod_et_tile(EP, X, wave, lane, acc);  // E_P^T (C_PQ V_Q)
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          X[acc_row(wave, lane, t, q)][acc_col(wave, lane, u)] =
              own[t][u][q] + (tpart[t][u][q] + acc[t][u][q]);
    __syncthreads();
    store_pair_tile(C, ldc, IP, IQ, P == Q, X);
    return;
  }
  b -= np * np;
  const int yt = b / np, Q = b % np;
  if (!active[Q]) return;
  if (tid == 0) atomicAdd(&work[1], 1);
  const int y0 = yt * JP;
  const int2 IQ = circle_pair(nb, r, Q);
  const double *EQ = Ep + (long long)Q * JP * JP;
  for (int e = tid; e < JP * JP; e += 256) {
    const int a = e / JP, c = e % JP;
    X[a][c] = (y0 + a < n_aux) ? Y[(long long)(y0 + a) * ldy + pair_index(IQ, c)] : 0.0;
  }
  __syncthreads();
  prod_tile_e(X, EQ, wave, lane, acc);  // Y_tile E_Q
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int lr = acc_row(wave, lane, t, q), row = y0 + lr;
      if (row >= n_aux) continue;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int lc = acc_col(wave, lane, u);
        Y[(long long)row * ldy + pair_index(IQ, lc)] = X[lr][lc] + acc[t][u][q];
      }
    }
}

__global__ void zero_counter_kernel(int *__restrict__ x, int n) {
  if ((int)threadIdx.x < n) x[threadIdx.x] = 0;
}

// Omega_nu = sqrt(C_nu,nu) for nu < n (1 for the padding); omega_sorted gets
// them in ascending order (rank by counting; ties by index).
__global__ void __launch_bounds__(256)
excitations_kernel(const double *__restrict__ C, long long ldc, int n, int n_pad,
                   double *__restrict__ Om) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_pad) return;
  Om[v] = v < n ? sqrt(C[(long long)v * ldc + v]) : 1.0;
}

__global__ void __launch_bounds__(256)
rank_sort_kernel(const double *__restrict__ Om, int n, double *__restrict__ sorted) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double x = Om[v];
  int rank = 0;
  for (int u = 0; u < n; ++u) {
    const double y = Om[u];
    rank += (y < x) || (y == x && u < v);
  }
  sorted[rank] = x;
}

// Bp[P][c nb + m] = M^P_{n_c m} (m < n_occ from M_oo, else M_ov).
__global__ void __launch_bounds__(256)
pack_pairs_kernel(const double *__restrict__ M_oo, const double *__restrict__ M_ov, int n_aux,
                  int n_occ, int n_virt, const int *__restrict__ core, int n_core,
                  double *__restrict__ Bp) {
  const int nb = n_occ + n_virt, cols = n_core * nb;
  const long long total = (long long)n_aux * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int P = (int)(e / cols), cm = (int)(e % cols), c = cm / nb, m = cm % nb;
    const int n = core[c];
    Bp[e] = m < n_occ ? M_oo[((long long)P * n_occ + n) * n_occ + m]
                      : M_ov[((long long)P * n_occ + n) * n_virt + (m - n_occ)];
  }
}

// Partial pole sums of Eq. sigma_spectral over the excitations of one block of
// 64 (blockIdx.x) for core c (blockIdx.y) at points j (blockIdx.z * 256 + tid):
// point j < n_real is omega_real[c][j], j = n_real is eps_{n_c}.
//   term = rho^2 / (a - i s eta), a = w - eps_m + s Omega, s = +1 (occupied m) / -1,
//   rho^2 = 2 Q[r + m][nu]^2 / Omega_nu, or Q[r + m][nu] itself when `squared`;
//   row base r = c nb, or row_state[c] nb when row_state is given.
// eps holds the energies in G (eps_m); point n_real is w = eps[core[c]].
__global__ void __launch_bounds__(256)
pole_sum_kernel(const double *__restrict__ Q, long long ldq, const double *__restrict__ Om, int n_ov,
                const double *__restrict__ eps, int n_occ, int n_basis,
                const int *__restrict__ core, const double *__restrict__ omega_real, int n_real,
                double eta, int squared, const int *__restrict__ row_state,
                double2 *__restrict__ part) {
  constexpr int MB = 16, VB = 64;
  __shared__ double r2[MB][VB + 1];
  __shared__ double oms[VB];
  const int tid = threadIdx.x;
  const int v0 = blockIdx.x * VB, c = blockIdx.y, n_core = gridDim.y;
  const int npts = n_real + 1;
  const int j = blockIdx.z * 256 + tid;
  const double w = j < n_real ? omega_real[(long long)c * n_real + j] : eps[core[c]];
  const double eta2 = eta * eta;
  if (tid < VB) oms[tid] = v0 + tid < n_ov ? Om[v0 + tid] : 1.0;
  double re = 0.0, im = 0.0;
  for (int m0 = 0; m0 < n_basis; m0 += MB) {
    __syncthreads();
    for (int e = tid; e < MB * VB; e += 256) {
      const int mm = e / VB, v = e % VB, m = m0 + mm, nu = v0 + v;
      double x = 0.0;
      if (m < n_basis && nu < n_ov) {
        const long long r0 = (long long)(row_state ? row_state[c] : c) * n_basis;
        const double q = Q[(r0 + m) * ldq + nu];
        x = squared ? q : 2.0 * q * q / Om[nu];
      }
      r2[mm][v] = x;
    }
    __syncthreads();
    const int mend = min(MB, n_basis - m0);
    for (int mm = 0; mm < mend; ++mm) {
      const int m = m0 + mm;
      const double sg = m < n_occ ? 1.0 : -1.0;
      const double a0 = w - eps[m];
      double sre = 0.0, sim = 0.0;
#pragma unroll 8
      for (int v = 0; v < VB; ++v) {
        const double a = a0 + sg * oms[v];
        const double inv = r2[mm][v] / (a * a + eta2);
        sre = fma(a, inv, sre);
        sim += inv;
      }
      re += sre;
      im += sg * eta * sim;
    }
  }
  if (j < npts) part[((long long)blockIdx.x * n_core + c) * npts + j] = make_double2(re, im);
}

// sigma[c][j] = sum over excitation blocks of the partial sums (fixed order).
__global__ void __launch_bounds__(256)
pole_reduce_kernel(const double2 *__restrict__ part, int n_blocks, int n_core, int npts,
                   double2 *__restrict__ sigma) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_core * npts) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < n_blocks; ++b) {
    const double2 x = part[(long long)b * n_core * npts + e];
    re += x.x;
    im += x.y;
  }
  sigma[e] = make_double2(re, im);
}

// E_QP (Eq. QPGWC), Sigma^c outputs and the spectral functions of Eq.
// A_explicit_real_imaginary: A^G0W0 at w_j and A^{G_DH W0} at w_j + DH_n.
__global__ void __launch_bounds__(256)
analytic_finish_kernel(const double2 *__restrict__ sigma, int n_real, const double *__restrict__ eps,
                       const int *__restrict__ core, const double *__restrict__ omega_real,
                       const double *__restrict__ sigma_x, const double *__restrict__ vxc,
                       double *__restrict__ sigma_c, double *__restrict__ sigma_c_eps,
                       double *__restrict__ e_qp, double *__restrict__ a_gw,
                       double *__restrict__ a_dh) {
  const int c = blockIdx.x, npts = n_real + 1;
  const double en = eps[core[c]], sx = sigma_x[c], vx = vxc[c];
  const double2 se = sigma[(long long)c * npts + n_real];
  const double eqp = en + sx + se.x - vx;
  const double dh = eqp - en;
  const double PI_D = 3.14159265358979323846;
  if (threadIdx.x == 0) {
    e_qp[c] = eqp;
    sigma_c_eps[2 * c] = se.x;
    sigma_c_eps[2 * c + 1] = se.y;
  }
  for (int j = threadIdx.x; j < n_real; j += blockDim.x) {
    const double2 s = sigma[(long long)c * npts + j];
    const double w = omega_real[(long long)c * n_real + j];
    sigma_c[((long long)c * n_real + j) * 2] = s.x;
    sigma_c[((long long)c * n_real + j) * 2 + 1] = s.y;
    const double re = w - en + vx - sx - s.x, im2 = s.y * s.y;
    a_gw[(long long)c * n_real + j] = fabs(s.y) / (PI_D * (re * re + im2));
    const double rd = re + dh;
    a_dh[(long long)c * n_real + j] = fabs(s.y) / (PI_D * (rd * rd + im2));
  }
}

// ---------------------------------------------------------------------------
// Launchers

void launch_casida_operands(const double *M_ov, const double *eps, const int *perm, int n_aux,
                            int n_occ, int n_virt, int ld, double *Vt, double *Y, hipStream_t s) {
  const long long total = (long long)n_aux * ld;
  const int grid = (int)std::min<long long>((total + 255) / 256, 65536);
  casida_operands_kernel<<<grid, 256, 0, s>>>(M_ov, eps, perm, n_aux, n_occ, n_virt, ld, Vt, Y);
}

void launch_gemm_tn(const double *A, long long lda, const double *B, long long ldb, int M, int N,
                    int K, double *out, long long ldo, const double *diag, int n_diag,
                    hipStream_t s) {
  if (M < 1 || N < 1) return;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  gemm_tn_kernel<<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, out, ldo, diag, n_diag);
}

int jacobi_block() { return JB; }

void launch_zero_counters(int *x, int n, hipStream_t s) { zero_counter_kernel<<<1, 64, 0, s>>>(x, n); }

void launch_jacobi_pairs(const double *C, long long ldc, int nb, int r, double tol, double *Ep,
                         int *active, int *rotations, hipStream_t s) {
  jacobi_pair_kernel<<<nb / 2, JPT, 0, s>>>(C, ldc, nb, r, tol, Ep, active, rotations);
}

void launch_jacobi_apply(double *C, long long ldc, int nb, int r, const double *Ep,
                         const int *active, double *Y, long long ldy, int n_aux, int *work,
                         hipStream_t s) {
  const int np = nb / 2, ytiles = (n_aux + JP - 1) / JP;
  jacobi_apply_kernel<<<np * np + ytiles * np, 256, 0, s>>>(C, ldc, nb, r, Ep, active, Y, ldy,
                                                            n_aux, work);
}

void launch_excitations(const double *C, long long ldc, int n, int n_pad, double *Om,
                        double *sorted, hipStream_t s) {
  excitations_kernel<<<(n_pad + 255) / 256, 256, 0, s>>>(C, ldc, n, n_pad, Om);
  if (sorted) rank_sort_kernel<<<(n + 255) / 256, 256, 0, s>>>(Om, n, sorted);
}

void launch_pack_pairs(const double *M_oo, const double *M_ov, int n_aux, int n_occ, int n_virt,
                       const int *core, int n_core, double *Bp, hipStream_t s) {
  const long long total = (long long)n_aux * n_core * (n_occ + n_virt);
  const int grid = (int)std::min<long long>((total + 255) / 256, 65536);
  pack_pairs_kernel<<<grid, 256, 0, s>>>(M_oo, M_ov, n_aux, n_occ, n_virt, core, n_core, Bp);
}

int pole_sum_blocks(int n_ov) { return (n_ov + 63) / 64; }

void launch_pole_sum(const double *Q, long long ldq, const double *Om, int n_ov, const double *eps,
                     int n_occ, int n_basis, const int *core, int n_core, const double *omega_real,
                     int n_real, double eta, int squared, const int *row_state, double2 *part,
                     double2 *sigma, hipStream_t s) {
  const int nblk = pole_sum_blocks(n_ov), npts = n_real + 1;
  dim3 grid(nblk, n_core, (npts + 255) / 256);
  pole_sum_kernel<<<grid, 256, 0, s>>>(Q, ldq, Om, n_ov, eps, n_occ, n_basis, core, omega_real,
                                       n_real, eta, squared, row_state, part);
  pole_reduce_kernel<<<(n_core * npts + 255) / 256, 256, 0, s>>>(part, nblk, n_core, npts, sigma);
}

void launch_analytic_finish(const double2 *sigma, int n_core, int n_real, const double *eps,
                            const int *core, const double *omega_real, const double *sigma_x,
                            const double *vxc, double *sigma_c, double *sigma_c_eps, double *e_qp,
                            double *a_gw, double *a_dh, hipStream_t s) {
  analytic_finish_kernel<<<n_core, 256, 0, s>>>(sigma, n_real, eps, core, omega_real, sigma_x, vxc,
                                                sigma_c, sigma_c_eps, e_qp, a_gw, a_dh);
}

}  // namespace gwc
