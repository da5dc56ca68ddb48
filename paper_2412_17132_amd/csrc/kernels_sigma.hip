// Border vectors, exchange, the imaginary-axis quadrature and the assembly of
// Sigma^c = -I + R with the quasiparticle energy.  These kernels are small next
// to the Pi build and the LU; all reductions run in a fixed order so results
// do not depend on scheduling.
#include "gwc_internal.h"

namespace gwc {

constexpr double PI_D = 3.14159265358979323846;

// Deterministic sum over a 256-thread block (fixed tree).
__device__ double block_sum_256(double v, double *sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// b_nm = M^P_nm for an occupied n and any m (occupied first).
__device__ __forceinline__ double pair_coef(const double *M_oo, const double *M_ov, int n_occ,
                                            int n_virt, int P, int n, int m) {
  return (m < n_occ) ? M_oo[((long long)P * n_occ + n) * n_occ + m]
                     : M_ov[((long long)P * n_occ + n) * n_virt + (m - n_occ)];
}

// Border of the bordered matrix: column N + r and row N + r hold b_r, the
// border-border block is zero; bb[f][r] = b_r^T b_r.  Grid (R, F).
__global__ void __launch_bounds__(256)
border_kernel(const double *__restrict__ M_oo, const double *__restrict__ M_ov, int n_aux,
              int n_occ, int n_virt, const int *__restrict__ task_n, const int *__restrict__ task_m,
              int R, double2 *__restrict__ G, long long g_stride, int ldg, double *__restrict__ bb) {
  __shared__ double sh[256];
  const int r = blockIdx.x, f = blockIdx.y, tid = threadIdx.x;
  const int n = task_n[f];
  const int m = task_m[f] >= 0 ? task_m[f] : r;
  double2 *A = G + (long long)f * g_stride;
  const int N = n_aux;
  double acc = 0.0;
  for (int P = tid; P < N; P += 256) {
    const double b = pair_coef(M_oo, M_ov, n_occ, n_virt, P, n, m);
    A[(long long)P * ldg + N + r] = make_double2(b, 0.0);
    A[(long long)(N + r) * ldg + P] = make_double2(b, 0.0);
    acc += b * b;
  }
  for (int q = tid; q < R; q += 256) A[(long long)(N + r) * ldg + N + q] = make_double2(0.0, 0.0);
  const double s = block_sum_256(acc, sh);
  if (tid == 0) bb[(long long)f * R + r] = s;
}

void launch_border(const double *M_oo, const double *M_ov, int n_aux, int n_occ, int n_virt,
                   const int *task_n, const int *task_m, int F, int R, double2 *G,
                   long long g_stride, int ldg, double *bb, hipStream_t stream) {
  dim3 grid(R, F);
  border_kernel<<<grid, 256, 0, stream>>>(M_oo, M_ov, n_aux, n_occ, n_virt, task_n, task_m, R, G,
                                          g_stride, ldg, bb);
}

// Sigma^x_n = -sum_{i occ} sum_P (M^P_ni)^2  (exchange over occupied orbitals).
__global__ void __launch_bounds__(256)
sigma_x_kernel(const double *__restrict__ M_oo, int n_aux, int n_occ,
               const int *__restrict__ core_idx, double *__restrict__ sigma_x) {
  __shared__ double sh[256];
  const int c = blockIdx.x, n = core_idx[c];
  double acc = 0.0;
  const long long total = (long long)n_aux * n_occ;
  for (long long idx = threadIdx.x; idx < total; idx += 256) {
    const int P = (int)(idx / n_occ), i = (int)(idx - (long long)P * n_occ);
    const double v = M_oo[((long long)P * n_occ + n) * n_occ + i];
    acc += v * v;
  }
  const double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) sigma_x[c] = -s;
}

void launch_sigma_x(const double *M_oo, int n_aux, int n_occ, const int *core_idx, int n_core,
                    double *sigma_x, hipStream_t stream) {
  sigma_x_kernel<<<n_core, 256, 0, stream>>>(M_oo, n_aux, n_occ, core_idx, sigma_x);
}

// I_n(w) = (1/pi) sum_k w_k sum_m W^c_nm(i w_k) a / (a^2 + w_k^2), a = w - eps_m.
// Grid (n_real + 1, n_core); point j = n_real is w = eps_n.  When
// grid_points == 1 only the eps_n point is evaluated.
__global__ void __launch_bounds__(256)
quadrature_kernel(const double2 *__restrict__ W_imag, const double *__restrict__ eps, int n_basis,
                  const double *__restrict__ omega_imag, const double *__restrict__ w_imag,
                  int n_imag, const double *__restrict__ omega_real, int n_real,
                  const int *__restrict__ core_idx, int grid_points, double *__restrict__ I_out) {
  __shared__ double sh[256];
  const int c = blockIdx.y;
  const int j = (grid_points == 1) ? n_real : blockIdx.x;
  const int n = core_idx[c];
  const double omega = (j < n_real) ? omega_real[(long long)c * n_real + j] : eps[n];
  const long long total = (long long)n_basis * n_imag;
  double acc = 0.0;
  for (long long idx = threadIdx.x; idx < total; idx += 256) {
    const int m = (int)(idx / n_imag), k = (int)(idx - (long long)m * n_imag);
    const double a = omega - eps[m];
    const double wk = omega_imag[k];
    acc += w_imag[k] * W_imag[((long long)c * n_basis + m) * n_imag + k].x * (a / (a * a + wk * wk));
  }
  const double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) I_out[(long long)c * (n_real + 1) + j] = s / PI_D;
}

void launch_quadrature(const double2 *W_imag, const double *eps, int n_basis,
                       const double *omega_imag, const double *w_imag, int n_imag,
                       const double *omega_real, int n_real, const int *core_idx, int n_core,
                       int grid_points, double *I_out, hipStream_t stream) {
  dim3 grid(grid_points, n_core);
  quadrature_kernel<<<grid, 256, 0, stream>>>(W_imag, eps, n_basis, omega_imag, w_imag, n_imag,
                                              omega_real, n_real, core_idx, grid_points, I_out);
}

// Residue sum and assembly, one thread per (core, point).  Tasks of a point
// are contiguous and ordered by m, so the sum order is fixed.
__global__ void assemble_kernel(const double2 *__restrict__ W_real, const double *__restrict__ f_task,
                                const int *__restrict__ cj_offset, const int *__restrict__ task_dec,
                                const double *__restrict__ I, int n_core, int n_real,
                                const double *__restrict__ eps, const int *__restrict__ core_idx,
                                const double *__restrict__ sigma_x, const double *__restrict__ vxc,
                                int full, double *__restrict__ sigma_c, double *__restrict__ im_dec,
                                double *__restrict__ sigma_c_eps, double *__restrict__ e_qp) {
  const int cj = blockIdx.x * blockDim.x + threadIdx.x;
  const int npts = n_real + 1;
  if (cj >= n_core * npts) return;
  const int c = cj / npts, j = cj - c * npts;
  // residue sum in m order; Im Sigma^dec over the equivalent set's terms
  double rr = 0.0, ri = 0.0, imd = 0.0;
  for (int t = cj_offset[cj]; t < cj_offset[cj + 1]; ++t) {
    rr += f_task[t] * W_real[t].x;
    ri += f_task[t] * W_real[t].y;
    if (task_dec[t]) imd += f_task[t] * W_real[t].y;
  }
  if (j < n_real) {
    if (full) {
      const double Iv = I[(long long)c * npts + j];
      sigma_c[2 * ((long long)c * n_real + j)] = -Iv + rr;
      sigma_c[2 * ((long long)c * n_real + j) + 1] = ri;
    }
    im_dec[(long long)c * n_real + j] = imd;
  } else {
    const double Iv = I[(long long)c * npts + j];
    const double sr = -Iv + rr;
    sigma_c_eps[2 * c] = sr;
    sigma_c_eps[2 * c + 1] = ri;
    e_qp[c] = eps[core_idx[c]] + sigma_x[c] + sr - vxc[c];
  }
}

void launch_assemble(const double2 *W_real, const double *f_task, const int *task_dec,
                     const int *cj_offset, const double *I, int n_core,
                     int n_real, const double *eps, const int *core_idx, const double *sigma_x,
                     const double *vxc, int full, double *sigma_c, double *im_dec,
                     double *sigma_c_eps, double *e_qp, hipStream_t stream) {
  const int total = n_core * (n_real + 1);
  assemble_kernel<<<(total + 63) / 64, 64, 0, stream>>>(W_real, f_task, cj_offset, task_dec, I,
                                                        n_core, n_real, eps, core_idx, sigma_x,
                                                        vxc, full, sigma_c, im_dec, sigma_c_eps,
                                                        e_qp);
}

// Count of non-finite values (for input validation of device-resident arrays).
__global__ void nonfinite_kernel(const double *__restrict__ x, long long n, int *__restrict__ flag) {
  int bad = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) atomicOr(flag, 1);
}

void launch_nonfinite(const double *x, long long n, int *flag, hipStream_t stream) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  nonfinite_kernel<<<(unsigned)blocks, 256, 0, stream>>>(x, n, flag);
}

}  // namespace gwc
