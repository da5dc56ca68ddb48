// CD-WAC: W^c_nm continued analytically by a Pade approximant in continued-
// fraction form (paper section "Numerical GW+C scheme", Eq. pade_approximation)
//
//   W(z) ~ a_1 / (1 + a_2 (z - z_1) / (1 + a_3 (z - z_2) / (1 + ...)))
//
// fitted through reference points z_1..z_P by Thiele's reciprocal differences
//   g_1(z_j) = W(z_j),
//   g_p(z_j) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_j)) / ((z_j - z_{p-1}) g_{p-1}(z_j)),
//   a_p = g_p(z_p),
// and evaluated at every residue argument |eps_m - w| + i eta.
#include "gwc_internal.h"

namespace gwc {

namespace {

__device__ __forceinline__ double2 wmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 wsub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
// a / b with scaling by the larger component of b (Smith)
__device__ __forceinline__ double2 wdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return make_double2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}

}  // namespace

// One wave per pair.  pair = (c, m, j0, P): its nodes are node_z[off .. off+P)
// (the n_imag imaginary nodes, then its window's real points); its values are
// W_imag[(c nb + m) ni + k] for k < ni and W_ref[(c R_w + m) n_rr + j0 + j].
// The recursion overwrites g in place; a_p is g[p] once step p is done.
__global__ void __launch_bounds__(64)
pade_fit_kernel(const int4 *__restrict__ pairs, const long long *__restrict__ node_off,
                const double2 *__restrict__ node_z, const double2 *__restrict__ W_imag, int nb,
                int ni, const double2 *__restrict__ W_ref, int R_w, int n_rr,
                double2 *__restrict__ coef, int *__restrict__ status) {
  __shared__ double2 g[WAC_MAX_NODES];
  __shared__ double2 zs[WAC_MAX_NODES];
  const int p = blockIdx.x, lane = threadIdx.x;
  const int4 pr = pairs[p];
  const int c = pr.x, m = pr.y, j0 = pr.z, P = pr.w;
  const long long off = node_off[p];
  for (int j = lane; j < P; j += 64) {
    zs[j] = node_z[off + j];
    g[j] = j < ni ? W_imag[((long long)c * nb + m) * ni + j]
                  : W_ref[((long long)c * R_w + m) * n_rr + j0 + (j - ni)];
  }
  __syncthreads();
  for (int q = 1; q < P; ++q) {
    const double2 prev = g[q - 1], zp = zs[q - 1];
    for (int j = q + lane; j < P; j += 64) g[j] = wdiv(wsub(prev, g[j]), wmul(wsub(zs[j], zp), g[j]));
    __syncthreads();
  }
  int bad = 0;
  for (int j = lane; j < P; j += 64) {
    coef[off + j] = g[j];
    bad |= !(isfinite(g[j].x) && isfinite(g[j].y));
  }
  if (bad) atomicOr(status, 1);
}

// One thread per residue task: W = a_1 / t, t from the innermost level out,
// t = 1 + a_P (z - z_{P-1}), then t = 1 + a_p (z - z_{p-1}) / t.
__global__ void __launch_bounds__(256)
pade_eval_kernel(const double2 *__restrict__ z_task, const int *__restrict__ pair_of_task,
                 const int4 *__restrict__ pairs, const long long *__restrict__ node_off,
                 const double2 *__restrict__ node_z, const double2 *__restrict__ coef, int T,
                 double2 *__restrict__ W_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int p = pair_of_task[t];
  const long long off = node_off[p];
  const int P = pairs[p].w;
  const double2 z = z_task[t];
  double2 acc = make_double2(1.0, 0.0);
  for (int q = P - 1; q >= 1; --q) {
    const double2 u = wdiv(wmul(coef[off + q], wsub(z, node_z[off + q - 1])), acc);
    acc = make_double2(1.0 + u.x, u.y);
  }
  W_out[t] = wdiv(coef[off], acc);
}

void launch_pade_fit(const int4 *pairs, int n_pairs, const long long *node_off,
                     const double2 *node_z, const double2 *W_imag, int nb, int ni,
                     const double2 *W_ref, int R_w, int n_rr, double2 *coef, int *status,
                     hipStream_t stream) {
  if (n_pairs < 1) return;
  pade_fit_kernel<<<n_pairs, 64, 0, stream>>>(pairs, node_off, node_z, W_imag, nb, ni, W_ref, R_w,
                                              n_rr, coef, status);
}

void launch_pade_eval(const double2 *z_task, const int *pair_of_task, const int4 *pairs,
                      const long long *node_off, const double2 *node_z, const double2 *coef,
                      int T, double2 *W_out, hipStream_t stream) {
  if (T < 1) return;
  pade_eval_kernel<<<(T + 255) / 256, 256, 0, stream>>>(z_task, pair_of_task, pairs, node_off,
                                                        node_z, coef, T, W_out);
}

}  // namespace gwc
