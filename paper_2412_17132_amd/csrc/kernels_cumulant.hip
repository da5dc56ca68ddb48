// GW+C tail: the numerical Landau cumulant on the time grid, the cumulant
// propagator, the FFT to frequency and the spectral function.
//
//   c_j   = q_j |Im Sigma_j| / (pi nu_j^2),  nu_j = w_j - eps_n   (c_j = 0 at nu_j = 0)
//   C~(t) = sum_j c_j (e^{-i nu_j t} - 1)                  (Eq. landau_cumulant_truncated)
//   G(t)  = -i theta(t) e^{-i E_QP t - eta t} e^{C~(t)}    (Eq. cumulant_propagator_numerical_time)
//   G(w_l) = dt sum_k G(t_k) e^{i w_l t_k}                 (Eqs. cumulant_propagator_fourier,
//                                                          cumulant_propagator_convolution)
//   A(w)  = -Im G(w) / pi                                  (Eq. eq:AGWC)
//
// With w_l = w_0 + l d_omega and dt = 2 pi / (n_t d_omega) the sum over k is an
// inverse DFT of G(t_k) e^{i w_0 t_k}; the factor e^{i w_0 t_k} and dt are
// folded into the time-domain kernel.  The cumulant loop is ALU-bound
// (n_t x n_real complex exponentials); the FFT is a radix-2 Stockham.
#include "gwc_internal.h"

namespace gwc {

constexpr double PI_D = 3.14159265358979323846;

// One block: trapezoid weights, nu_j, c_j, and (Z, 1 - Z).
__global__ void __launch_bounds__(256)
cumulant_weights_kernel(const double *__restrict__ w, const double *__restrict__ im, int n_real,
                        double eps_n, double *__restrict__ nu, double *__restrict__ c,
                        double *__restrict__ z_out) {
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int j = tid; j < n_real; j += 256) {
    double q = 0.0;
    if (n_real > 1) {
      if (j > 0) q += 0.5 * (w[j] - w[j - 1]);
      if (j < n_real - 1) q += 0.5 * (w[j + 1] - w[j]);
    }
    const double v = w[j] - eps_n;
    const double g = fabs(im[j]) / PI_D;
    const double cj = (v != 0.0) ? q * g / (v * v) : 0.0;
    nu[j] = v;
    c[j] = cj;
    acc += cj;
  }
  sh[tid] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  if (tid == 0 && z_out) {
    const double Z = exp(-sh[0]);
    z_out[0] = Z;
    z_out[1] = 1.0 - Z;
  }
}

void launch_cumulant_weights(const double *omega_real, const double *im_sigma, int n_real,
                             double eps_n, double *nu, double *c, double *z_out,
                             hipStream_t stream) {
  cumulant_weights_kernel<<<1, 256, 0, stream>>>(omega_real, im_sigma, n_real, eps_n, nu, c,
                                                 z_out);
}

// One thread per time point; nu and c are staged through LDS in chunks.
constexpr int CT_CHUNK = 512;
__global__ void __launch_bounds__(256)
cumulant_time_kernel(const double *__restrict__ nu, const double *__restrict__ c, int n_real,
                     int n_t, double dt, double e_qp, double omega0, double eta,
                     double2 *__restrict__ Gt) {
  __shared__ double snu[CT_CHUNK], sc[CT_CHUNK];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const double t = (double)k * dt;
  double cr = 0.0, ci = 0.0;
  for (int j0 = 0; j0 < n_real; j0 += CT_CHUNK) {
    const int nj = min(CT_CHUNK, n_real - j0);
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
      snu[j] = nu[j0 + j];
      sc[j] = c[j0 + j];
    }
    __syncthreads();
    for (int j = 0; j < nj; ++j) {
      double s, co;
      sincos(snu[j] * t, &s, &co);
      cr += sc[j] * (co - 1.0);
      ci -= sc[j] * s;
    }
    __syncthreads();
  }
  if (k >= n_t) return;
  const double theta = (k == 0) ? 0.5 : 1.0;
  const double mag = theta * dt * exp(cr - eta * t);
  const double phi = ci - (e_qp - omega0) * t;
  double s, co;
  sincos(phi, &s, &co);
  // -i * mag * (cos phi + i sin phi)
  Gt[k] = make_double2(mag * s, -mag * co);
}

void launch_cumulant_time(const double *nu, const double *c, int n_real, int n_t, double dt,
                          double e_qp, double omega0, double eta, double2 *Gt,
                          hipStream_t stream) {
  cumulant_time_kernel<<<(n_t + 255) / 256, 256, 0, stream>>>(nu, c, n_real, n_t, dt, e_qp,
                                                              omega0, eta, Gt);
}

// One radix-2 Stockham pass of the unnormalised inverse DFT (e^{+2 pi i l k / n}).
__global__ void fft_pass_kernel(const double2 *__restrict__ in, double2 *__restrict__ out, int half,
                                int m) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= half) return;
  const int k = j & (m - 1);
  double s, co;
  sincospi((double)k / (double)m, &s, &co);
  const double2 u = in[j];
  const double2 x = in[j + half];
  const double2 v = make_double2(x.x * co - x.y * s, x.x * s + x.y * co);
  const int o = ((j - k) << 1) + k;
  out[o] = make_double2(u.x + v.x, u.y + v.y);
  out[o + m] = make_double2(u.x - v.x, u.y - v.y);
}

void launch_fft_inverse(double2 *buf_a, double2 *buf_b, int log2n, double2 **result,
                        hipStream_t stream) {
  const int n = 1 << log2n, half = n >> 1;
  double2 *in = buf_a, *out = buf_b;
  for (int s = 0; s < log2n; ++s) {
    fft_pass_kernel<<<(half + 255) / 256, 256, 0, stream>>>(in, out, half, 1 << s);
    double2 *t = in;
    in = out;
    out = t;
  }
  *result = in;
}

__global__ void extract_kernel(const double2 *__restrict__ Gw, int n_out, double *__restrict__ A) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n_out) A[l] = -Gw[l].y / PI_D;
}

void launch_extract_spectrum(const double2 *Gw, int n_out, double *A_out, hipStream_t stream) {
  extract_kernel<<<(n_out + 255) / 256, 256, 0, stream>>>(Gw, n_out, A_out);
}

}  // namespace gwc
