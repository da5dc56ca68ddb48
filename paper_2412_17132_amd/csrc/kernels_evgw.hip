// evGW0 (paper section "GW for core levels: beyond G0W0", Eq. ev_sigma_spectral):
// the quasiparticle energies of every state are iterated with the current
// energies in G, while Omega^nu and rho^nu_nm stay those of the RPA on the
// mean-field energies (the analytic route's eigensolve, kernels_analytic.hip).
//
//   Sigma^c,ev_n(w; e) = sum_{m,nu} (rho^nu_nm)^2 / (w - e_m + (Omega^nu - i eta) s_m),
//   s_m = +1 for occupied, -1 for virtual m (mean-field occupations).
//
// ev_solve_kernel: one workgroup per state n solves f(E) = E - eps_n -
// Sigma^x_n - Re Sigma^c,ev_n(E; e) + v^xc_n = 0 from E0 = e_n: points
// E0 + d eta 2^j (d = -sign f(E0); f ~ E for large |E|) until f changes sign,
// then Newton steps from the bracket end with the smaller |f|, each replaced by
// the Illinois false-position point of the shrinking bracket (the midpoint if
// that rounds onto an end) when it leaves the bracket, until |Delta E| < tol.  Every f is a
// block-wide reduction over (m, nu) in a fixed order; all threads run the same
// scalar control flow on the broadcast result.
#include "gwc_internal.h"

namespace gwc {

namespace {

constexpr int EVT = 1024;  // threads per state

// Re Sigma and d Re Sigma / dE of one state at E (all threads receive them).
__device__ void ev_sigma(const double *__restrict__ r2row, int n_ov, const double *__restrict__ Om,
                         const double *__restrict__ e, int nb, int n_occ, double eta, double E,
                         double *red, double &re, double &dre) {
  const int tid = threadIdx.x;
  const double eta2 = eta * eta;
  double sr = 0.0, sd = 0.0;
  for (int m = 0; m < nb; ++m) {
    const double sg = m < n_occ ? 1.0 : -1.0;
    const double a0 = E - e[m];
    const double *row = r2row + (long long)m * n_ov;
    for (int v = tid; v < n_ov; v += EVT) {
      const double a = a0 + sg * Om[v];
      const double inv = 1.0 / (a * a + eta2);
      const double w = row[v] * inv;
      sr = fma(w, a, sr);
      sd = fma(w * inv, eta2 - a * a, sd);
    }
  }
  red[tid] = sr;
  red[EVT + tid] = sd;
  __syncthreads();
  for (int st = EVT / 2; st > 0; st >>= 1) {
    if (tid < st) {
      red[tid] += red[tid + st];
      red[EVT + tid] += red[EVT + tid + st];
    }
    __syncthreads();
  }
  re = red[0];
  dre = red[EVT];
  __syncthreads();
}

}  // namespace

// Bp[P][n nb + m] = M^P_nm for every pair of states (oo, ov, vo = ov^T, vv).
__global__ void __launch_bounds__(256)
pack_all_pairs_kernel(const double *__restrict__ M_oo, const double *__restrict__ M_ov,
                      const double *__restrict__ M_vv, int n_aux, int n_occ, int n_virt,
                      double *__restrict__ Bp) {
  const int nb = n_occ + n_virt;
  const long long cols = (long long)nb * nb, total = (long long)n_aux * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int P = (int)(e / cols);
    const int nm = (int)(e % cols), n = nm / nb, m = nm % nb;
    double x;
    if (n < n_occ && m < n_occ) x = M_oo[((long long)P * n_occ + n) * n_occ + m];
    else if (n < n_occ) x = M_ov[((long long)P * n_occ + n) * n_virt + (m - n_occ)];
    else if (m < n_occ) x = M_ov[((long long)P * n_occ + m) * n_virt + (n - n_occ)];
    else x = M_vv[((long long)P * n_virt + (n - n_occ)) * n_virt + (m - n_occ)];
    Bp[e] = x;
  }
}

// Q <- 2 Q^2 / Omega_nu in place (rows of n_ov): rho^2 from the projected densities.
__global__ void __launch_bounds__(256)
square_moments_kernel(double *__restrict__ Q, long long rows, int n_ov, const double *__restrict__ Om) {
  const long long total = rows * n_ov;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const double q = Q[e];
    Q[e] = 2.0 * q * q / Om[e % n_ov];
  }
}

// Sigma^x_n = -sum_i sum_P (M^P_ni)^2 for every state n (one block per state).
__global__ void __launch_bounds__(256)
exchange_all_kernel(const double *__restrict__ M_oo, const double *__restrict__ M_ov, int n_aux,
                    int n_occ, int n_virt, double *__restrict__ sx) {
  __shared__ double red[256];
  const int n = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int e = tid; e < n_aux * n_occ; e += 256) {
    const int P = e / n_occ, i = e % n_occ;
    const double x = n < n_occ ? M_oo[((long long)P * n_occ + n) * n_occ + i]
                               : M_ov[((long long)P * n_occ + i) * n_virt + (n - n_occ)];
    s = fma(x, x, s);
  }
  red[tid] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) sx[n] = -red[0];
}

// One outer iteration: every state's quasiparticle equation with the energies
// e in G (see the header).  r2 rows: [(n nb + m) n_ov + nu].
__global__ void __launch_bounds__(EVT)
ev_solve_kernel(const double *__restrict__ r2, int n_ov, const double *__restrict__ Om,
                const double *__restrict__ eps, const double *__restrict__ e,
                const double *__restrict__ sx, const double *__restrict__ vxc, int nb, int n_occ,
                double eta, double tol, int max_steps, double *__restrict__ e_new,
                int *__restrict__ steps) {
  __shared__ double red[2 * EVT];
  const int n = blockIdx.x;
  const double *r2row = r2 + (long long)n * nb * n_ov;
  const double en = eps[n], sxn = sx[n], vxn = vxc[n];
  double re, dre;
  auto fval = [&](double E, double &f, double &df) {
    ev_sigma(r2row, n_ov, Om, e, nb, n_occ, eta, E, red, re, dre);
    f = E - en - sxn - re + vxn;
    df = 1.0 - dre;
  };
  const double E0 = e[n];
  double f0, df0;
  fval(E0, f0, df0);
  double root = E0;
  int nsteps = 0;
  bool done = f0 == 0.0;
  if (!done) {
    const double d = f0 > 0.0 ? -1.0 : 1.0;
    double a = E0, fa = f0, da = df0, b = E0, fb = f0, db = df0, h = eta;
    for (int j = 0; j < 1100; ++j) {
      b = E0 + d * h;
      fval(b, fb, db);
      if (fb == 0.0) {
        root = b;
        done = true;
        break;
      }
      if ((fb > 0.0) != (fa > 0.0)) break;
      a = b;
      fa = fb;
      da = db;
      h *= 2.0;
    }
    if (!done) {
      double lo, hi, flo, fhi;
      if (a < b) { lo = a; hi = b; flo = fa; fhi = fb; } else { lo = b; hi = a; flo = fb; fhi = fa; }
      double E, f, df;
      if (fabs(fa) <= fabs(fb)) { E = a; f = fa; df = da; } else { E = b; f = fb; df = db; }
      int kept = 0;  // -1: the last update moved lo, +1: it moved hi
      nsteps = -1;
      for (int it = 1; it <= max_steps; ++it) {
        double En = df != 0.0 ? E - f / df : lo - 1.0;
        // a step onto an end is kept: at a root found at an end the step
        // rounds to zero, and that is convergence, not a step out
        if (!(lo <= En && En <= hi)) {
          // false position on the bracket, the Illinois way: the f of an end
          // kept through two updates in a row is halved
          En = (lo * fhi - hi * flo) / (fhi - flo);
          if (!(lo < En && En < hi)) En = 0.5 * (lo + hi);
        }
        if (fabs(En - E) < tol) {
          E = En;
          nsteps = it;
          break;
        }
        E = En;
        fval(E, f, df);
        if (f == 0.0) {
          nsteps = it;
          break;
        }
        if ((f > 0.0) == (flo > 0.0)) {
          lo = E;
          flo = f;
          if (kept == -1) fhi *= 0.5;
          kept = -1;
        } else {
          hi = E;
          fhi = f;
          if (kept == 1) flo *= 0.5;
          kept = 1;
        }
      }
      root = E;
    }
  }
  if (threadIdx.x == 0) {
    e_new[n] = root;
    steps[n] = nsteps;
  }
}

// Sigma^c,ev on the core grids (from the pole sums) and A of Eq.
// A_explicit_real_imaginary with Sigma = Sigma^x + Sigma^c,ev.
__global__ void __launch_bounds__(256)
ev_finish_kernel(const double2 *__restrict__ sigma, int n_real, const double *__restrict__ eps,
                 const int *__restrict__ core, const double *__restrict__ omega_real,
                 const double *__restrict__ sx, const double *__restrict__ vxc,
                 double *__restrict__ sigma_c, double *__restrict__ a_ev) {
  const int c = blockIdx.x, npts = n_real + 1, n = core[c];
  const double PI_D = 3.14159265358979323846;
  for (int j = threadIdx.x; j < n_real; j += blockDim.x) {
    const double2 s = sigma[(long long)c * npts + j];
    const double w = omega_real[(long long)c * n_real + j];
    sigma_c[((long long)c * n_real + j) * 2] = s.x;
    sigma_c[((long long)c * n_real + j) * 2 + 1] = s.y;
    const double re = w - eps[n] + vxc[n] - sx[n] - s.x;
    a_ev[(long long)c * n_real + j] = fabs(s.y) / (PI_D * (re * re + s.y * s.y));
  }
}

void launch_pack_all_pairs(const double *M_oo, const double *M_ov, const double *M_vv, int n_aux,
                           int n_occ, int n_virt, double *Bp, hipStream_t s) {
  const long long total = (long long)n_aux * (n_occ + n_virt) * (n_occ + n_virt);
  const int grid = (int)std::min<long long>((total + 255) / 256, 65536);
  pack_all_pairs_kernel<<<grid, 256, 0, s>>>(M_oo, M_ov, M_vv, n_aux, n_occ, n_virt, Bp);
}

void launch_square_moments(double *Q, long long rows, int n_ov, const double *Om, hipStream_t s) {
  const long long total = rows * n_ov;
  const int grid = (int)std::min<long long>((total + 255) / 256, 65536);
  square_moments_kernel<<<grid, 256, 0, s>>>(Q, rows, n_ov, Om);
}

void launch_exchange_all(const double *M_oo, const double *M_ov, int n_aux, int n_occ, int n_virt,
                         double *sx, hipStream_t s) {
  exchange_all_kernel<<<n_occ + n_virt, 256, 0, s>>>(M_oo, M_ov, n_aux, n_occ, n_virt, sx);
}

void launch_ev_solve(const double *r2, int n_ov, const double *Om, const double *eps,
                     const double *e, const double *sx, const double *vxc, int nb, int n_occ,
                     double eta, double tol, int max_steps, double *e_new, int *steps,
                     hipStream_t s) {
  ev_solve_kernel<<<nb, EVT, 0, s>>>(r2, n_ov, Om, eps, e, sx, vxc, nb, n_occ, eta, tol, max_steps,
                                     e_new, steps);
}

void launch_ev_finish(const double2 *sigma, int n_core, int n_real, const double *eps,
                      const int *core, const double *omega_real, const double *sx,
                      const double *vxc, double *sigma_c, double *a_ev, hipStream_t s) {
  ev_finish_kernel<<<n_core, 256, 0, s>>>(sigma, n_real, eps, core, omega_real, sx, vxc, sigma_c,
                                          a_ev);
}

}  // namespace gwc
