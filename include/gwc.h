/*
 * gwc.h - C ABI of libgwc: the G0W0 correlation self-energy of core states by
 * contour deformation (CD) with the resolution of the identity (RI), and the
 * GW+C cumulant spectral function, on one AMD MI355X (gfx950).
 *
 * Paper: Kocklauner & Golze, "GW plus cumulant approach for predicting
 * core-level shake-up satellites in large molecules" (arXiv:2412.17132).
 *
 * Conventions for every entry point
 *   - Energies and frequencies in Hartree; arrays are row-major float64;
 *     sizes are int32.
 *   - The caller owns every buffer.  A pointer may address host memory or
 *     device memory of the current HIP device; the library detects which and
 *     stages host data itself.  No pointer is kept after the call returns.
 *   - Calls are synchronous: they return after the outputs are written.  All
 *     device work is ordered on `hip_stream` (NULL = the default stream).
 *   - On error the outputs are unspecified, the status below is returned, no
 *     exception crosses the ABI and the process is never aborted;
 *     gwc_last_error() then describes the failure (thread-local).
 *   - Calls from several host threads may run at once, each ordered on its own
 *     stream (the request server's workers do so); the library's shared state
 *     (its device-memory cache, a resident system's split operands, the
 *     timing registry) is guarded by locks.  gwc_spectral_cumulant_noalloc is
 *     the exception: see there.
 *   - Device temporaries come from a library-owned cache of device blocks per
 *     GPU: a block freed by a call is kept (up to half the device's memory)
 *     and handed out again, to the same stream at once and to another stream
 *     once the freeing stream has passed the block's last use; only a miss
 *     calls hipMalloc, and a failed allocation first returns the idle blocks.
 *     The cached bytes stay allocated until then or the process ends.
 */
#ifndef GWC_H
#define GWC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GWC_VERSION 10300 /* 1.3.0 */

enum gwc_status {
  GWC_OK = 0,
  GWC_ERR_INVALID_ARG = -1,     /* NULL pointer, unknown mode/precision, bad grid order */
  GWC_ERR_SHAPE = -2,           /* a size < 1, core index out of range, size too large */
  GWC_ERR_NONPOSITIVE_GAP = -3, /* max eps_occ >= min eps_virt: chi would change sign */
  GWC_ERR_NONFINITE = -4,       /* NaN/Inf in an input */
  GWC_ERR_FACTORIZATION = -5,   /* exactly singular pivot in the LU of 1 - Pi(z) */
  GWC_ERR_OUT_OF_MEMORY = -6,
  GWC_ERR_DEVICE = -7,          /* any other HIP runtime failure */
  GWC_ERR_UNSUPPORTED = -8      /* a valid request the library does not implement */
};

enum gwc_mode {
  /* Sigma^c_n on every real grid point with all residue terms
   * (Eqs. cd_terms, cd_imaginary, cd_residue, cd_prefactors). */
  GWC_MODE_FULL = 0,
  /* Decoupling approximation (Eq. cd_sigma_imaginary_decoupled): on the grid
   * only the residues of n's equivalent set (m = n, or the symmetry-equivalent
   * core levels given by sym_group, Eq. sigma_spectral_decoupled_symmetric),
   * giving Im Sigma^dec; Sigma^c_n(eps_n) is still computed with every term
   * for the quasiparticle energy. */
  GWC_MODE_DECOUPLED = 1
};

enum gwc_precision {
  GWC_PREC_FP64 = 0,   /* everything in float64 */
  GWC_PREC_BF16X3 = 1, /* Pi build as hi*hi + hi*lo + lo*hi bf16 products, fp32 accumulation */
  GWC_PREC_FP16X3 = 2, /* same with fp16 and power-of-two column and frequency scaling */
  GWC_PREC_FP8 = 3     /* fp8 e4m3 hi*hi + hi*lo + lo*hi, fp32 accumulation, power-of-two column
                        * and frequency scaling aimed below the e4m3 limit (448); ~2^-7
                        * relative per product, so ~1e-3 on Sigma^c: a throughput option */
};

/* A closed-shell system in the RI representation.
 * Orbitals are ordered occupied first: m < n_occ occupied (occ = 2),
 * m >= n_occ virtual (occ = 0); n_basis = n_occ + n_virt.
 *   eps  [n_basis]              Kohn-Sham eigenvalues (Ha)
 *   occ  [n_basis]              occupations, each exactly 2.0 or 0.0, occupied first
 *   M_oo [n_aux][n_occ][n_occ]  RI coefficients M^P_ij (Coulomb-metric symmetrised,
 *                               so that W = (1 - Pi)^-1 - 1 in this basis)
 *   M_ov [n_aux][n_occ][n_virt] RI coefficients M^P_ia
 * M_vv is never needed: the states n are occupied, so every pair (n, m) lies
 * in the oo or ov block. */
typedef struct {
  int32_t n_aux, n_occ, n_virt;
  const double *eps;
  const double *occ;
  const double *M_oo;
  const double *M_ov;
} gwc_system;

/* CD-WAC settings (paper section "Numerical GW+C scheme", Eq. pade_approximation;
 * the paper's values in section "Computational Details": 100 + 100 points,
 * core window 0..40 eV, valence margins 0.08 and 0.01).  W^c_nm is computed
 * at reference points only -- the imaginary nodes of the I_n quadrature and
 * real points z = x + i eta -- and every residue W^c_nm(|eps_m - w| + i eta)
 * is taken from a continued-fraction (Thiele) fit through them:
 *   a pair (n, m) lies in the core window when every residue argument
 *   x = |eps_m - w| of the pair is <= core_max; its real points are then
 *   n_core_pts values spaced evenly on [core_min, core_max];
 *   the other pairs of n use n_val_pts points spaced evenly on
 *   [(1 - delta_lower) x_min, (1 + delta_upper) x_max], x_min / x_max the
 *   smallest / largest residue argument over those pairs;
 *   a pair's nodes are the imaginary nodes (ascending) then its window's points.
 * Each window point costs one bordered factorisation with every orbital that
 * has residue terms as border (the occupied ones for core-level grids).
 * Constraints: n_core_pts, n_val_pts >= 2; 0 <= core_min < core_max;
 * 0 <= delta_lower < 1; delta_upper >= 0; n_imag + max(n_core_pts, n_val_pts)
 * <= 1024 (GWC_ERR_INVALID_ARG / GWC_ERR_SHAPE otherwise).  A fit that breaks
 * down (a zero reciprocal difference) returns GWC_ERR_FACTORIZATION. */
typedef struct {
  int32_t n_core_pts;
  double core_min, core_max;
  int32_t n_val_pts;
  double delta_lower, delta_upper;
} gwc_wac_params;

/* Newton solution of the G0W0 quasiparticle equation (Eq. quasiparticle_equation)
 *   E = eps_n + Sigma^x_n + Re Sigma^c_n(E) - v^xc_n
 * from E = eps_n: f(E) = E - eps_n - Sigma^x_n - Re Sigma^c_n(E) + v^xc_n,
 * f'(E) from the centred difference (f(E + step) - f(E - step)) / (2 step),
 * E <- E - f(E) / f'(E), until |Delta E| < tol or max_iter steps.  Every
 * iteration evaluates Sigma^c_n by contour deformation at E - step, E, E + step
 * (the imaginary-axis W is computed once).  Constraints: max_iter >= 1,
 * tol > 0, step > 0, finite (GWC_ERR_INVALID_ARG / GWC_ERR_NONFINITE). */
typedef struct {
  int32_t max_iter;
  double tol;
  double step;
} gwc_qp_params;

/* Arguments of gwc_sigma_core.
 *   core_idx   [n_core]          occupied states n (each < n_occ), the "core states"
 *   omega_imag [n_imag], w_imag  nodes (> 0, strictly increasing) and weights (> 0)
 *                                of a quadrature for int_0^inf (imaginary axis)
 *   omega_real [n_core][n_real]  real frequencies per core state, strictly increasing
 *   eta        > 0               broadening of the residue arguments |eps_m - w| + i eta
 *   vxc        [n_core] or NULL  <n|v_xc|n>, NULL means 0
 *   mode       enum gwc_mode
 *   precision  enum gwc_precision: the Pi builds (both axes) in that form; chi(z),
 *              the LU of 1 - Pi, the residue sums and E_QP stay FP64
 *   sym_group  [n_basis] or NULL  labels of symmetry-equivalent core levels
 *              (Eq. sigma_spectral_decoupled_symmetric): the equivalent set of a
 *              core state n is every orbital carrying n's label when that label
 *              is >= 0, else {n}; NULL means {n} for every n.  A set must hold
 *              occupied orbitals only (GWC_ERR_INVALID_ARG otherwise).  It
 *              selects the residues of Im Sigma^dec.
 *   wac        NULL: contour deformation, every residue W from its own
 *              factorisation; else CD-WAC with these settings (host memory)
 *   qp         NULL, or the settings of the Newton quasiparticle solve (host
 *              memory; contour deformation only: with wac set it returns
 *              GWC_ERR_UNSUPPORTED) */
typedef struct {
  int32_t n_core;
  const int32_t *core_idx;
  int32_t n_imag;
  const double *omega_imag;
  const double *w_imag;
  int32_t n_real;
  const double *omega_real;
  double eta;
  const double *vxc;
  int32_t mode;
  int32_t precision;
  const int32_t *sym_group;
  const gwc_wac_params *wac;
  const gwc_qp_params *qp;
} gwc_sigma_args;

/* Outputs of gwc_sigma_core (each may be host or device memory).
 *   sigma_c      [n_core][n_real][2]  Sigma^c_n(w) = -I_n(w) + R_n(w) as (re, im);
 *                                     required in FULL mode, ignored (may be NULL)
 *                                     in DECOUPLED mode
 *   im_sigma_dec [n_core][n_real]     sum over n's equivalent set S of
 *                                     f_i Im W^c_ni(|eps_i - w| + i eta), in ascending
 *                                     i (S = {n} by default), or NULL
 *   sigma_c_eps  [n_core][2]          Sigma^c_n(eps_n) (re, im), or NULL
 *   sigma_x      [n_core]             Sigma^x_n = -sum_i (n i|i n), or NULL
 *   e_qp         [n_core]             E_QP = eps_n + Sigma^x_n + Re Sigma^c_n(eps_n) - v^xc_n
 *                                     (Eq. QPGWC), or NULL
 *   e_qp_newton  [n_core]             with args->qp: the Newton solution of Eq.
 *                                     quasiparticle_equation (the last iterate when it
 *                                     did not converge), or NULL
 *   qp_iterations [n_core] int32      with args->qp: Newton steps taken, -1 when
 *                                     max_iter steps did not converge, or NULL */
typedef struct {
  double *sigma_c;
  double *im_sigma_dec;
  double *sigma_c_eps;
  double *sigma_x;
  double *e_qp;
  double *e_qp_newton;
  int32_t *qp_iterations;
} gwc_sigma_out;

/* Correlation self-energy of the requested core states by contour
 * deformation (paper section "Self-energy evaluation"):
 *   Sigma^c_n(w) = -I_n(w) + R_n(w)                                (Eq. cd_terms)
 *   I_n(w) = (1/pi) sum_k w_k sum_m W^c_nm(i w_k) a/(a^2 + w_k^2),
 *            a = w - eps_m                 (Eq. cd_imaginary, folded to (0, inf))
 *   R_n(w) = sum_m f_m W^c_nm(|eps_m - w| + i eta)                  (Eq. cd_residue)
 *   f_m    = -Theta(eps_F - eps_m) Theta(eps_m - w)
 *            + Theta(eps_m - eps_F) Theta(w - eps_m), Theta(0) = 1/2 (Eq. cd_prefactors)
 * with the RI screened interaction W^c_nm(z) = M_nm^T [(1 - Pi(z))^-1 - 1] M_nm,
 * Pi_PQ(z) = sum_ia M^P_ia M^Q_ia 4 Delta_ia / (z^2 - Delta_ia^2).
 * Returns GWC_OK or a negative gwc_status. */
int gwc_sigma_core(const gwc_system *sys, const gwc_sigma_args *args, gwc_sigma_out *out,
                   void *hip_stream);

/* Arguments of gwc_spectral_cumulant (one core state).
 *   omega_real [n_real], im_sigma [n_real]  Im Sigma^c_n on a strictly increasing
 *                                          grid in the G0W0 frame (zero outside it)
 *   eps_n, e_qp        the mean-field level and the GW+C quasiparticle energy
 *   eta > 0            broadening of G^QP_0 (Eq. eq:GQP)
 *   n_t                number of time points = FFT length, a power of two in [2^4, 2^24]
 *   d_omega > 0        frequency resolution; dt = 2 pi / (n_t d_omega)
 *   n_out in [1, n_t]  number of output frequencies omega_out_min + l d_omega */
typedef struct {
  int32_t n_real;
  const double *omega_real;
  const double *im_sigma;
  double eps_n, e_qp, eta;
  int32_t n_t;
  double d_omega;
  int32_t n_out;
  double omega_out_min;
} gwc_cumulant_args;

/* GW+C spectral function of one state (paper section "Numerical GW+C scheme"):
 *   C~(t) = (1/pi) int dw |Im Sigma^c_n(w + eps_n)| / w^2 (e^{-iwt} - 1)
 *                                      (Eq. landau_cumulant_truncated; trapezoid
 *                                       sum on the grid, the w = 0 term is 0)
 *   G^C(t) = -i Theta(t) e^{-i E_QP t - eta t} e^{C~(t)}, Theta(0) = 1/2
 *                                      (Eq. cumulant_propagator_numerical_time)
 *   G^C(w) = dt sum_k G^C(t_k) e^{i w t_k} by FFT    (Eqs. cumulant_propagator_fourier,
 *                                                     cumulant_propagator_convolution)
 *   A(w)   = -Im G^C(w) / pi                         (Eq. eq:AGWC)
 *   A_out [n_out]            spectral function on omega_out_min + l d_omega
 *   z_out [2] or NULL        (Z, 1 - Z) with Z = exp(-(1/pi) int |Im Sigma| / w^2)
 * Returns GWC_OK or a negative gwc_status. */
int gwc_spectral_cumulant(const gwc_cumulant_args *args, double *A_out, double *z_out,
                          void *hip_stream);

/* gwc_spectral_cumulant without device allocation, for callers that cannot
 * allocate (code under stream capture, serving loops that forbid hipMalloc):
 * the same arguments, kernels, results and errors, with every temporary in one
 * library-owned device array per GPU (about 21 MB, held until the process
 * ends) instead of the library's cache of device blocks.  Limits: n_t <= 2^19 and
 * n_real <= 2^15; larger sizes return GWC_ERR_SHAPE.  Inputs and outputs may
 * be host or device memory, as for gwc_spectral_cumulant.  All calls on one GPU
 * share that array: calls that overlap on one GPU (several host threads or
 * streams) race and must be serialised by the caller. */
int gwc_spectral_cumulant_noalloc(const gwc_cumulant_args *args, double *A_out, double *z_out,
                                  void *hip_stream);

/* Arguments of gwc_sigma_analytic.
 *   core_idx   [n_core]         occupied states n (each < n_occ)
 *   omega_real [n_core][n_real] real frequencies per core state, strictly increasing
 *   eta        > 0              broadening of the poles (Eq. sigma_spectral)
 *   vxc        [n_core] or NULL <n|v_xc|n>, NULL means 0 */
typedef struct {
  int32_t n_core;
  const int32_t *core_idx;
  int32_t n_real;
  const double *omega_real;
  double eta;
  const double *vxc;
} gwc_analytic_args;

/* Outputs of gwc_sigma_analytic (each may be host or device memory).
 *   sigma_c     [n_core][n_real][2]  Sigma^c_n(w) (re, im), Eq. sigma_spectral (required)
 *   sigma_c_eps [n_core][2]          Sigma^c_n(eps_n), or NULL
 *   sigma_x     [n_core]             Sigma^x_n = -sum_i (n i|i n), or NULL
 *   e_qp        [n_core]             eps_n + Sigma^x_n + Re Sigma^c_n(eps_n) - v^xc_n (Eq.
 *                                    QPGWC); DH_n = e_qp - eps_n is the Hedin shift (Eq.
 *                                    hedin_shift), or NULL
 *   a_gw        [n_core][n_real]     A^G0W0_n(w) of Eq. A_explicit_real_imaginary, or NULL
 *   a_dh        [n_core][n_real]     A^{G_DH W0}_n at w + DH_n, i.e. with Sigma^c_n(w) and
 *                                    w - eps_n replaced by w + DH_n - eps_n (Eq.
 *                                    hedin_sigma_spectral), or NULL
 *   omega_exc   [n_occ * n_virt]     RPA excitation energies Omega^nu ascending, or NULL
 *   sweeps      [1] int32            block-Jacobi sweeps taken, or NULL */
typedef struct {
  double *sigma_c;
  double *sigma_c_eps;
  double *sigma_x;
  double *e_qp;
  double *a_gw;
  double *a_dh;
  double *omega_exc;
  int32_t *sweeps;
} gwc_analytic_out;

/* Fully analytic G0W0 self-energy of the requested core states (paper section
 * "GW for core levels"):
 *   RPA excitations from Eqs. rpa_casida, rpa_matrices for real orbitals, closed-shell
 *   singlet, in the symmetric form C Z = Omega^2 Z with
 *     C = Delta^2 + 4 Delta^1/2 K Delta^1/2,  K_ia,jb = (ia|jb) = sum_P M^P_ia M^P_jb,
 *     X + Y = Delta^1/2 Z Omega^-1/2;
 *   rho^nu_nm = sqrt(2) sum_ia (nm|ia) (X + Y)^nu_ia            (Eq. density_shifts)
 *   Sigma^c_n(w) = sum_{m,nu} (rho^nu_nm)^2 /
 *                  (w - eps_m + (Omega^nu - i eta) sgn(eps_F - eps_m))  (Eq. sigma_spectral)
 * C is diagonalised on the device by cyclic block Jacobi (converged when a sweep
 * applies no rotation larger than the working precision; more than 60 sweeps
 * return GWC_ERR_FACTORIZATION).  Device memory ~ 8 (n_ov^2 + 3 n_aux n_ov +
 * n_core n_basis (n_aux + n_ov)) bytes, n_ov = n_occ * n_virt <= 65536
 * (GWC_ERR_SHAPE otherwise).  Returns GWC_OK or a negative gwc_status. */
int gwc_sigma_analytic(const gwc_system *sys, const gwc_analytic_args *args, gwc_analytic_out *out,
                       void *hip_stream);

/* Settings of gwc_evgw0 (all > 0; GWC_ERR_INVALID_ARG otherwise). */
typedef struct {
  int32_t max_outer;   /* outer iterations on the energies in G */
  double tol_outer;    /* stop when max_n |e^(k+1)_n - e^(k)_n| < tol_outer (Ha) */
  int32_t max_newton;  /* Newton steps per state and iteration after bracketing */
  double tol_newton;   /* a state's solve ends when |Delta E| < tol_newton (Ha) */
} gwc_evgw_params;

/* Arguments of gwc_evgw0.
 *   M_vv       [n_aux][n_virt][n_virt]  RI coefficients M^P_ab (symmetric in a, b):
 *                                       every state's energy is updated, so pairs
 *                                       of two virtual states occur (required)
 *   core_idx   [n_core]                 occupied states whose Sigma^c,ev and A are
 *                                       returned on omega_real [n_core][n_real]
 *                                       (strictly increasing per core)
 *   eta > 0                             broadening of the poles
 *   vxc        [n_basis] or NULL        <n|v_xc|n> of every state, NULL means 0
 *   params     NULL: max_outer 100, tol_outer 1e-8, max_newton 200, tol_newton 1e-10 */
typedef struct {
  const double *M_vv;
  int32_t n_core;
  const int32_t *core_idx;
  int32_t n_real;
  const double *omega_real;
  double eta;
  const double *vxc;
  const gwc_evgw_params *params;
} gwc_evgw_args;

/* Outputs of gwc_evgw0 (each may be host or device memory).
 *   e_qp     [n_basis]                 evGW0 quasiparticle energies (required)
 *   e_first  [n_basis]                 energies after the first iteration (the G0W0
 *                                      solutions found from eps), or NULL
 *   sigma_x  [n_basis]                 Sigma^x_n = -sum_i (n i|i n), or NULL
 *   sigma_c  [n_core][n_real][2]       Sigma^c,ev_n(w) with the final energies in G, or NULL
 *   a_ev     [n_core][n_real]          A of Eq. A_explicit_real_imaginary with Sigma^x +
 *                                      Sigma^c,ev, or NULL
 *   newton   [n_basis] int32           Newton steps of each state in the last iteration,
 *                                      -1 where max_newton did not converge, or NULL
 *   outer    [1] int32                 iterations taken, -1 when max_outer did not
 *                                      converge (the last iterate is returned), or NULL */
typedef struct {
  double *e_qp;
  double *e_first;
  double *sigma_x;
  double *sigma_c;
  double *a_ev;
  int32_t *newton;
  int32_t *outer;
} gwc_evgw_out;

/* Eigenvalue-self-consistent evGW0 (paper section "GW for core levels: beyond
 * G0W0", Eq. ev_sigma_spectral): with Omega^nu and rho^nu_nm of the RPA on the
 * mean-field energies (as in gwc_sigma_analytic, for every pair of states),
 *   Sigma^c,ev_n(w; e) = sum_{m,nu} (rho^nu_nm)^2 / (w - e_m + (Omega^nu - i eta) s_m),
 *   s_m = +1 for occupied, -1 for virtual m,
 * every state's quasiparticle equation (Eq. quasiparticle_equation)
 *   E = eps_n + Sigma^x_n + Re Sigma^c,ev_n(E; e^(k)) - v^xc_n
 * is solved from E0 = e^(k)_n (e^(0) = eps): points E0 + d eta 2^j, d = -sign f(E0),
 * until f changes sign, then Newton steps (analytic derivative) from the bracket end
 * with the smaller |f|, each replaced by the Illinois false-position point of the
 * shrinking bracket when it leaves it (the midpoint if that point rounds onto an end);
 * e^(k+1) = the roots, until max_n |e^(k+1)_n - e^(k)_n| < tol_outer.
 * Device memory ~ 8 (n_basis^2 (n_ov + n_aux) + n_ov^2 + 3 n_aux n_ov) bytes,
 * n_ov = n_occ * n_virt <= 65536.  Non-convergence is reported in `outer` and
 * `newton`, not as an error.  Returns GWC_OK or a negative gwc_status. */
int gwc_evgw0(const gwc_system *sys, const gwc_evgw_args *args, gwc_evgw_out *out,
              void *hip_stream);

/* ---------------------------------------------------------------------------
 * Device-resident systems (serving form).  gwc_system_create validates a
 * system as gwc_sigma_core does and keeps library-owned device copies of eps,
 * M_oo, M_ov and the packed L (plus, on first use, the split operands of the
 * mixed-precision Pi build) until gwc_system_destroy; the caller's arrays may
 * be freed after create returns.  gwc_sigma_core_resident is gwc_sigma_core on
 * such a handle (same arguments, outputs and errors).  A handle may be used by
 * several threads and server requests at once; destroy waits for the device
 * and must not race with calls that use the handle. */
typedef struct gwc_resident_system_s *gwc_system_handle;
int gwc_system_create(const gwc_system *sys, gwc_system_handle *handle);
int gwc_system_destroy(gwc_system_handle handle);
int gwc_sigma_core_resident(gwc_system_handle handle, const gwc_sigma_args *args,
                            gwc_sigma_out *out, void *hip_stream);

/* Request server (continuous batching of single-core-state solves).
 * n_slots worker threads, each with its own HIP stream, take queued requests
 * in arrival order as soon as a slot is free and the request's predicted
 * device footprint fits in hbm_budget_bytes beside the running requests;
 * requests that can never fit are refused at submit (GWC_ERR_OUT_OF_MEMORY).
 * batch_bytes (0 = budget / 4) bounds the batched matrices of one launch of a
 * request and is the same for every request, so each result is independent
 * of what runs beside it.  A request's footprint includes the split operands
 * of the mixed-precision forms when its system has none for its precision
 * yet; the request that builds them leaves them with the system, and they
 * stay counted against the budget until the server is destroyed (a queued
 * request that then no longer fits fails with GWC_ERR_OUT_OF_MEMORY).  One request = gwc_sigma_core for one core state
 * (mode, precision as given) followed by gwc_spectral_cumulant of its
 * Im Sigma^dec when n_t > 0, with the output window starting at
 * E_QP + omega_out_min_rel.  Times are seconds since server creation. */
typedef struct gwc_server_s *gwc_server_handle;
typedef struct {
  int32_t n_slots;          /* 1..64 */
  double hbm_budget_bytes;  /* > 0 */
  double batch_bytes;       /* 0 = hbm_budget_bytes / 4 */
} gwc_server_config;
typedef struct {
  gwc_system_handle system;
  int32_t core_idx;                   /* < n_occ of the system */
  int32_t n_imag;
  const double *omega_imag, *w_imag;  /* host arrays, copied at submit */
  int32_t n_real;
  const double *omega_real;           /* host array, copied at submit */
  double eta, vxc;
  int32_t mode, precision;
  int32_t n_t;                        /* 0 = no cumulant */
  double d_omega;
  int32_t n_out;
  double omega_out_min_rel;
} gwc_request;
typedef struct {
  int32_t status;                     /* gwc_status of the request */
  double e_qp, sigma_x, sigma_c_eps[2], z[2];
  double *im_sigma_dec;               /* [n_real] host buffer to fill, or NULL */
  double *A;                          /* [n_out] host buffer to fill, or NULL */
  double *sigma_c;                    /* [n_real][2] host buffer (FULL mode), or NULL */
  double t_submit, t_start, t_end;
  double footprint_bytes;
} gwc_request_result;
typedef struct {
  int32_t queued, active, peak_active;
  long long completed;
  double in_use_bytes, peak_in_use_bytes, budget_bytes;
  double kept_bytes;  /* split operands built by requests, kept with their systems */
  long long refused;  /* queued requests failed because they no longer fit */
} gwc_server_stats_t;
int gwc_server_create(const gwc_server_config *cfg, gwc_server_handle *server);
int gwc_server_submit(gwc_server_handle server, const gwc_request *request, int64_t *ticket);
/* Blocks until the request has finished; fills `result` and returns its status.
 * A ticket is consumed by its wait: waiting on it again, or from a second
 * thread while the first still waits, returns GWC_ERR_INVALID_ARG. */
int gwc_server_wait(gwc_server_handle server, int64_t ticket, gwc_request_result *result);
int gwc_server_stats(gwc_server_handle server, gwc_server_stats_t *stats);
/* Finishes every queued request, then stops the workers. */
int gwc_server_destroy(gwc_server_handle server);

/* Kernel timing (diagnostics for profiling harnesses, not part of the method).
 * gwc_timing_enable(1) clears the counters and, until gwc_timing_enable(0),
 * brackets every launch of the named hot kernels with HIP events recorded on
 * the stream the kernel runs on.  gwc_timing_get returns, for one kernel name
 * ("pi_build_f64", "pi_build_mixed" or "lu_bordered"), the summed event time in ms, the number
 * of launches and the algorithmic flop count of those launches (Pi build, in
 * either precision: 2 N_aux (N_aux + 1) N_ov per complex residue frequency,
 * half that on the imaginary axis; LU: (8/3) N^3 + 8 N^2 R per bordered N x N matrix with R
 * border vectors).  Returns GWC_ERR_INVALID_ARG for an unknown name. */
int gwc_timing_enable(int on);
int gwc_timing_get(const char *kernel, double *total_ms, long long *launches, double *flops);

/* Peak-rate probe (diagnostics, not part of the method): runs a
 * microbenchmark on the current device, ordered on hip_stream (NULL: default
 * stream), and returns through *value what the device reaches:
 *   kind 0  FP64 MFMA (v_mfma_f64_16x16x4f64), TFLOP/s
 *   kind 1  BF16 MFMA (v_mfma_f32_16x16x32_bf16), TFLOP/s
 *   kind 2  FP16 MFMA (v_mfma_f32_16x16x32_f16), TFLOP/s
 *   kind 3  device-memory copy of 4 GiB, GB/s counting bytes read + written
 *   kind 4  FP8 MFMA, K = 32 (v_mfma_f32_16x16x32_fp8_fp8, E4M3), TFLOP/s
 *   kind 5  FP8 MFMA, K = 128 (v_mfma_f32_16x16x128_f8f6f4, E4M3, no block
 *           scales), TFLOP/s
 * The MFMA probes keep operands in registers (independent accumulator chains,
 * no memory traffic in the loop); each figure is the median of five timed
 * launches after one untimed launch.  Allocates temporaries (2 x 4 GiB for
 * kind 3) from the stream-ordered pool and frees them before returning.
 * GWC_ERR_INVALID_ARG for another kind or a NULL value; GWC_ERR_DEVICE or
 * GWC_ERR_OUT_OF_MEMORY on a HIP failure. */
int gwc_probe_peak(int kind, double *value, void *hip_stream);

/* Message describing the last non-OK return on the calling thread ("" if none). */
const char *gwc_last_error(void);

/* GWC_VERSION of the loaded library. */
int gwc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GWC_H */
