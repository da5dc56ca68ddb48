// Internal declarations shared by the host orchestration and the HIP kernels of
// libgwc.  Everything here is gfx950-only HIP C++.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gwc {

// ---------------------------------------------------------------------------
// Tiling constants of the FP64 polarisability build (one 64 x 64 output tile
// per workgroup, 4 waves of 32 x 32, K staged through LDS in chunks of KC).
constexpr int PI_TILE = 64;
constexpr int PI_KC = 32;
constexpr int PI_FB = 2;        // frequencies per workgroup (Re and Im each)
constexpr int PI_THREADS = 256;

// Rows of the packed L = M_ov matrix and its row stride are padded with zeros
// to these multiples so the Pi kernel needs no bounds checks on loads.
constexpr int L_ROW_ALIGN = PI_TILE;
constexpr int L_COL_ALIGN = PI_KC;

// Bordered LU (one workgroup per matrix).
constexpr int LU_NB = 16;
constexpr int LU_THREADS = 256;

// ---------------------------------------------------------------------------
// Launchers (all enqueue on `stream`, no synchronisation).
void launch_pack_l(const double *M_ov, int n_aux, int n_ov, double *Lp, int n_aux_pad, int ldl,
                   hipStream_t stream);
void launch_chi(const double *eps, int n_occ, int n_virt, const double2 *z, int F, int ldl,
                double *chi_re, double *chi_im, hipStream_t stream);
void launch_pi_build_f64(const double *Lp, int ldl, int n_aux, const double *chi_re,
                         const double *chi_im, int F, const int2 *tiles, int n_tiles,
                         double2 *G, long long g_stride, int ldg, hipStream_t stream);
// Mixed-precision Pi build.  Tiles are mixed_tile_rows(prec) x MX_TILE_COLS
// blocks (128 x 256); the split operands have their rows padded to a multiple
// of MX_TILE_COLS and their columns to mixed_ldl(prec, ldl) (the form's K
// chunk: 32 for the 16-bit forms; for FP8 a pair of 64-wide chunks, 128).
constexpr int MX_TILE_COLS = 256;
constexpr int mixed_tile_rows(int) { return 128; }
constexpr int mixed_ldl(int prec, int ldl) { return prec == 3 ? (ldl + 127) / 128 * 128 : ldl; }
// prec 1 BF16X3, 2 FP16X3, 3 FP8X3; Bhi / Blo hold 16-bit (1, 2) or 8-bit (3)
// elements, rows_pad x ldlk of them (ldlk = mixed_ldl(prec, ldl)); Lf, the
// A operand's source, as many FP32 values of L (1, 2) or FP16 values of L
// times its column scales (3).
constexpr int mixed_a_bytes(int prec) { return prec == 3 ? 2 : 4; }
constexpr int mixed_b_bytes(int prec) { return prec == 3 ? 1 : 2; }
void launch_mixed_prep(int prec, const double *Lp, int n_aux_pad, int rows_pad, int ldl, int ldlk,
                       void *Lf, void *Bhi, void *Blo, float *colscale, float *inv_colscale,
                       float *acol, hipStream_t stream);
// chi_f32 is a workspace of F x 2 x ldl floats (the 16-bit forms' scaled FP32 chi).
void launch_pi_build_mixed(int prec, const void *Lf, const void *Bhi, const void *Blo, int ldl,
                           int n_aux, const double *chi_re, const double *chi_im,
                           const float *inv_colscale, const float *acol, float *tscale, float *chi_f32,
                           int F, const int2 *tiles, int n_tiles, double2 *G, long long g_stride,
                           int ldg, hipStream_t stream);
void launch_border(const double *M_oo, const double *M_ov, int n_aux, int n_occ, int n_virt,
                   const int *task_n, const int *task_m, int F, int R, double2 *G,
                   long long g_stride, int ldg, double *bb, hipStream_t stream);
// Batched bordered LU; `scratch` must hold lu_scratch_bytes(F) bytes.  Orders
// up to lu_max_order() (= N + R) are supported.
size_t lu_scratch_bytes(int F);
int lu_max_order();
// Issues the factorisation on `stream`; returns the first HIP launch error.
hipError_t launch_lu_bordered(double2 *G, long long g_stride, int ldg, int N, int R, int F,
                              const double *bb, const long long *out_base, const int *out_stride,
                              double2 *W_out, int *status, void *scratch, hipStream_t stream);

// Pieces shared by the LU and the symmetric factorisation: the trailing update
// of the symmetric factorisation, A[r0.., c0..c1) -= L[r0.., K] A[K, c0..c1)
// over K = [kstart, kstart + klen) with L[r][k] = A[k][r] dinv[f dinv_ld + k]
// (the panels' rows hold W^T = D L^T; lower: only the tiles on or below the
// diagonal of the square range from r0 = c0 to n), the border's W from the
// Schur complement, and clearing the per-matrix status flags.
void launch_trailing_update_sym(double2 *G, long long gs, int ldg, int N, int R, int F, int r0,
                                int c0, int c1, int kstart, int klen, bool lower,
                                const double2 *dinv, int dinv_ld, hipStream_t s);
void launch_bordered_finish(const double2 *G, long long gs, int ldg, int N, int R, int F,
                            const double *bb, const long long *out_base, const int *out_stride,
                            double2 *W_out, hipStream_t s);
void launch_zero_status(int *status, int F, hipStream_t s);
// Batched bordered LDL^T without pivoting (complex symmetric 1 - Pi with a
// positive semidefinite imaginary part, or real SPD): same arguments and
// outputs as launch_lu_bordered; `scratch` holds ldlt_scratch_bytes(F, N)
// bytes; status[f] = 1 flags an exactly zero pivot.
size_t ldlt_scratch_bytes(int F, int N);
hipError_t launch_ldlt_bordered(double2 *G, long long g_stride, int ldg, int N, int R, int F,
                                const double *bb, const long long *out_base, const int *out_stride,
                                double2 *W_out, int *status, void *scratch, hipStream_t stream);
void launch_sigma_x(const double *M_oo, int n_aux, int n_occ, const int *core_idx, int n_core,
                    double *sigma_x, hipStream_t stream);
void launch_quadrature(const double2 *W_imag, const double *eps, int n_basis,
                       const double *omega_imag, const double *w_imag, int n_imag,
                       const double *omega_real, int n_real, const int *core_idx, int n_core,
                       int grid_points, double *I_out, hipStream_t stream);
void launch_assemble(const double2 *W_real, const double *f_task, const int *task_dec,
                     const int *cj_offset, const double *I, int n_core,
                     int n_real, const double *eps, const int *core_idx, const double *sigma_x,
                     const double *vxc, int full, double *sigma_c, double *im_dec,
                     double *sigma_c_eps, double *e_qp, hipStream_t stream);

void launch_nonfinite(const double *x, long long n, int *flag, hipStream_t stream);

// Cumulant tail.
void launch_cumulant_weights(const double *omega_real, const double *im_sigma, int n_real,
                             double eps_n, double *nu, double *c, double *z_out,
                             hipStream_t stream);
void launch_cumulant_time(const double *nu, const double *c, int n_real, int n_t, double dt,
                          double e_qp, double omega0, double eta, double2 *Gt,
                          hipStream_t stream);
void launch_fft_inverse(double2 *buf_a, double2 *buf_b, int log2n, double2 **result,
                        hipStream_t stream);
void launch_extract_spectrum(const double2 *Gw, int n_out, double *A_out, hipStream_t stream);

// Peak-rate probes (diagnostics): kind 0 FP64 MFMA, 1 BF16 MFMA, 2 FP16 MFMA
// (TFLOP/s), 3 HBM copy (GB/s, read + write).
hipError_t probe_peak(int kind, hipStream_t s, double *value);

// CD-WAC Pade fits (kernels_wac.hip): at most WAC_MAX_NODES reference points
// per fitted pair (imaginary nodes plus one real window).
constexpr int WAC_MAX_NODES = 1024;
void launch_pade_fit(const int4 *pairs, int n_pairs, const long long *node_off,
                     const double2 *node_z, const double2 *W_imag, int nb, int ni,
                     const double2 *W_ref, int R_w, int n_rr, double2 *coef, int *status,
                     hipStream_t stream);
void launch_pade_eval(const double2 *z_task, const int *pair_of_task, const int4 *pairs,
                      const long long *node_off, const double2 *node_z, const double2 *coef,
                      int T, double2 *W_out, hipStream_t stream);

// Fully analytic G0W0 (kernels_analytic.hip).  Casida matrix C (n_pad x n_pad,
// ld n_pad) and Y = Delta^1/2 L (n_aux x n_pad) are zero-padded to n_pad, a
// multiple of 2 jacobi_block().
int jacobi_block();
// Transition-space column k holds ia = perm[k] (a permutation of [0, n_occ n_virt)).
void launch_casida_operands(const double *M_ov, const double *eps, const int *perm, int n_aux,
                            int n_occ, int n_virt, int ld, double *Vt, double *Y, hipStream_t s);
// out[i][j] = sum_k A[k][i] B[k][j] (+ diag[i] for i == j < n_diag when diag != NULL).
void launch_gemm_tn(const double *A, long long lda, const double *B, long long ldb, int M, int N,
                    int K, double *out, long long ldo, const double *diag, int n_diag,
                    hipStream_t s);
void launch_zero_counters(int *x, int n, hipStream_t s);  // n <= 64
// One round r of a block-Jacobi sweep over nb blocks: pair rotations V stored as
// Ep = V - I (nb/2 x 64 x 64), active[nb/2] flags pairs that rotated, counted in
// *rotations; then C <- V^T C V and Y <- Y V, adding the 64 x 64 C and Y tiles
// it updated to work[0] and work[1].
void launch_jacobi_pairs(const double *C, long long ldc, int nb, int r, double tol, double *Ep,
                         int *active, int *rotations, hipStream_t s);
void launch_jacobi_apply(double *C, long long ldc, int nb, int r, const double *Ep,
                         const int *active, double *Y, long long ldy, int n_aux, int *work,
                         hipStream_t s);
// Om[nu] = sqrt(C[nu][nu]) (nu < n; 1 on the padding); sorted (may be NULL) ascending.
void launch_excitations(const double *C, long long ldc, int n, int n_pad, double *Om,
                        double *sorted, hipStream_t s);
void launch_pack_pairs(const double *M_oo, const double *M_ov, int n_aux, int n_occ, int n_virt,
                       const int *core, int n_core, double *Bp, hipStream_t s);
// part holds pole_sum_blocks(n_ov) x n_core x (n_real + 1) double2.  Q rows
// (c or row_state[c]) * n_basis + m hold projected densities, or rho^2 when
// `squared`; eps are the energies in G.
int pole_sum_blocks(int n_ov);
void launch_pole_sum(const double *Q, long long ldq, const double *Om, int n_ov, const double *eps,
                     int n_occ, int n_basis, const int *core, int n_core, const double *omega_real,
                     int n_real, double eta, int squared, const int *row_state, double2 *part,
                     double2 *sigma, hipStream_t s);
void launch_analytic_finish(const double2 *sigma, int n_core, int n_real, const double *eps,
                            const int *core, const double *omega_real, const double *sigma_x,
                            const double *vxc, double *sigma_c, double *sigma_c_eps, double *e_qp,
                            double *a_gw, double *a_dh, hipStream_t s);

// evGW0 (kernels_evgw.hip).
void launch_pack_all_pairs(const double *M_oo, const double *M_ov, const double *M_vv, int n_aux,
                           int n_occ, int n_virt, double *Bp, hipStream_t s);
void launch_square_moments(double *Q, long long rows, int n_ov, const double *Om, hipStream_t s);
void launch_exchange_all(const double *M_oo, const double *M_ov, int n_aux, int n_occ, int n_virt,
                         double *sx, hipStream_t s);
void launch_ev_solve(const double *r2, int n_ov, const double *Om, const double *eps,
                     const double *e, const double *sx, const double *vxc, int nb, int n_occ,
                     double eta, double tol, int max_steps, double *e_new, int *steps,
                     hipStream_t s);
void launch_ev_finish(const double2 *sigma, int n_core, int n_real, const double *eps,
                      const int *core, const double *omega_real, const double *sx,
                      const double *vxc, double *sigma_c, double *a_ev, hipStream_t s);

}  // namespace gwc
