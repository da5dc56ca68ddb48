// C ABI of libgwc: argument validation, staging, task lists and the launch
// sequence of the contour-deformation self-energy and the cumulant tail.
//
// gwc_sigma_core, in order (paper section "Self-energy evaluation"):
//   1. pack L = M_ov into a zero-padded N_aux x N_ov buffer;
//   2. imaginary axis: one task per (node w_k, core n) with all b_nm as border
//      vectors -> W^c_nm(i w_k) for every m (input of Eq. cd_imaginary);
//   3. residues: one task per (core n, point w, orbital m) with f_m != 0
//      (Eq. cd_prefactors, Theta(0) = 1/2) at z = |eps_m - w| + i eta
//      (Eq. cd_residue) -> W^c_nm(z);
//      each task batch runs chi -> Pi build (FP64 MFMA) -> border -> bordered LU;
//   4. exchange, imaginary-axis quadrature, residue sums and E_QP (Eqs. cd_terms,
//      sigma_x, QPGWC).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "gwc.h"
#include "gwc_internal.h"

namespace {

thread_local std::string g_last_error;
std::mutex g_mutex;

// Kernel timing (diagnostics): event pairs recorded around hot launches on the
// launch stream, resolved after the stream synchronises.
struct TimerStat {
  double total_ms = 0.0;
  long long launches = 0;
  double flops = 0.0;
};
struct PendingTiming {
  int kernel;  // index into kTimedKernels
  hipEvent_t a, b;
  double flops;
};
bool g_timing = false;
constexpr int kNumTimed = 3;
TimerStat g_stats[kNumTimed];
std::vector<PendingTiming> g_pending;
const char *const kTimedKernels[kNumTimed] = {"pi_build_f64", "lu_bordered", "pi_build_mixed"};

struct GwcError {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw GwcError{code, std::string(buf)};
}

#define HIPCHECK(x)                                                                           \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess)                                                                     \
      fail(e_ == hipErrorOutOfMemory ? GWC_ERR_OUT_OF_MEMORY : GWC_ERR_DEVICE, "%s: %s", #x, \
           hipGetErrorString(e_));                                                            \
  } while (0)

hipEvent_t timing_mark(hipStream_t s) {
  hipEvent_t e;
  HIPCHECK(hipEventCreate(&e));
  HIPCHECK(hipEventRecord(e, s));
  return e;
}

// Folds the recorded event pairs into the counters (stream must be idle).
void timing_resolve() {
  for (auto &p : g_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_stats[p.kernel].total_ms += ms;
      g_stats[p.kernel].launches += 1;
      g_stats[p.kernel].flops += p.flops;
    } else {
      (void)hipGetLastError();
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
}

// Device allocation owned for the duration of one call.
struct DevBuf {
  void *p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t bytes) {
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      fail(e == hipErrorOutOfMemory ? GWC_ERR_OUT_OF_MEMORY : GWC_ERR_DEVICE,
           "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
  }
  template <class T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

bool is_device_ptr(const void *ptr) {
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.isManaged;
}

// Copy `count` elements of a host-or-device array into a host vector.
template <class T>
std::vector<T> to_host(const T *p, size_t count, hipStream_t s) {
  std::vector<T> v(count);
  if (count == 0) return v;
  if (is_device_ptr(p)) {
    HIPCHECK(hipMemcpyAsync(v.data(), p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  } else {
    std::copy(p, p + count, v.begin());
  }
  return v;
}

template <class T>
T *upload(DevBuf &buf, const std::vector<T> &v, hipStream_t s) {
  buf.alloc(v.size() * sizeof(T));
  if (!v.empty())
    HIPCHECK(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return buf.as<T>();
}

// A device view of a host-or-device input array; host data is copied in.
template <class T>
const T *device_view(const T *p, size_t count, DevBuf &holder, hipStream_t s) {
  if (is_device_ptr(p)) return p;
  holder.alloc(count * sizeof(T));
  HIPCHECK(hipMemcpyAsync(holder.p, p, count * sizeof(T), hipMemcpyHostToDevice, s));
  return holder.as<const T>();
}

void copy_out(void *dst, const void *src_dev, size_t bytes, hipStream_t s) {
  if (!dst || bytes == 0) return;
  HIPCHECK(hipMemcpyAsync(dst, src_dev, bytes, hipMemcpyDefault, s));
}

bool all_finite(const std::vector<double> &v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bytes of device memory the batched matrices of one launch may use.
size_t batch_budget_bytes() {
  size_t budget = size_t(48) << 30;
  if (const char *e = std::getenv("GWC_BATCH_BYTES")) {
    const long long v = std::atoll(e);
    if (v > 0) budget = (size_t)v;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
    budget = std::min(budget, free_b / 2);
  else
    (void)hipGetLastError();
  return budget;
}

int max_batch_tasks() {
  int f = 1024;
  if (const char *e = std::getenv("GWC_MAX_BATCH")) {
    const int v = std::atoi(e);
    if (v > 0) f = v;
  }
  return f;
}

// Screening tasks of one kind (uniform border width R).
struct TaskList {
  std::vector<double2> z;
  std::vector<int> n, m;
  std::vector<long long> out_base;
  std::vector<int> out_stride;
  size_t size() const { return z.size(); }
};

struct Resident {
  const double *M_oo, *M_ov, *eps;
  int n_aux, n_occ, n_virt;
  const double *Lp;
  int n_aux_pad, ldl;
  const int2 *tiles;
  int n_tiles;
  // mixed-precision Pi build (precision != FP64)
  int precision = GWC_PREC_FP64;
  const float *Lf = nullptr;
  const unsigned short *Bhi = nullptr, *Blo = nullptr;
  const float *inv_colscale = nullptr, *acol = nullptr;
  const int2 *mx_tiles = nullptr;
  int mx_n_tiles = 0;
};

// Runs every task of `tl` (border width R) and writes W into W_out.
void run_screening(const Resident &rs, const TaskList &tl, int R, double2 *W_out,
                   std::vector<int> &status_all, hipStream_t s) {
  const size_t T = tl.size();
  if (T == 0) return;
  const int N = rs.n_aux;
  const int n = N + R;
  const int ldg = n;
  const size_t mat_elems = (size_t)n * ldg;
  const size_t mat_bytes = mat_elems * sizeof(double2);
  size_t fb = batch_budget_bytes() / std::max<size_t>(mat_bytes, 1);
  fb = std::min<size_t>(fb, (size_t)max_batch_tasks());
  fb = std::min(fb, T);
  if (fb < 1) fail(GWC_ERR_OUT_OF_MEMORY, "one %d x %d complex matrix (%zu bytes) exceeds the batch budget", n, n, mat_bytes);
  const int F = (int)fb;

  if (n > gwc::lu_max_order())
    fail(GWC_ERR_UNSUPPORTED, "bordered order %d exceeds %d", n, gwc::lu_max_order());
  DevBuf dG, dchr, dchi, dz, dn, dm, dob, dos, dbb, dst, dscr, dts;
  dG.alloc(mat_bytes * F);
  dscr.alloc(gwc::lu_scratch_bytes(F));
  dts.alloc((size_t)F * sizeof(float));
  dchr.alloc((size_t)F * rs.ldl * sizeof(double));
  dchi.alloc((size_t)F * rs.ldl * sizeof(double));
  dz.alloc(T * sizeof(double2));
  dn.alloc(T * sizeof(int));
  dm.alloc(T * sizeof(int));
  dob.alloc(T * sizeof(long long));
  dos.alloc(T * sizeof(int));
  dbb.alloc((size_t)F * R * sizeof(double));
  dst.alloc(T * sizeof(int));
  HIPCHECK(hipMemcpyAsync(dz.p, tl.z.data(), T * sizeof(double2), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(dn.p, tl.n.data(), T * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(dm.p, tl.m.data(), T * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(dob.p, tl.out_base.data(), T * sizeof(long long), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(dos.p, tl.out_stride.data(), T * sizeof(int), hipMemcpyHostToDevice, s));

  for (size_t t0 = 0; t0 < T; t0 += F) {
    const int Fb = (int)std::min<size_t>(F, T - t0);
    const double2 *z = dz.as<double2>() + t0;
    gwc::launch_chi(rs.eps, rs.n_occ, rs.n_virt, z, Fb, rs.ldl, dchr.as<double>(),
                    dchi.as<double>(), s);
    hipEvent_t ea = g_timing ? timing_mark(s) : nullptr;
    if (rs.precision == GWC_PREC_FP64) {
      gwc::launch_pi_build_f64(rs.Lp, rs.ldl, N, dchr.as<double>(), dchi.as<double>(), Fb,
                               rs.tiles, rs.n_tiles, dG.as<double2>(), (long long)mat_elems, ldg, s);
    } else {
      gwc::launch_pi_build_mixed(rs.precision, rs.Lf, rs.Bhi, rs.Blo, rs.ldl, N, dchr.as<double>(),
                                 dchi.as<double>(), rs.inv_colscale, rs.acol, dts.as<float>(), Fb,
                                 rs.mx_tiles, rs.mx_n_tiles, dG.as<double2>(), (long long)mat_elems,
                                 ldg, s);
    }
    if (g_timing) {
      double fl = 0.0;
      for (int t = 0; t < Fb; ++t) fl += (tl.z[t0 + t].x == 0.0 ? 1.0 : 2.0);
      fl *= (double)N * (N + 1) * (double)rs.n_occ * rs.n_virt;
      g_pending.push_back({rs.precision == GWC_PREC_FP64 ? 0 : 2, ea, timing_mark(s), fl});
    }
    gwc::launch_border(rs.M_oo, rs.M_ov, N, rs.n_occ, rs.n_virt, dn.as<int>() + t0,
                       dm.as<int>() + t0, Fb, R, dG.as<double2>(), (long long)mat_elems, ldg,
                       dbb.as<double>(), s);
    hipEvent_t eb = g_timing ? timing_mark(s) : nullptr;
    gwc::launch_lu_bordered(dG.as<double2>(), (long long)mat_elems, ldg, N, R, Fb,
                            dbb.as<double>(), dob.as<long long>() + t0, dos.as<int>() + t0, W_out,
                            dst.as<int>() + t0, dscr.p, s);
    if (g_timing) {
      const double fl = Fb * ((8.0 / 3.0) * N * (double)N * N + 8.0 * (double)N * N * R);
      g_pending.push_back({1, eb, timing_mark(s), fl});
    }
    HIPCHECK(hipGetLastError());
  }
  std::vector<int> st(T);
  HIPCHECK(hipMemcpyAsync(st.data(), dst.p, T * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  timing_resolve();
  status_all.insert(status_all.end(), st.begin(), st.end());
}

double prefactor(double eps_m, bool occupied, double omega) {
  if (occupied) {
    if (eps_m > omega) return -1.0;
    if (eps_m == omega) return -0.5;
    return 0.0;
  }
  if (eps_m < omega) return 1.0;
  if (eps_m == omega) return 0.5;
  return 0.0;
}

int sigma_core_impl(const gwc_system *sys, const gwc_sigma_args *args, gwc_sigma_out *out,
                    hipStream_t s) {
  if (!sys || !args || !out) fail(GWC_ERR_INVALID_ARG, "NULL system, args or out");
  const int N = sys->n_aux, no = sys->n_occ, nv = sys->n_virt;
  if (N < 1 || no < 1 || nv < 1) fail(GWC_ERR_SHAPE, "n_aux, n_occ, n_virt must be >= 1");
  if ((long long)no * nv > (1LL << 30) || N > (1 << 16))
    fail(GWC_ERR_SHAPE, "system too large (n_aux %d, n_occ*n_virt %lld)", N, (long long)no * nv);
  const int nb = no + nv;
  const int nc = args->n_core, ni = args->n_imag, nr = args->n_real;
  if (nc < 1 || ni < 1 || nr < 1) fail(GWC_ERR_SHAPE, "n_core, n_imag, n_real must be >= 1");
  if (!sys->eps || !sys->occ || !sys->M_oo || !sys->M_ov || !args->core_idx ||
      !args->omega_imag || !args->w_imag || !args->omega_real)
    fail(GWC_ERR_INVALID_ARG, "NULL input array");
  if (args->mode != GWC_MODE_FULL && args->mode != GWC_MODE_DECOUPLED)
    fail(GWC_ERR_INVALID_ARG, "unknown mode %d", args->mode);
  if (args->precision < GWC_PREC_FP64 || args->precision > GWC_PREC_FP8)
    fail(GWC_ERR_INVALID_ARG, "unknown precision %d", args->precision);
  if (args->precision == GWC_PREC_FP8)
    fail(GWC_ERR_UNSUPPORTED, "precision %d (FP8) is not implemented in this build", args->precision);
  const bool full = args->mode == GWC_MODE_FULL;
  if (full && !out->sigma_c) fail(GWC_ERR_INVALID_ARG, "sigma_c is required in FULL mode");

  // ---- small inputs: host copies for validation and task construction
  const std::vector<double> eps = to_host(sys->eps, nb, s);
  const std::vector<double> occ = to_host(sys->occ, nb, s);
  const std::vector<int> core = to_host(args->core_idx, nc, s);
  const std::vector<double> wi = to_host(args->omega_imag, ni, s);
  const std::vector<double> wwi = to_host(args->w_imag, ni, s);
  const std::vector<double> wr = to_host(args->omega_real, (size_t)nc * nr, s);
  std::vector<double> vxc(nc, 0.0);
  if (args->vxc) vxc = to_host(args->vxc, nc, s);

  if (!all_finite(eps) || !all_finite(occ) || !all_finite(wi) || !all_finite(wwi) ||
      !all_finite(wr) || !all_finite(vxc) || !std::isfinite(args->eta))
    fail(GWC_ERR_NONFINITE, "non-finite value in eps, occ, grids, eta or vxc");
  for (int m = 0; m < nb; ++m)
    if (occ[m] != (m < no ? 2.0 : 0.0))
      fail(GWC_ERR_INVALID_ARG, "occ[%d] = %g: occupations must be 2 for the first n_occ orbitals and 0 after", m, occ[m]);
  double max_occ = eps[0], min_virt = eps[no];
  for (int m = 0; m < no; ++m) max_occ = std::max(max_occ, eps[m]);
  for (int m = no; m < nb; ++m) min_virt = std::min(min_virt, eps[m]);
  if (!(max_occ < min_virt))
    fail(GWC_ERR_NONPOSITIVE_GAP, "highest occupied %g >= lowest virtual %g", max_occ, min_virt);
  for (int c = 0; c < nc; ++c)
    if (core[c] < 0 || core[c] >= no) fail(GWC_ERR_SHAPE, "core_idx[%d] = %d not in [0, n_occ)", c, core[c]);
  for (int k = 0; k < ni; ++k) {
    if (!(wi[k] > 0.0) || !(wwi[k] > 0.0)) fail(GWC_ERR_INVALID_ARG, "imaginary nodes and weights must be > 0");
    if (k > 0 && !(wi[k] > wi[k - 1])) fail(GWC_ERR_INVALID_ARG, "imaginary nodes must increase");
  }
  for (int c = 0; c < nc; ++c)
    for (int j = 1; j < nr; ++j)
      if (!(wr[(size_t)c * nr + j] > wr[(size_t)c * nr + j - 1]))
        fail(GWC_ERR_INVALID_ARG, "omega_real of core %d must increase", c);
  if (!(args->eta > 0.0)) fail(GWC_ERR_INVALID_ARG, "eta must be > 0");

  // ---- large inputs: device views, checked for non-finite values on device
  DevBuf hMoo, hMov, dflag;
  const size_t n_oo = (size_t)N * no * no, n_ovt = (size_t)N * no * nv;
  const double *dMoo = device_view(sys->M_oo, n_oo, hMoo, s);
  const double *dMov = device_view(sys->M_ov, n_ovt, hMov, s);
  dflag.alloc(sizeof(int));
  HIPCHECK(hipMemsetAsync(dflag.p, 0, sizeof(int), s));
  gwc::launch_nonfinite(dMoo, (long long)n_oo, dflag.as<int>(), s);
  gwc::launch_nonfinite(dMov, (long long)n_ovt, dflag.as<int>(), s);
  int flag = 0;
  HIPCHECK(hipMemcpyAsync(&flag, dflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (flag) fail(GWC_ERR_NONFINITE, "non-finite value in M_oo or M_ov");

  DevBuf deps, dcore, dwi, dwwi, dwr, dvxc;
  const double *d_eps = upload(deps, eps, s);
  const int *d_core = upload(dcore, core, s);
  const double *d_wi = upload(dwi, wi, s);
  const double *d_wwi = upload(dwwi, wwi, s);
  const double *d_wr = upload(dwr, wr, s);
  const double *d_vxc = upload(dvxc, vxc, s);

  // ---- pack L and the tile list of the upper triangle
  const int n_ov = no * nv;
  const int n_aux_pad = (int)round_up(N, gwc::L_ROW_ALIGN);
  const int ldl = (int)round_up(n_ov, gwc::L_COL_ALIGN);
  DevBuf dL, dtiles;
  dL.alloc((size_t)n_aux_pad * ldl * sizeof(double));
  gwc::launch_pack_l(dMov, N, n_ov, dL.as<double>(), n_aux_pad, ldl, s);
  std::vector<int2> tiles;
  const int nt = n_aux_pad / gwc::PI_TILE;
  for (int i = 0; i < nt; ++i)
    for (int j = i; j < nt; ++j) tiles.push_back(make_int2(i, j));
  const int2 *d_tiles = upload(dtiles, tiles, s);
  HIPCHECK(hipGetLastError());

  Resident rs{dMoo, dMov, d_eps, N, no, nv, dL.as<double>(), n_aux_pad, ldl, d_tiles,
              (int)tiles.size()};
  DevBuf dLf, dBh, dBl, dcs, dics, dacol, dmxt;
  if (args->precision != GWC_PREC_FP64) {
    // split operands for the mixed-precision Pi build, rows padded to 256
    const int rows_pad = (int)round_up(N, gwc::MX_TILE_COLS);
    const size_t elems = (size_t)rows_pad * ldl;
    dLf.alloc(elems * sizeof(float));
    dBh.alloc(elems * sizeof(unsigned short));
    dBl.alloc(elems * sizeof(unsigned short));
    dcs.alloc(ldl * sizeof(float));
    dics.alloc(ldl * sizeof(float));
    dacol.alloc(ldl * sizeof(float));
    gwc::launch_mixed_prep(args->precision, dL.as<double>(), n_aux_pad, rows_pad, ldl, dLf.as<float>(),
                           dBh.as<unsigned short>(), dBl.as<unsigned short>(), dcs.as<float>(),
                           dics.as<float>(), dacol.as<float>(), s);
    std::vector<int2> mt;
    const int nr_t = (N + gwc::MX_TILE_ROWS - 1) / gwc::MX_TILE_ROWS;
    const int nc_t = (N + gwc::MX_TILE_COLS - 1) / gwc::MX_TILE_COLS;
    for (int i = 0; i < nr_t; ++i)
      for (int j = 0; j < nc_t; ++j)
        if ((j + 1) * gwc::MX_TILE_COLS > i * gwc::MX_TILE_ROWS) mt.push_back(make_int2(i, j));
    rs.precision = args->precision;
    rs.Lf = dLf.as<float>();
    rs.Bhi = dBh.as<unsigned short>();
    rs.Blo = dBl.as<unsigned short>();
    rs.inv_colscale = args->precision == GWC_PREC_FP16X3 ? dics.as<float>() : nullptr;
    rs.acol = dacol.as<float>();
    rs.mx_tiles = upload(dmxt, mt, s);
    rs.mx_n_tiles = (int)mt.size();
    HIPCHECK(hipGetLastError());
  }
  std::vector<int> status;

  // ---- imaginary axis: W_imag[c][m][k]
  DevBuf dWi;
  dWi.alloc((size_t)nc * nb * ni * sizeof(double2));
  {
    TaskList tl;
    for (int k = 0; k < ni; ++k)
      for (int c = 0; c < nc; ++c) {
        tl.z.push_back(make_double2(0.0, wi[k]));
        tl.n.push_back(core[c]);
        tl.m.push_back(-1);
        tl.out_base.push_back((long long)c * nb * ni + k);
        tl.out_stride.push_back(ni);
      }
    run_screening(rs, tl, nb, dWi.as<double2>(), status, s);
  }

  // ---- residue tasks, ordered by (core, point, m); point nr is w = eps_n
  const int npts = nr + 1;
  TaskList tr;
  std::vector<double> ftask;
  std::vector<int> cj_off((size_t)nc * npts + 1, 0), cj_self((size_t)nc * npts, -1);
  for (int c = 0; c < nc; ++c) {
    const int nst = core[c];
    for (int j = 0; j < npts; ++j) {
      const double w = (j < nr) ? wr[(size_t)c * nr + j] : eps[nst];
      const size_t cj = (size_t)c * npts + j;
      cj_off[cj] = (int)tr.size();
      for (int m = 0; m < nb; ++m) {
        if (!full && j < nr && m != nst) continue;
        const double f = prefactor(eps[m], m < no, w);
        if (f == 0.0) continue;
        if (m == nst) cj_self[cj] = (int)tr.size();
        tr.z.push_back(make_double2(std::fabs(eps[m] - w), args->eta));
        tr.n.push_back(nst);
        tr.m.push_back(m);
        tr.out_base.push_back((long long)tr.size() - 1);
        tr.out_stride.push_back(0);
        ftask.push_back(f);
      }
    }
  }
  cj_off[(size_t)nc * npts] = (int)tr.size();
  DevBuf dWr;
  dWr.alloc(std::max<size_t>(tr.size(), 1) * sizeof(double2));
  run_screening(rs, tr, 1, dWr.as<double2>(), status, s);
  for (int v : status)
    if (v) fail(GWC_ERR_FACTORIZATION, "exactly singular pivot in the LU of 1 - Pi(z)");

  // ---- exchange, quadrature, assembly
  DevBuf dsx, dI, dft, dcjo, dcjs, dsig, dimd, dse, deq;
  dsx.alloc(nc * sizeof(double));
  gwc::launch_sigma_x(dMoo, N, no, d_core, nc, dsx.as<double>(), s);
  dI.alloc((size_t)nc * npts * sizeof(double));
  gwc::launch_quadrature(dWi.as<double2>(), d_eps, nb, d_wi, d_wwi, ni, d_wr, nr, d_core, nc,
                         full ? npts : 1, dI.as<double>(), s);
  const double *d_f = upload(dft, ftask, s);
  const int *d_cjo = upload(dcjo, cj_off, s);
  const int *d_cjs = upload(dcjs, cj_self, s);
  dsig.alloc((size_t)nc * nr * 2 * sizeof(double));
  dimd.alloc((size_t)nc * nr * sizeof(double));
  dse.alloc((size_t)nc * 2 * sizeof(double));
  deq.alloc((size_t)nc * sizeof(double));
  gwc::launch_assemble(dWr.as<double2>(), d_f, nullptr, d_cjo, d_cjs, dI.as<double>(), nc, nr,
                       d_eps, d_core, dsx.as<double>(), d_vxc, full ? 1 : 0, dsig.as<double>(),
                       dimd.as<double>(), dse.as<double>(), deq.as<double>(), s);
  HIPCHECK(hipGetLastError());
  if (full) copy_out(out->sigma_c, dsig.p, (size_t)nc * nr * 2 * sizeof(double), s);
  copy_out(out->im_sigma_dec, dimd.p, (size_t)nc * nr * sizeof(double), s);
  copy_out(out->sigma_c_eps, dse.p, (size_t)nc * 2 * sizeof(double), s);
  copy_out(out->sigma_x, dsx.p, (size_t)nc * sizeof(double), s);
  copy_out(out->e_qp, deq.p, (size_t)nc * sizeof(double), s);
  HIPCHECK(hipStreamSynchronize(s));
  return GWC_OK;
}

int spectral_cumulant_impl(const gwc_cumulant_args *a, double *A_out, double *z_out,
                           hipStream_t s) {
  if (!a || !A_out) fail(GWC_ERR_INVALID_ARG, "NULL args or A_out");
  if (!a->omega_real || !a->im_sigma) fail(GWC_ERR_INVALID_ARG, "NULL omega_real or im_sigma");
  if (a->n_real < 1) fail(GWC_ERR_SHAPE, "n_real must be >= 1");
  const int nt = a->n_t;
  if (nt < 16 || nt > (1 << 24) || (nt & (nt - 1)) != 0)
    fail(GWC_ERR_SHAPE, "n_t = %d must be a power of two in [2^4, 2^24]", nt);
  if (a->n_out < 1 || a->n_out > nt) fail(GWC_ERR_SHAPE, "n_out must be in [1, n_t]");
  if (!std::isfinite(a->eps_n) || !std::isfinite(a->e_qp) || !std::isfinite(a->eta) ||
      !std::isfinite(a->d_omega) || !std::isfinite(a->omega_out_min))
    fail(GWC_ERR_NONFINITE, "non-finite scalar argument");
  if (!(a->eta > 0.0)) fail(GWC_ERR_INVALID_ARG, "eta must be > 0");
  if (!(a->d_omega > 0.0)) fail(GWC_ERR_INVALID_ARG, "d_omega must be > 0");
  const std::vector<double> w = to_host(a->omega_real, a->n_real, s);
  const std::vector<double> im = to_host(a->im_sigma, a->n_real, s);
  if (!all_finite(w) || !all_finite(im)) fail(GWC_ERR_NONFINITE, "non-finite grid or Im Sigma");
  for (int j = 1; j < a->n_real; ++j)
    if (!(w[j] > w[j - 1])) fail(GWC_ERR_INVALID_ARG, "omega_real must increase");

  int log2n = 0;
  while ((1 << log2n) < nt) ++log2n;
  const double PI_D = 3.14159265358979323846;
  const double dt = 2.0 * PI_D / ((double)nt * a->d_omega);

  DevBuf dw, dim, dnu, dc, dz, dA, dB, dAout;
  const double *d_w = upload(dw, w, s);
  const double *d_im = upload(dim, im, s);
  dnu.alloc(a->n_real * sizeof(double));
  dc.alloc(a->n_real * sizeof(double));
  dz.alloc(2 * sizeof(double));
  dA.alloc((size_t)nt * sizeof(double2));
  dB.alloc((size_t)nt * sizeof(double2));
  dAout.alloc((size_t)a->n_out * sizeof(double));
  gwc::launch_cumulant_weights(d_w, d_im, a->n_real, a->eps_n, dnu.as<double>(), dc.as<double>(),
                               dz.as<double>(), s);
  gwc::launch_cumulant_time(dnu.as<double>(), dc.as<double>(), a->n_real, nt, dt, a->e_qp,
                            a->omega_out_min, a->eta, dA.as<double2>(), s);
  double2 *res = nullptr;
  gwc::launch_fft_inverse(dA.as<double2>(), dB.as<double2>(), log2n, &res, s);
  gwc::launch_extract_spectrum(res, a->n_out, dAout.as<double>(), s);
  HIPCHECK(hipGetLastError());
  copy_out(A_out, dAout.p, (size_t)a->n_out * sizeof(double), s);
  if (z_out) copy_out(z_out, dz.p, 2 * sizeof(double), s);
  HIPCHECK(hipStreamSynchronize(s));
  return GWC_OK;
}

template <class F>
int guarded(F &&fn) {
  std::lock_guard<std::mutex> lock(g_mutex);
  g_last_error.clear();
  try {
    return fn();
  } catch (const GwcError &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return GWC_ERR_DEVICE;
  } catch (...) {
    g_last_error = "unknown error";
    return GWC_ERR_DEVICE;
  }
}

}  // namespace

extern "C" {

int gwc_sigma_core(const gwc_system *sys, const gwc_sigma_args *args, gwc_sigma_out *out,
                   void *hip_stream) {
  return guarded([&] { return sigma_core_impl(sys, args, out, (hipStream_t)hip_stream); });
}

int gwc_spectral_cumulant(const gwc_cumulant_args *args, double *A_out, double *z_out,
                          void *hip_stream) {
  return guarded([&] { return spectral_cumulant_impl(args, A_out, z_out, (hipStream_t)hip_stream); });
}

int gwc_timing_enable(int on) {
  std::lock_guard<std::mutex> lock(g_mutex);
  for (auto &p : g_pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
  for (int k = 0; k < kNumTimed; ++k) g_stats[k] = TimerStat{};
  g_timing = on != 0;
  return GWC_OK;
}

int gwc_timing_get(const char *kernel, double *total_ms, long long *launches, double *flops) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!kernel) return GWC_ERR_INVALID_ARG;
  for (int k = 0; k < kNumTimed; ++k) {
    if (std::string(kernel) == kTimedKernels[k]) {
      if (total_ms) *total_ms = g_stats[k].total_ms;
      if (launches) *launches = g_stats[k].launches;
      if (flops) *flops = g_stats[k].flops;
      return GWC_OK;
    }
  }
  return GWC_ERR_INVALID_ARG;
}

const char *gwc_last_error(void) { return g_last_error.c_str(); }

int gwc_version(void) { return GWC_VERSION; }

}  // extern "C"
