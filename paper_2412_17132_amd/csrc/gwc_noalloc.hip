// gwc_spectral_cumulant_noalloc: the cumulant spectral function with no device
// allocation, for callers that cannot allocate (code under stream capture,
// tight serving loops).  Same kernels and results as gwc_spectral_cumulant;
// their buffers live in one file-scope device array per GPU instead of the
// stream-ordered pool.
//
// The array's device address is taken with hipGetSymbolAddress once per
// device (the first call on that device, with it current) and kept in
// g_scratch_ptr[device]; host code only ever passes that address, never the
// array's own name (on the host the name is a stand-in, not a device address).
//
// Layout (doubles, each part 256-byte aligned):
//   Ga, Gb   [NT_MAX] double2   the time-domain propagator and the FFT ping-pong
//   Aout     [NT_MAX]           the spectral function before copy-out
//   w, im    [NR_MAX]           the staged real grid and Im Sigma
//   nu, c    [NR_MAX]           nu_j = w_j - eps_n and the cumulant weights
//   z        [2]                (Z, 1 - Z)
//   flag     [1]                input checks (written whole by one block)
// Nothing needs to start at zero: every element a call reads it has written
// first.  Calls that overlap on one GPU share the array and race.
#include <cmath>
#include <cstdarg>
#include <mutex>
#include <string>

#include "gwc.h"
#include "gwc_host.h"
#include "gwc_internal.h"

namespace {

constexpr int NT_MAX = 1 << 19;   // time points (twice the paper's 2^18)
constexpr int NR_MAX = 1 << 15;   // real-grid points
constexpr size_t OFF_GA = 0;
constexpr size_t OFF_GB = OFF_GA + 2 * (size_t)NT_MAX;
constexpr size_t OFF_AOUT = OFF_GB + 2 * (size_t)NT_MAX;
constexpr size_t OFF_W = OFF_AOUT + (size_t)NT_MAX;
constexpr size_t OFF_IM = OFF_W + NR_MAX;
constexpr size_t OFF_NU = OFF_IM + NR_MAX;
constexpr size_t OFF_C = OFF_NU + NR_MAX;
constexpr size_t OFF_Z = OFF_C + NR_MAX;
constexpr size_t OFF_FLAG = OFF_Z + 32;
constexpr size_t SCRATCH_DOUBLES = OFF_FLAG + 32;  // 22,020,608 bytes

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[MAX_DEVICES] = {};

constexpr int FLAG_NONFINITE = 1, FLAG_ORDER = 2;

// One block: flag = NONFINITE if a grid value or Im Sigma is not finite, else
// ORDER if the grid does not increase strictly, else 0.
__global__ void __launch_bounds__(256)
check_inputs_kernel(const double *__restrict__ w, const double *__restrict__ im, int n, int *flag) {
  __shared__ int sh[256];
  int bits = 0;
  for (int j = threadIdx.x; j < n; j += 256) {
    if (!isfinite(w[j]) || !isfinite(im[j])) bits |= FLAG_NONFINITE;
    if (j > 0 && !(w[j] > w[j - 1])) bits |= FLAG_ORDER;
  }
  sh[threadIdx.x] = bits;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] |= sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) flag[0] = sh[0];
}

void check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    gwc::fail(GWC_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  }
}

// The device address of this GPU's scratch array (looked up on first use).
double *scratch_on_current_device() {
  int dev = 0;
  check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) gwc::fail(GWC_ERR_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) gwc::fail(GWC_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  return g_scratch_ptr[dev];
}

void run_cumulant_noalloc(const gwc_cumulant_args *a, double *A_out, double *z_out, hipStream_t s) {
  if (!a || !A_out) gwc::fail(GWC_ERR_INVALID_ARG, "NULL args or A_out");
  if (!a->omega_real || !a->im_sigma) gwc::fail(GWC_ERR_INVALID_ARG, "NULL omega_real or im_sigma");
  if (a->n_real < 1) gwc::fail(GWC_ERR_SHAPE, "n_real must be >= 1");
  if (a->n_real > NR_MAX)
    gwc::fail(GWC_ERR_SHAPE, "n_real = %d exceeds the no-allocation limit %d", a->n_real, NR_MAX);
  const int nt = a->n_t;
  if (nt < 16 || nt > (1 << 24) || (nt & (nt - 1)) != 0)
    gwc::fail(GWC_ERR_SHAPE, "n_t = %d must be a power of two in [2^4, 2^24]", nt);
  if (nt > NT_MAX)
    gwc::fail(GWC_ERR_SHAPE, "n_t = %d exceeds the no-allocation limit %d", nt, NT_MAX);
  if (a->n_out < 1 || a->n_out > nt) gwc::fail(GWC_ERR_SHAPE, "n_out must be in [1, n_t]");
  if (!std::isfinite(a->eps_n) || !std::isfinite(a->e_qp) || !std::isfinite(a->eta) ||
      !std::isfinite(a->d_omega) || !std::isfinite(a->omega_out_min))
    gwc::fail(GWC_ERR_NONFINITE, "non-finite scalar argument");
  if (!(a->eta > 0.0)) gwc::fail(GWC_ERR_INVALID_ARG, "eta must be > 0");
  if (!(a->d_omega > 0.0)) gwc::fail(GWC_ERR_INVALID_ARG, "d_omega must be > 0");

  double *base = scratch_on_current_device();
  double2 *Ga = reinterpret_cast<double2 *>(base + OFF_GA);
  double2 *Gb = reinterpret_cast<double2 *>(base + OFF_GB);
  double *Aout = base + OFF_AOUT, *w = base + OFF_W, *im = base + OFF_IM;
  double *nu = base + OFF_NU, *c = base + OFF_C, *z = base + OFF_Z;
  int *flag = reinterpret_cast<int *>(base + OFF_FLAG);
  const size_t nr_bytes = (size_t)a->n_real * sizeof(double);
  check(hipMemcpyAsync(w, a->omega_real, nr_bytes, hipMemcpyDefault, s), "staging omega_real");
  check(hipMemcpyAsync(im, a->im_sigma, nr_bytes, hipMemcpyDefault, s), "staging im_sigma");
  check_inputs_kernel<<<1, 256, 0, s>>>(w, im, a->n_real, flag);

  int log2n = 0;
  while ((1 << log2n) < nt) ++log2n;
  const double PI_D = 3.14159265358979323846;
  const double dt = 2.0 * PI_D / ((double)nt * a->d_omega);
  gwc::launch_cumulant_weights(w, im, a->n_real, a->eps_n, nu, c, z, s);
  gwc::launch_cumulant_time(nu, c, a->n_real, nt, dt, a->e_qp, a->omega_out_min, a->eta, Ga, s);
  double2 *res = nullptr;
  gwc::launch_fft_inverse(Ga, Gb, log2n, &res, s);
  gwc::launch_extract_spectrum(res, a->n_out, Aout, s);
  check(hipGetLastError(), "kernel launch");
  check(hipMemcpyAsync(A_out, Aout, (size_t)a->n_out * sizeof(double), hipMemcpyDefault, s),
        "copying A out");
  if (z_out) check(hipMemcpyAsync(z_out, z, 2 * sizeof(double), hipMemcpyDefault, s), "copying Z out");
  int h_flag = 0;
  check(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s), "reading the input flag");
  check(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (h_flag & FLAG_NONFINITE) gwc::fail(GWC_ERR_NONFINITE, "non-finite grid or Im Sigma");
  if (h_flag & FLAG_ORDER) gwc::fail(GWC_ERR_INVALID_ARG, "omega_real must increase");
}

}  // namespace

extern "C" int gwc_spectral_cumulant_noalloc(const gwc_cumulant_args *args, double *A_out,
                                             double *z_out, void *hip_stream) {
  std::string &err = gwc::last_error();
  err.clear();
  try {
    run_cumulant_noalloc(args, A_out, z_out, (hipStream_t)hip_stream);
    return GWC_OK;
  } catch (const gwc::GwcError &e) {
    err = e.msg;
    return e.code;
  } catch (const std::exception &e) {
    err = e.what();
    return GWC_ERR_DEVICE;
  } catch (...) {
    err = "unknown error";
    return GWC_ERR_DEVICE;
  }
}
