// C ABI of libgwc: argument validation, staging, task lists and the launch
// sequence of the contour-deformation self-energy and the cumulant tail.
//
// run_sigma, in order (paper section "Self-energy evaluation"):
//   1. (resident system) L = M_ov packed into a zero-padded N_aux x N_ov buffer;
//   2. imaginary axis: one task per (node w_k, core n) with all b_nm as border
//      vectors -> W^c_nm(i w_k) for every m (input of Eq. cd_imaginary);
//   3. residues: one task per (core n, point w, orbital m) with f_m != 0
//      (Eq. cd_prefactors, Theta(0) = 1/2) at z = |eps_m - w| + i eta
//      (Eq. cd_residue) -> W^c_nm(z);
//      each task batch runs chi -> Pi build (MFMA) -> border -> bordered LU;
//   4. exchange, imaginary-axis quadrature, residue sums and E_QP (Eqs. cd_terms,
//      sigma_x, QPGWC).
// Calls from several host threads run concurrently (each on its own stream);
// temporaries come from the stream-ordered allocator.
#include <algorithm>
#include <limits>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gwc.h"
#include "gwc_host.h"
#include "gwc_internal.h"

namespace gwc {

void fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw GwcError{code, std::string(buf)};
}

}  // namespace gwc

namespace {

using gwc::fail;
using gwc::GwcError;


#define HIPCHECK(x)                                                                           \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess)                                                                     \
      fail(e_ == hipErrorOutOfMemory ? GWC_ERR_OUT_OF_MEMORY : GWC_ERR_DEVICE, "%s: %s", #x, \
           hipGetErrorString(e_));                                                            \
  } while (0)

// ---------------------------------------------------------------------------
// Kernel timing (diagnostics): event pairs recorded around hot launches on the
// launch stream, folded into the counters once that stream has synchronised.
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
constexpr int kNumTimed = 6;
const char *const kTimedKernels[kNumTimed] = {"pi_build_f64", "lu_bordered", "pi_build_mixed",
                                              "jacobi_apply", "jacobi_pairs", "ldlt_bordered"};
std::mutex g_timing_mutex;
std::atomic<bool> g_timing{false};
TimerStat g_stats[kNumTimed];

hipEvent_t timing_mark(hipStream_t s) {
  hipEvent_t e;
  HIPCHECK(hipEventCreate(&e));
  HIPCHECK(hipEventRecord(e, s));
  return e;
}

// Folds recorded event pairs into the counters (their stream must be idle).
void timing_resolve(std::vector<PendingTiming> &pending) {
  std::lock_guard<std::mutex> lock(g_timing_mutex);
  for (auto &p : pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      if (g_timing) {
        g_stats[p.kernel].total_ms += ms;
        g_stats[p.kernel].launches += 1;
        g_stats[p.kernel].flops += p.flops;
      }
    } else {
      (void)hipGetLastError();
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  pending.clear();
}

// ---------------------------------------------------------------------------
// Temporary device memory: a cache of device blocks by size class.
//
// A stream-ordered pool (hipMallocAsync) maps new memory whenever none of its
// freed blocks may go to the asking stream, and such a growth by several GB
// held every stream of the device for up to seconds: serving workers on
// their own streams, whose batch buffers reach a quarter of the HBM budget,
// met it on many requests.  Here a freed block waits in its size class with
// an event recorded on the freeing stream; it goes out again at once to the
// same stream (stream order covers it) and to another stream once the event
// has completed.  Only a miss allocates (hipMalloc).  Idle blocks are kept
// up to half the device's memory (beyond that the oldest are freed), and an
// allocation that fails first frees every idle block and tries again.
// Classes: powers of two up to 1 MiB, above that multiples of 1/32 of the
// next power of two (at most about 6 % of a block unused).
size_t cache_class(size_t bytes) {
  if (bytes <= 256) return 256;
  size_t p = 1;
  while (p < bytes) p <<= 1;
  if (p <= ((size_t)1 << 20)) return p;
  const size_t q = p >> 5;
  return (bytes + q - 1) / q * q;
}

class DeviceCache {
 public:
  // A block of `cls` bytes for use on stream s, or nullptr when the device
  // has none to give.
  void *get(size_t cls, hipStream_t s) {
    {
      // a pending event's query leaves hipErrorNotReady as the thread's last
      // error: cleared unless an earlier error is waiting to be reported
      const bool clean = hipPeekAtLastError() == hipSuccess;
      std::lock_guard<std::mutex> lock(mu_);
      for (size_t i = idle_.size(); i-- > 0;) {
        Block &b = idle_[i];
        if (b.cls != cls) continue;
        bool ready = b.s == s || !b.ev;
        if (!ready) {
          ready = hipEventQuery(b.ev) == hipSuccess;
          if (clean) (void)hipGetLastError();
        }
        if (!ready) continue;
        void *p = b.p;
        if (b.ev) (void)hipEventDestroy(b.ev);
        idle_bytes_ -= b.cls;
        idle_.erase(idle_.begin() + (long)i);
        return p;
      }
    }
    void *p = nullptr;
    if (hipMalloc(&p, cls) != hipSuccess) {
      (void)hipGetLastError();
      trim(0);
      p = nullptr;
      if (hipMalloc(&p, cls) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    return p;
  }
  // Bytes held idle (free for the library's next temporaries).
  size_t idle_bytes() {
    std::lock_guard<std::mutex> lock(mu_);
    return idle_bytes_;
  }
  // Takes back a block last used on stream s.
  void put(void *p, size_t cls, hipStream_t s) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, s) != hipSuccess) {
      (void)hipGetLastError();
      if (ev) (void)hipEventDestroy(ev);
      ev = nullptr;
      (void)hipStreamSynchronize(s);  // no event: the block is idle once the stream is
      (void)hipGetLastError();
    }
    size_t over = 0;
    {
      std::lock_guard<std::mutex> lock(mu_);
      idle_.push_back(Block{p, cls, s, ev});
      idle_bytes_ += cls;
      if (idle_bytes_ > cap()) over = idle_bytes_ - cap();
    }
    if (over) trim(cap());
  }

 private:
  struct Block {
    void *p;
    size_t cls;
    hipStream_t s;
    hipEvent_t ev;
  };
  size_t cap() {
    if (!cap_) {
      size_t free_b = 0, total = 0;
      if (hipMemGetInfo(&free_b, &total) != hipSuccess) {
        (void)hipGetLastError();
        total = (size_t)64 << 30;
      }
      cap_ = total / 2;
    }
    return cap_;
  }
  // Frees idle blocks, oldest first, until at most `keep` bytes stay idle.
  void trim(size_t keep) {
    std::vector<Block> out;
    {
      std::lock_guard<std::mutex> lock(mu_);
      size_t k = 0;
      while (k < idle_.size() && idle_bytes_ > keep) {
        idle_bytes_ -= idle_[k].cls;
        out.push_back(idle_[k]);
        ++k;
      }
      idle_.erase(idle_.begin(), idle_.begin() + (long)k);
    }
    for (Block &b : out) {
      if (b.ev) {
        (void)hipEventSynchronize(b.ev);
        (void)hipEventDestroy(b.ev);
      }
      (void)hipFree(b.p);
    }
    (void)hipGetLastError();
  }
  std::mutex mu_;
  std::vector<Block> idle_;  // oldest first
  size_t idle_bytes_ = 0, cap_ = 0;
};

constexpr int CACHE_DEVICES = 16;
DeviceCache &device_cache() {
  static DeviceCache caches[CACHE_DEVICES];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  return caches[dev >= 0 && dev < CACHE_DEVICES ? dev : 0];
}

// A temporary of one call, used on stream s and returned to the cache at
// scope exit (in stream order).
struct DevBuf {
  void *p = nullptr;
  size_t cls = 0;
  hipStream_t s = nullptr;
  DeviceCache *cache = nullptr;
  explicit DevBuf(hipStream_t stream) : s(stream) {}
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) cache->put(p, cls, s);
    p = nullptr;
  }
  void alloc(size_t bytes) {
    release();
    if (bytes == 0) bytes = 16;
    cache = &device_cache();
    cls = cache_class(bytes);
    p = cache->get(cls, s);
    if (!p) fail(GWC_ERR_OUT_OF_MEMORY, "allocation of %zu bytes failed", bytes);
  }
  template <class T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

// Long-lived allocation (resident systems).
struct PersistBuf {
  void *p = nullptr;
  size_t bytes = 0;
  PersistBuf() = default;
  PersistBuf(const PersistBuf &) = delete;
  PersistBuf &operator=(const PersistBuf &) = delete;
  ~PersistBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t b) {
    if (p) (void)hipFree(p);
    p = nullptr;
    if (b == 0) b = 16;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      fail(e == hipErrorOutOfMemory ? GWC_ERR_OUT_OF_MEMORY : GWC_ERR_DEVICE,
           "hipMalloc of %zu bytes failed: %s", b, hipGetErrorString(e));
    }
    bytes = b;
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

template <class T, class Buf>
T *upload(Buf &buf, const std::vector<T> &v, hipStream_t s) {
  buf.alloc(v.size() * sizeof(T));
  if (!v.empty())
    HIPCHECK(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return buf.template as<T>();
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

size_t default_batch_bytes() {
  size_t budget = size_t(48) << 30;
  if (const char *e = std::getenv("GWC_BATCH_BYTES")) {
    const long long v = std::atoll(e);
    if (v > 0) budget = (size_t)v;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
    budget = std::min(budget, (free_b + device_cache().idle_bytes()) / 2);  // idle cached blocks count as free
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

// Screening tasks of one kind (uniform border width R).
struct TaskList {
  std::vector<double2> z;
  std::vector<int> n, m;
  std::vector<long long> out_base;
  std::vector<int> out_stride;
  size_t size() const { return z.size(); }
};

}  // namespace

namespace gwc {

struct MixedOperands {
  PersistBuf Lf, Bh, Bl, cs, ics, acol, tiles;
  int n_tiles = 0;
  bool ready = false;
};

struct ResidentSystem {
  int N = 0, no = 0, nv = 0, nb = 0, n_ov = 0, n_aux_pad = 0, ldl = 0;
  std::vector<double> eps, occ;  // host copies
  PersistBuf d_eps, d_Moo, d_Mov, d_L, d_tiles;
  int n_tiles = 0;
  std::mutex mixed_mutex;
  MixedOperands mixed[4];  // by precision (1, 2, 3)
};

int resident_n_occ(const ResidentSystem &rs) { return rs.no; }
int resident_n_basis(const ResidentSystem &rs) { return rs.nb; }
double resident_eps(const ResidentSystem &rs, int m) { return rs.eps[m]; }

std::string &last_error() {
  static thread_local std::string msg;
  return msg;
}

size_t resident_bytes(const ResidentSystem &rs) {
  size_t b = rs.d_eps.bytes + rs.d_Moo.bytes + rs.d_Mov.bytes + rs.d_L.bytes + rs.d_tiles.bytes;
  for (const auto &m : rs.mixed)
    b += m.Lf.bytes + m.Bh.bytes + m.Bl.bytes + m.cs.bytes + m.ics.bytes + m.acol.bytes + m.tiles.bytes;
  return b;
}

ResidentSystem *create_resident(const gwc_system *sys, hipStream_t s) {
  if (!sys) fail(GWC_ERR_INVALID_ARG, "NULL system");
  const int N = sys->n_aux, no = sys->n_occ, nv = sys->n_virt;
  if (N < 1 || no < 1 || nv < 1) fail(GWC_ERR_SHAPE, "n_aux, n_occ, n_virt must be >= 1");
  if ((long long)no * nv > (1LL << 30) || N > (1 << 16))
    fail(GWC_ERR_SHAPE, "system too large (n_aux %d, n_occ*n_virt %lld)", N, (long long)no * nv);
  if (!sys->eps || !sys->occ || !sys->M_oo || !sys->M_ov) fail(GWC_ERR_INVALID_ARG, "NULL input array");
  std::unique_ptr<ResidentSystem> rs(new ResidentSystem());
  rs->N = N; rs->no = no; rs->nv = nv; rs->nb = no + nv; rs->n_ov = no * nv;
  const int nb = rs->nb;
  rs->eps = to_host(sys->eps, nb, s);
  rs->occ = to_host(sys->occ, nb, s);
  if (!all_finite(rs->eps) || !all_finite(rs->occ)) fail(GWC_ERR_NONFINITE, "non-finite value in eps or occ");
  for (int m = 0; m < nb; ++m)
    if (rs->occ[m] != (m < no ? 2.0 : 0.0))
      fail(GWC_ERR_INVALID_ARG, "occ[%d] = %g: occupations must be 2 for the first n_occ orbitals and 0 after", m, rs->occ[m]);
  double max_occ = rs->eps[0], min_virt = rs->eps[no];
  for (int m = 0; m < no; ++m) max_occ = std::max(max_occ, rs->eps[m]);
  for (int m = no; m < nb; ++m) min_virt = std::min(min_virt, rs->eps[m]);
  if (!(max_occ < min_virt))
    fail(GWC_ERR_NONPOSITIVE_GAP, "highest occupied %g >= lowest virtual %g", max_occ, min_virt);

  const size_t n_oo = (size_t)N * no * no, n_ovt = (size_t)N * no * nv;
  rs->d_Moo.alloc(n_oo * sizeof(double));
  rs->d_Mov.alloc(n_ovt * sizeof(double));
  HIPCHECK(hipMemcpyAsync(rs->d_Moo.p, sys->M_oo, n_oo * sizeof(double), hipMemcpyDefault, s));
  HIPCHECK(hipMemcpyAsync(rs->d_Mov.p, sys->M_ov, n_ovt * sizeof(double), hipMemcpyDefault, s));
  DevBuf dflag(s);
  dflag.alloc(sizeof(int));
  HIPCHECK(hipMemsetAsync(dflag.p, 0, sizeof(int), s));
  launch_nonfinite(rs->d_Moo.as<double>(), (long long)n_oo, dflag.as<int>(), s);
  launch_nonfinite(rs->d_Mov.as<double>(), (long long)n_ovt, dflag.as<int>(), s);
  int flag = 0;
  HIPCHECK(hipMemcpyAsync(&flag, dflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (flag) fail(GWC_ERR_NONFINITE, "non-finite value in M_oo or M_ov");
  upload(rs->d_eps, rs->eps, s);

  rs->n_aux_pad = (int)round_up(N, L_ROW_ALIGN);
  rs->ldl = (int)round_up(rs->n_ov, L_COL_ALIGN);
  rs->d_L.alloc((size_t)rs->n_aux_pad * rs->ldl * sizeof(double));
  launch_pack_l(rs->d_Mov.as<double>(), N, rs->n_ov, rs->d_L.as<double>(), rs->n_aux_pad, rs->ldl, s);
  std::vector<int2> tiles;
  const int nt = rs->n_aux_pad / PI_TILE;
  for (int i = 0; i < nt; ++i)
    for (int j = i; j < nt; ++j) tiles.push_back(make_int2(i, j));
  upload(rs->d_tiles, tiles, s);
  rs->n_tiles = (int)tiles.size();
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));
  return rs.release();
}

void destroy_resident(ResidentSystem *rs) { delete rs; }

// Tiles of the mixed-precision Pi build that touch the upper triangle.
std::vector<int2> mixed_tiles(int N, int prec) {
  std::vector<int2> mt;
  const int tr = mixed_tile_rows(prec);
  const int nr_t = (N + tr - 1) / tr;
  const int nc_t = (N + MX_TILE_COLS - 1) / MX_TILE_COLS;
  for (int i = 0; i < nr_t; ++i)
    for (int j = 0; j < nc_t; ++j)
      if ((j + 1) * MX_TILE_COLS > i * tr) mt.push_back(make_int2(i, j));
  return mt;
}

// Device bytes of the split operands of one precision (the A source L, hi and
// lo parts, column scales, tile list), rows padded to 256 and columns to the
// form's K chunk.
size_t split_operand_bytes(const ResidentSystem &rs, int prec) {
  const int rows_pad = (int)round_up(rs.N, MX_TILE_COLS);
  const size_t elems = (size_t)rows_pad * mixed_ldl(prec, rs.ldl);
  return elems * (mixed_a_bytes(prec) + 2 * mixed_b_bytes(prec)) + 3 * (size_t)rs.ldl * sizeof(float) +
         mixed_tiles(rs.N, prec).size() * sizeof(int2);
}

size_t mixed_operand_bytes(ResidentSystem &rs, int prec) {
  if (prec == GWC_PREC_FP64) return 0;
  std::lock_guard<std::mutex> lock(rs.mixed_mutex);
  return rs.mixed[prec].ready ? 0 : split_operand_bytes(rs, prec);
}

// Split operands of the mixed-precision Pi build, created once per system and
// precision (rows padded to 256); *built (when given) receives the bytes this
// call allocated (0 when they existed).
const MixedOperands &mixed_operands(ResidentSystem &rs, int prec, hipStream_t s, size_t *built) {
  std::lock_guard<std::mutex> lock(rs.mixed_mutex);
  MixedOperands &m = rs.mixed[prec];
  if (built) *built = 0;
  if (m.ready) return m;
  const int rows_pad = (int)round_up(rs.N, MX_TILE_COLS);
  const int ldlk = mixed_ldl(prec, rs.ldl);
  const size_t elems = (size_t)rows_pad * ldlk;
  m.Lf.alloc(elems * mixed_a_bytes(prec));
  m.Bh.alloc(elems * mixed_b_bytes(prec));
  m.Bl.alloc(elems * mixed_b_bytes(prec));
  m.cs.alloc(rs.ldl * sizeof(float));
  m.ics.alloc(rs.ldl * sizeof(float));
  m.acol.alloc(rs.ldl * sizeof(float));
  launch_mixed_prep(prec, rs.d_L.as<double>(), rs.n_aux_pad, rows_pad, rs.ldl, ldlk,
                    m.Lf.p, m.Bh.p, m.Bl.p, m.cs.as<float>(), m.ics.as<float>(),
                    m.acol.as<float>(), s);
  const std::vector<int2> mt = mixed_tiles(rs.N, prec);
  upload(m.tiles, mt, s);
  m.n_tiles = (int)mt.size();
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));
  m.ready = true;
  if (built)
    *built = m.Lf.bytes + m.Bh.bytes + m.Bl.bytes + m.cs.bytes + m.ics.bytes + m.acol.bytes + m.tiles.bytes;
  return m;
}

size_t prepare_mixed_operands(ResidentSystem &rs, int prec, hipStream_t s) {
  if (prec == GWC_PREC_FP64) return 0;
  size_t built = 0;
  (void)mixed_operands(rs, prec, s, &built);
  return built;
}

namespace {

struct BatchPlan {
  int F = 0;
  size_t mat_bytes = 0, bytes = 0;
};

BatchPlan plan_batch(const ResidentSystem &rs, size_t T, int R, size_t batch_bytes) {
  BatchPlan p;
  if (T == 0) return p;
  const size_t n = (size_t)rs.N + R;
  p.mat_bytes = n * n * sizeof(double2);
  size_t fb = batch_bytes / std::max<size_t>(p.mat_bytes, 1);
  fb = std::min<size_t>(fb, (size_t)max_batch_tasks());
  fb = std::min(fb, T);
  p.F = (int)fb;
  p.bytes = fb * p.mat_bytes + std::max(lu_scratch_bytes((int)std::max<size_t>(fb, 1)),
                                          ldlt_scratch_bytes((int)std::max<size_t>(fb, 1), rs.N)) +
            fb * (2 * (size_t)rs.ldl * (sizeof(double) + sizeof(float)) + R * sizeof(double) + sizeof(float)) +
            T * (sizeof(double2) + 3 * sizeof(int) + sizeof(long long) + sizeof(int)) + 4096;
  return p;
}

// Factorisation of the bordered matrices: LDL^T without pivoting (default;
// 1 - Pi(z) is complex symmetric with a positive semidefinite imaginary part,
// or real SPD on the imaginary axis) or the partial-pivoting LU
// (GWC_FACTORIZATION=lu, and the retry of any matrix whose LDL^T met an
// exactly zero pivot).
enum Factorization { FACT_LDLT = 0, FACT_LU = 1 };

Factorization default_factorization() {
  const char *e = std::getenv("GWC_FACTORIZATION");
  return (e && std::string(e) == "lu") ? FACT_LU : FACT_LDLT;
}

// Runs every task of `tl` (border width R) and writes W into W_out.
void run_screening(ResidentSystem &rs, const MixedOperands *mx, int precision, const TaskList &tl,
                   int R, double2 *W_out, std::vector<int> &status_all, hipStream_t s,
                   size_t batch_bytes, Factorization fact = default_factorization()) {
  const size_t T = tl.size();
  if (T == 0) return;
  const int N = rs.N;
  const int n = N + R;
  const int ldg = n;
  if (n > lu_max_order()) fail(GWC_ERR_UNSUPPORTED, "bordered order %d exceeds %d", n, lu_max_order());
  const BatchPlan plan = plan_batch(rs, T, R, batch_bytes);
  if (plan.F < 1)
    fail(GWC_ERR_OUT_OF_MEMORY, "one %d x %d complex matrix (%zu bytes) exceeds the batch budget", n, n, plan.mat_bytes);
  const int F = plan.F;
  const size_t mat_elems = (size_t)n * ldg;

  DevBuf dG(s), dchr(s), dchi(s), dz(s), dn(s), dm(s), dob(s), dos(s), dbb(s), dst(s), dscr(s), dts(s);
  DevBuf dcf(s);
  dG.alloc(plan.mat_bytes * F);
  if (precision != GWC_PREC_FP64) dcf.alloc((size_t)F * 2 * rs.ldl * sizeof(float));
  dscr.alloc(fact == FACT_LU ? lu_scratch_bytes(F) : ldlt_scratch_bytes(F, N));
  dts.alloc((size_t)F * sizeof(float));
  dchr.alloc((size_t)F * rs.ldl * sizeof(double));
  dchi.alloc((size_t)F * rs.ldl * sizeof(double));
  const double2 *z_d = upload(dz, tl.z, s);
  const int *n_d = upload(dn, tl.n, s);
  const int *m_d = upload(dm, tl.m, s);
  const long long *ob_d = upload(dob, tl.out_base, s);
  const int *os_d = upload(dos, tl.out_stride, s);
  dbb.alloc((size_t)F * R * sizeof(double));
  dst.alloc(T * sizeof(int));

  std::vector<PendingTiming> pending;
  const bool timing = g_timing;
  for (size_t t0 = 0; t0 < T; t0 += F) {
    const int Fb = (int)std::min<size_t>(F, T - t0);
    launch_chi(rs.d_eps.as<double>(), rs.no, rs.nv, z_d + t0, Fb, rs.ldl, dchr.as<double>(),
               dchi.as<double>(), s);
    hipEvent_t ea = timing ? timing_mark(s) : nullptr;
    if (precision == GWC_PREC_FP64) {
      launch_pi_build_f64(rs.d_L.as<double>(), rs.ldl, N, dchr.as<double>(), dchi.as<double>(), Fb,
                          rs.d_tiles.as<int2>(), rs.n_tiles, dG.as<double2>(), (long long)mat_elems,
                          ldg, s);
    } else {
      launch_pi_build_mixed(precision, mx->Lf.p, mx->Bh.p, mx->Bl.p, rs.ldl, N,
                            dchr.as<double>(), dchi.as<double>(),
                            precision != GWC_PREC_BF16X3 ? mx->ics.as<float>() : nullptr,
                            mx->acol.as<float>(), dts.as<float>(), dcf.as<float>(), Fb, mx->tiles.as<int2>(),
                            mx->n_tiles, dG.as<double2>(), (long long)mat_elems, ldg, s);
    }
    if (timing) {
      double fl = 0.0;
      for (int t = 0; t < Fb; ++t) fl += (tl.z[t0 + t].x == 0.0 ? 1.0 : 2.0);
      fl *= (double)N * (N + 1) * (double)rs.no * rs.nv;
      pending.push_back({precision == GWC_PREC_FP64 ? 0 : 2, ea, timing_mark(s), fl});
    }
    launch_border(rs.d_Moo.as<double>(), rs.d_Mov.as<double>(), N, rs.no, rs.nv, n_d + t0, m_d + t0,
                  Fb, R, dG.as<double2>(), (long long)mat_elems, ldg, dbb.as<double>(), s);
    hipEvent_t eb = timing ? timing_mark(s) : nullptr;
    if (fact == FACT_LU) {
      HIPCHECK(launch_lu_bordered(dG.as<double2>(), (long long)mat_elems, ldg, N, R, Fb, dbb.as<double>(),
                                  ob_d + t0, os_d + t0, W_out, dst.as<int>() + t0, dscr.p, s));
    } else {
      HIPCHECK(launch_ldlt_bordered(dG.as<double2>(), (long long)mat_elems, ldg, N, R, Fb,
                                    dbb.as<double>(), ob_d + t0, os_d + t0, W_out, dst.as<int>() + t0,
                                    dscr.p, s));
    }
    if (timing) {
      // algorithmic flops: LU (8/3) N^3 + 8 N^2 R; LDL^T half the elimination
      // and one border side, (4/3) N^3 + 4 N^2 R
      const double nn = (double)N * N;
      const double fl = fact == FACT_LU ? Fb * ((8.0 / 3.0) * nn * N + 8.0 * nn * R)
                                        : Fb * ((4.0 / 3.0) * nn * N + 4.0 * nn * R);
      pending.push_back({fact == FACT_LU ? 1 : 5, eb, timing_mark(s), fl});
    }
    HIPCHECK(hipGetLastError());
  }
  std::vector<int> st(T);
  HIPCHECK(hipMemcpyAsync(st.data(), dst.p, T * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  timing_resolve(pending);
  if (fact == FACT_LDLT) {
    // a zero pivot of the unpivoted elimination (Im(1 - Pi) vanishing in
    // floating point): those matrices again with partial pivoting
    TaskList retry;
    std::vector<size_t> which;
    for (size_t t = 0; t < T; ++t)
      if (st[t]) {
        retry.z.push_back(tl.z[t]);
        retry.n.push_back(tl.n[t]);
        retry.m.push_back(tl.m[t]);
        retry.out_base.push_back(tl.out_base[t]);
        retry.out_stride.push_back(tl.out_stride[t]);
        which.push_back(t);
      }
    if (!which.empty()) {
      std::vector<int> st_lu;
      run_screening(rs, mx, precision, retry, R, W_out, st_lu, s, batch_bytes, FACT_LU);
      for (size_t k = 0; k < which.size(); ++k) st[which[k]] = st_lu[k];
    }
  }
  status_all.insert(status_all.end(), st.begin(), st.end());
}

struct SigmaInputs {
  std::vector<int> core;
  std::vector<double> wi, wwi, wr, vxc;
  std::vector<std::vector<int>> sym;  // per core: its equivalent set, ascending
  bool wac = false;
  gwc_wac_params wp{};
  bool qp = false;
  gwc_qp_params qpp{};
};

SigmaInputs check_sigma_args(int n_occ, int n_basis, const gwc_sigma_args *args,
                             const gwc_sigma_out *out, hipStream_t s) {
  if (!args) fail(GWC_ERR_INVALID_ARG, "NULL args");
  const int nc = args->n_core, ni = args->n_imag, nr = args->n_real;
  if (nc < 1 || ni < 1 || nr < 1) fail(GWC_ERR_SHAPE, "n_core, n_imag, n_real must be >= 1");
  if (!args->core_idx || !args->omega_imag || !args->w_imag || !args->omega_real)
    fail(GWC_ERR_INVALID_ARG, "NULL input array");
  if (args->mode != GWC_MODE_FULL && args->mode != GWC_MODE_DECOUPLED)
    fail(GWC_ERR_INVALID_ARG, "unknown mode %d", args->mode);
  if (args->precision < GWC_PREC_FP64 || args->precision > GWC_PREC_FP8)
    fail(GWC_ERR_INVALID_ARG, "unknown precision %d", args->precision);
  if (out && args->mode == GWC_MODE_FULL && !out->sigma_c)
    fail(GWC_ERR_INVALID_ARG, "sigma_c is required in FULL mode");
  SigmaInputs in;
  in.core = to_host(args->core_idx, nc, s);
  in.wi = to_host(args->omega_imag, ni, s);
  in.wwi = to_host(args->w_imag, ni, s);
  in.wr = to_host(args->omega_real, (size_t)nc * nr, s);
  in.vxc.assign(nc, 0.0);
  if (args->vxc) in.vxc = to_host(args->vxc, nc, s);
  if (!all_finite(in.wi) || !all_finite(in.wwi) || !all_finite(in.wr) || !all_finite(in.vxc) ||
      !std::isfinite(args->eta))
    fail(GWC_ERR_NONFINITE, "non-finite value in grids, eta or vxc");
  for (int c = 0; c < nc; ++c)
    if (in.core[c] < 0 || in.core[c] >= n_occ)
      fail(GWC_ERR_SHAPE, "core_idx[%d] = %d not in [0, n_occ)", c, in.core[c]);
  for (int k = 0; k < ni; ++k) {
    if (!(in.wi[k] > 0.0) || !(in.wwi[k] > 0.0)) fail(GWC_ERR_INVALID_ARG, "imaginary nodes and weights must be > 0");
    if (k > 0 && !(in.wi[k] > in.wi[k - 1])) fail(GWC_ERR_INVALID_ARG, "imaginary nodes must increase");
  }
  for (int c = 0; c < nc; ++c)
    for (int j = 1; j < nr; ++j)
      if (!(in.wr[(size_t)c * nr + j] > in.wr[(size_t)c * nr + j - 1]))
        fail(GWC_ERR_INVALID_ARG, "omega_real of core %d must increase", c);
  if (!(args->eta > 0.0)) fail(GWC_ERR_INVALID_ARG, "eta must be > 0");
  if (args->wac) {
    in.wac = true;
    in.wp = *args->wac;
    const gwc_wac_params &w = in.wp;
    if (!std::isfinite(w.core_min) || !std::isfinite(w.core_max) || !std::isfinite(w.delta_lower) ||
        !std::isfinite(w.delta_upper))
      fail(GWC_ERR_NONFINITE, "non-finite CD-WAC setting");
    if (w.n_core_pts < 2 || w.n_val_pts < 2) fail(GWC_ERR_SHAPE, "CD-WAC windows need >= 2 points each");
    if (ni + std::max(w.n_core_pts, w.n_val_pts) > WAC_MAX_NODES)
      fail(GWC_ERR_SHAPE, "n_imag + window points exceeds %d", WAC_MAX_NODES);
    if (!(w.core_min >= 0.0 && w.core_max > w.core_min))
      fail(GWC_ERR_INVALID_ARG, "CD-WAC core window must satisfy 0 <= core_min < core_max");
    if (!(w.delta_lower >= 0.0 && w.delta_lower < 1.0 && w.delta_upper >= 0.0))
      fail(GWC_ERR_INVALID_ARG, "CD-WAC margins must satisfy 0 <= delta_lower < 1, delta_upper >= 0");
  }
  if (args->qp) {
    in.qp = true;
    in.qpp = *args->qp;
    const gwc_qp_params &q = in.qpp;
    if (!std::isfinite(q.tol) || !std::isfinite(q.step)) fail(GWC_ERR_NONFINITE, "non-finite Newton setting");
    if (q.max_iter < 1 || !(q.tol > 0.0) || !(q.step > 0.0))
      fail(GWC_ERR_INVALID_ARG, "Newton settings need max_iter >= 1, tol > 0, step > 0");
    if (args->wac) fail(GWC_ERR_UNSUPPORTED, "the Newton quasiparticle solve runs with contour deformation only");
  }
  std::vector<int> labels;
  if (args->sym_group) labels = to_host(args->sym_group, n_basis, s);
  in.sym.resize(nc);
  for (int c = 0; c < nc; ++c) {
    const int n = in.core[c];
    if (labels.empty() || labels[n] < 0) {
      in.sym[c].push_back(n);
      continue;
    }
    for (int m = 0; m < n_basis; ++m)
      if (labels[m] == labels[n]) {
        if (m >= n_occ) fail(GWC_ERR_INVALID_ARG, "equivalent set of core %d holds unoccupied orbital %d", n, m);
        in.sym[c].push_back(m);
      }
  }
  return in;
}

// Residue tasks, ordered by (core, point, m); point n_real is w = eps_n.
// dec[t] marks the tasks of the equivalent set (the terms of Im Sigma^dec).
void build_residue_tasks(const ResidentSystem &rs, const gwc_sigma_args *args, const SigmaInputs &in,
                         TaskList &tr, std::vector<double> &ftask, std::vector<int> &cj_off,
                         std::vector<int> &dec) {
  const int nc = args->n_core, nr = args->n_real, npts = nr + 1;
  const bool full = args->mode == GWC_MODE_FULL;
  cj_off.assign((size_t)nc * npts + 1, 0);
  std::vector<char> in_set(rs.nb);
  for (int c = 0; c < nc; ++c) {
    const int nst = in.core[c];
    std::fill(in_set.begin(), in_set.end(), 0);
    for (int m : in.sym[c]) in_set[m] = 1;
    for (int j = 0; j < npts; ++j) {
      const double w = (j < nr) ? in.wr[(size_t)c * nr + j] : rs.eps[nst];
      const size_t cj = (size_t)c * npts + j;
      cj_off[cj] = (int)tr.size();
      for (int m = 0; m < rs.nb; ++m) {
        if (!full && j < nr && !in_set[m]) continue;
        const double f = prefactor(rs.eps[m], m < rs.no, w);
        if (f == 0.0) continue;
        dec.push_back(in_set[m]);
        tr.z.push_back(make_double2(std::fabs(rs.eps[m] - w), args->eta));
        tr.n.push_back(nst);
        tr.m.push_back(m);
        tr.out_base.push_back((long long)tr.size() - 1);
        tr.out_stride.push_back(0);
        ftask.push_back(f);
      }
    }
  }
  cj_off[(size_t)nc * npts] = (int)tr.size();
}

// Evenly spaced points on [a, b], rounded as numpy.linspace rounds them
// (j * step + a, the last point b itself).
std::vector<double> even_points(double a, double b, int n) {
  std::vector<double> y(n);
  const double step = (b - a) / (double)(n - 1);
  for (int j = 0; j < n; ++j) {
    const double t = (double)j * step;
    y[j] = t + a;
  }
  y[n - 1] = b;
  return y;
}

// CD-WAC: W at the reference points, one continued-fraction fit per pair
// (core c, orbital m) with residue terms, and W_real[t] of every residue task
// from its pair's fit (Eq. pade_approximation).
void run_wac(ResidentSystem &rs, const MixedOperands *mx, const gwc_sigma_args *args,
             const SigmaInputs &in, const TaskList &tr, const std::vector<int> &cj_off,
             const double2 *d_Wimag, double2 *d_Wreal, std::vector<int> &status, hipStream_t s,
             size_t batch_bytes) {
  const gwc_wac_params &wp = in.wp;
  const int nc = args->n_core, ni = args->n_imag, nb = rs.nb, npts = args->n_real + 1;
  const size_t T = tr.size();
  if (T == 0) return;
  const double INF = std::numeric_limits<double>::infinity();
  std::vector<double> xlo((size_t)nc * nb, INF), xhi((size_t)nc * nb, -INF);
  std::vector<int> task_core(T);
  int R_w = 0;
  for (int c = 0; c < nc; ++c)
    for (int t = cj_off[(size_t)c * npts]; t < cj_off[(size_t)(c + 1) * npts]; ++t) {
      const size_t k = (size_t)c * nb + tr.m[t];
      xlo[k] = std::min(xlo[k], tr.z[t].x);
      xhi[k] = std::max(xhi[k], tr.z[t].x);
      task_core[t] = c;
      R_w = std::max(R_w, tr.m[t] + 1);
    }
  const int NC = wp.n_core_pts, NV = wp.n_val_pts, n_rr = NC + NV;
  const std::vector<double> xc = even_points(wp.core_min, wp.core_max, NC);
  std::vector<std::vector<double>> xv(nc);
  std::vector<char> has_core(nc, 0), has_val(nc, 0);
  for (int c = 0; c < nc; ++c) {
    double lo = INF, hi = -INF;
    for (int m = 0; m < nb; ++m) {
      const size_t k = (size_t)c * nb + m;
      if (!(xhi[k] >= 0.0)) continue;  // no residue terms
      if (xhi[k] <= wp.core_max) {
        has_core[c] = 1;
      } else {
        has_val[c] = 1;
        lo = std::min(lo, xlo[k]);
        hi = std::max(hi, xhi[k]);
      }
    }
    if (has_val[c]) xv[c] = even_points((1.0 - wp.delta_lower) * lo, (1.0 + wp.delta_upper) * hi, NV);
  }
  // reference screening: W[c][m][j] for m < R_w, j < NC (core window) and
  // NC + j (valence window of core c)
  TaskList tl;
  for (int c = 0; c < nc; ++c) {
    const long long base = (long long)c * R_w * n_rr;
    if (has_core[c])
      for (int j = 0; j < NC; ++j) {
        tl.z.push_back(make_double2(xc[j], args->eta));
        tl.n.push_back(in.core[c]);
        tl.m.push_back(-1);
        tl.out_base.push_back(base + j);
        tl.out_stride.push_back(n_rr);
      }
    if (has_val[c])
      for (int j = 0; j < NV; ++j) {
        tl.z.push_back(make_double2(xv[c][j], args->eta));
        tl.n.push_back(in.core[c]);
        tl.m.push_back(-1);
        tl.out_base.push_back(base + NC + j);
        tl.out_stride.push_back(n_rr);
      }
  }
  DevBuf dWref(s);
  dWref.alloc((size_t)nc * R_w * n_rr * sizeof(double2));
  run_screening(rs, mx, args->precision, tl, R_w, dWref.as<double2>(), status, s, batch_bytes);

  // pairs and their nodes: imaginary nodes, then the window's real points
  std::vector<int4> pairs;
  std::vector<long long> noff;
  std::vector<double2> nz;
  std::vector<int> pidx((size_t)nc * nb, -1);
  for (int c = 0; c < nc; ++c)
    for (int m = 0; m < nb; ++m) {
      const size_t k = (size_t)c * nb + m;
      if (!(xhi[k] >= 0.0)) continue;
      const bool core = xhi[k] <= wp.core_max;
      const std::vector<double> &xs = core ? xc : xv[c];
      pidx[k] = (int)pairs.size();
      pairs.push_back(make_int4(c, m, core ? 0 : NC, ni + (int)xs.size()));
      noff.push_back((long long)nz.size());
      for (int q = 0; q < ni; ++q) nz.push_back(make_double2(0.0, in.wi[q]));
      for (double x : xs) nz.push_back(make_double2(x, args->eta));
    }
  std::vector<int> pot(T);
  for (size_t t = 0; t < T; ++t) pot[t] = pidx[(size_t)task_core[t] * nb + tr.m[t]];
  DevBuf dpairs(s), dnoff(s), dnz(s), dcoef(s), dpot(s), dzt(s), dst(s);
  const int4 *d_pairs = upload(dpairs, pairs, s);
  const long long *d_noff = upload(dnoff, noff, s);
  const double2 *d_nz = upload(dnz, nz, s);
  const int *d_pot = upload(dpot, pot, s);
  const double2 *d_zt = upload(dzt, tr.z, s);
  dcoef.alloc(nz.size() * sizeof(double2));
  const std::vector<int> zero(1, 0);
  int *d_st = upload(dst, zero, s);
  launch_pade_fit(d_pairs, (int)pairs.size(), d_noff, d_nz, d_Wimag, nb, ni, dWref.as<double2>(),
                  R_w, n_rr, dcoef.as<double2>(), d_st, s);
  launch_pade_eval(d_zt, d_pot, d_pairs, d_noff, d_nz, dcoef.as<double2>(), (int)T, d_Wreal, s);
  HIPCHECK(hipGetLastError());
  int flag = 0;
  HIPCHECK(hipMemcpyAsync(&flag, d_st, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (flag) fail(GWC_ERR_FACTORIZATION, "CD-WAC continued-fraction fit broke down (zero reciprocal difference)");
}

// Newton solution of the quasiparticle equation (Eq. quasiparticle_equation)
// for every core: per iteration Sigma^c at E - h, E, E + h by contour
// deformation on the cores still iterating, then the update on the host.
void run_qp_newton(ResidentSystem &rs, const MixedOperands *mx, const gwc_sigma_args *args,
                   const SigmaInputs &in, const double2 *d_Wimag, const double *d_wi,
                   const double *d_wwi, const std::vector<double> &sx, std::vector<double> &E,
                   std::vector<int> &iters, std::vector<int> &status, hipStream_t s,
                   size_t batch_bytes) {
  const gwc_qp_params &q = in.qpp;
  const int nc = args->n_core, ni = args->n_imag, nb = rs.nb;
  E.resize(nc);
  iters.assign(nc, -1);
  std::vector<char> active(nc, 1);
  for (int c = 0; c < nc; ++c) E[c] = rs.eps[in.core[c]];
  for (int it = 1; it <= q.max_iter; ++it) {
    std::vector<int> idx;
    for (int c = 0; c < nc; ++c)
      if (active[c]) idx.push_back(c);
    if (idx.empty()) break;
    const int na = (int)idx.size();
    SigmaInputs sub;
    sub.wi = in.wi;
    sub.wwi = in.wwi;
    std::vector<double> sxa(na);
    for (int k = 0; k < na; ++k) {
      const int c = idx[k];
      sub.core.push_back(in.core[c]);
      sub.vxc.push_back(in.vxc[c]);
      sub.sym.push_back({in.core[c]});
      sxa[k] = sx[c];
      sub.wr.push_back(E[c] - q.step);
      sub.wr.push_back(E[c]);
      sub.wr.push_back(E[c] + q.step);
    }
    gwc_sigma_args sa = *args;
    sa.n_core = na;
    sa.n_real = 3;
    sa.mode = GWC_MODE_FULL;
    TaskList tr;
    std::vector<double> ftask;
    std::vector<int> cj_off, tdec;
    build_residue_tasks(rs, &sa, sub, tr, ftask, cj_off, tdec);
    DevBuf dW(s), dWr(s), dcore(s), dwr(s), dsx(s), dvxc(s), dI(s), dft(s), dcjo(s), dtd(s);
    DevBuf dsig(s), dimd(s), dse(s), deq(s);
    dW.alloc((size_t)na * nb * ni * sizeof(double2));
    for (int k = 0; k < na; ++k)
      HIPCHECK(hipMemcpyAsync(dW.as<double2>() + (size_t)k * nb * ni, d_Wimag + (size_t)idx[k] * nb * ni,
                              (size_t)nb * ni * sizeof(double2), hipMemcpyDeviceToDevice, s));
    dWr.alloc(std::max<size_t>(tr.size(), 1) * sizeof(double2));
    run_screening(rs, mx, args->precision, tr, 1, dWr.as<double2>(), status, s, batch_bytes);
    for (int v : status)
      if (v) fail(GWC_ERR_FACTORIZATION, "exactly singular pivot in the LU of 1 - Pi(z)");
    const int *d_core = upload(dcore, sub.core, s);
    const double *d_wr = upload(dwr, sub.wr, s);
    const double *d_sx = upload(dsx, sxa, s);
    const double *d_vxc = upload(dvxc, sub.vxc, s);
    dI.alloc((size_t)na * 4 * sizeof(double));
    launch_quadrature(dW.as<double2>(), rs.d_eps.as<double>(), nb, d_wi, d_wwi, ni, d_wr, 3, d_core, na,
                      4, dI.as<double>(), s);
    const double *d_f = upload(dft, ftask, s);
    const int *d_cjo = upload(dcjo, cj_off, s);
    const int *d_td = upload(dtd, tdec, s);
    dsig.alloc((size_t)na * 3 * 2 * sizeof(double));
    dimd.alloc((size_t)na * 3 * sizeof(double));
    dse.alloc((size_t)na * 2 * sizeof(double));
    deq.alloc((size_t)na * sizeof(double));
    launch_assemble(dWr.as<double2>(), d_f, d_td, d_cjo, dI.as<double>(), na, 3, rs.d_eps.as<double>(),
                    d_core, d_sx, d_vxc, 1, dsig.as<double>(), dimd.as<double>(), dse.as<double>(),
                    deq.as<double>(), s);
    HIPCHECK(hipGetLastError());
    std::vector<double> sig((size_t)na * 6);
    HIPCHECK(hipMemcpyAsync(sig.data(), dsig.p, sig.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int k = 0; k < na; ++k) {
      const int c = idx[k];
      const double en = rs.eps[in.core[c]];
      const double Em = E[c] - q.step, Ep = E[c] + q.step;
      const double fm = Em - en - sx[c] - sig[(size_t)k * 6 + 0] + in.vxc[c];
      const double f0 = E[c] - en - sx[c] - sig[(size_t)k * 6 + 2] + in.vxc[c];
      const double fp = Ep - en - sx[c] - sig[(size_t)k * 6 + 4] + in.vxc[c];
      const double dE = -f0 / ((fp - fm) / (2.0 * q.step));
      E[c] = E[c] + dE;
      if (std::fabs(dE) < q.tol) {
        active[c] = 0;
        iters[c] = it;
      }
    }
  }
}

}  // namespace

void validate_sigma_args(int n_occ, int n_basis, const gwc_sigma_args *args,
                         const gwc_sigma_out *out, hipStream_t s) {
  (void)check_sigma_args(n_occ, n_basis, args, out, s);
}

size_t predict_sigma_bytes(const ResidentSystem &rs, const gwc_sigma_args *args, size_t batch_bytes) {
  if (batch_bytes == 0) batch_bytes = default_batch_bytes();
  const int nc = std::max(args->n_core, 1), nr = std::max(args->n_real, 1), ni = std::max(args->n_imag, 1);
  // residue task count bounded without reading the grids: every orbital at
  // every point (FULL), or the equivalent set (at most every occupied orbital)
  // per point plus every orbital at eps_n (DECOUPLED)
  const size_t per_point = args->sym_group ? (size_t)rs.no : 1;
  const size_t t_real = args->mode == GWC_MODE_FULL ? (size_t)nc * (nr + 1) * rs.nb
                                                    : (size_t)nc * ((size_t)nr * per_point + rs.nb);
  const BatchPlan pi = plan_batch(rs, (size_t)ni * nc, rs.nb, batch_bytes);
  BatchPlan pr = plan_batch(rs, t_real, 1, batch_bytes);
  if (args->wac) {
    const gwc_wac_params &w = *args->wac;
    const BatchPlan pw = plan_batch(rs, (size_t)nc * (std::max(w.n_core_pts, 0) + std::max(w.n_val_pts, 0)),
                                    rs.nb, batch_bytes);
    if (pw.bytes > pr.bytes) pr = pw;
  }
  const size_t fixed = (size_t)nc * rs.nb * ni * sizeof(double2) + t_real * (sizeof(double2) + sizeof(double)) +
                       (size_t)nc * (nr + 1) * 8 * sizeof(double) + (1 << 20);
  return std::max(pi.bytes, pr.bytes) + fixed;
}

void run_sigma(ResidentSystem &rs, const gwc_sigma_args *args, gwc_sigma_out *out, hipStream_t s,
               size_t batch_bytes) {
  if (!out) fail(GWC_ERR_INVALID_ARG, "NULL out");
  const SigmaInputs in = check_sigma_args(rs.no, rs.nb, args, out, s);
  if (batch_bytes == 0) batch_bytes = default_batch_bytes();
  const int N = rs.N, nb = rs.nb;
  const int nc = args->n_core, ni = args->n_imag, nr = args->n_real;
  const bool full = args->mode == GWC_MODE_FULL;
  const MixedOperands *mx = nullptr;
  if (args->precision != GWC_PREC_FP64) mx = &mixed_operands(rs, args->precision, s, nullptr);

  DevBuf dcore(s), dwi(s), dwwi(s), dwr(s), dvxc(s);
  const int *d_core = upload(dcore, in.core, s);
  const double *d_wi = upload(dwi, in.wi, s);
  const double *d_wwi = upload(dwwi, in.wwi, s);
  const double *d_wr = upload(dwr, in.wr, s);
  const double *d_vxc = upload(dvxc, in.vxc, s);
  std::vector<int> status;

  // ---- imaginary axis: W_imag[c][m][k]
  DevBuf dWi(s);
  dWi.alloc((size_t)nc * nb * ni * sizeof(double2));
  {
    TaskList tl;
    for (int k = 0; k < ni; ++k)
      for (int c = 0; c < nc; ++c) {
        tl.z.push_back(make_double2(0.0, in.wi[k]));
        tl.n.push_back(in.core[c]);
        tl.m.push_back(-1);
        tl.out_base.push_back((long long)c * nb * ni + k);
        tl.out_stride.push_back(ni);
      }
    run_screening(rs, mx, args->precision, tl, nb, dWi.as<double2>(), status, s, batch_bytes);
  }

  // ---- residues
  TaskList tr;
  std::vector<double> ftask;
  std::vector<int> cj_off, tdec;
  build_residue_tasks(rs, args, in, tr, ftask, cj_off, tdec);
  DevBuf dWr(s);
  dWr.alloc(std::max<size_t>(tr.size(), 1) * sizeof(double2));
  if (in.wac)
    run_wac(rs, mx, args, in, tr, cj_off, dWi.as<double2>(), dWr.as<double2>(), status, s, batch_bytes);
  else
    run_screening(rs, mx, args->precision, tr, 1, dWr.as<double2>(), status, s, batch_bytes);
  for (int v : status)
    if (v) fail(GWC_ERR_FACTORIZATION, "exactly singular pivot in the LU of 1 - Pi(z)");

  // ---- exchange, quadrature, assembly
  const int npts = nr + 1;
  DevBuf dsx(s), dI(s), dft(s), dcjo(s), dcjs(s), dsig(s), dimd(s), dse(s), deq(s);
  dsx.alloc(nc * sizeof(double));
  launch_sigma_x(rs.d_Moo.as<double>(), N, rs.no, d_core, nc, dsx.as<double>(), s);
  dI.alloc((size_t)nc * npts * sizeof(double));
  launch_quadrature(dWi.as<double2>(), rs.d_eps.as<double>(), nb, d_wi, d_wwi, ni, d_wr, nr, d_core,
                    nc, full ? npts : 1, dI.as<double>(), s);
  const double *d_f = upload(dft, ftask, s);
  const int *d_cjo = upload(dcjo, cj_off, s);
  const int *d_tdec = upload(dcjs, tdec, s);
  dsig.alloc((size_t)nc * nr * 2 * sizeof(double));
  dimd.alloc((size_t)nc * nr * sizeof(double));
  dse.alloc((size_t)nc * 2 * sizeof(double));
  deq.alloc((size_t)nc * sizeof(double));
  launch_assemble(dWr.as<double2>(), d_f, d_tdec, d_cjo, dI.as<double>(), nc, nr,
                  rs.d_eps.as<double>(), d_core, dsx.as<double>(), d_vxc, full ? 1 : 0,
                  dsig.as<double>(), dimd.as<double>(), dse.as<double>(), deq.as<double>(), s);
  HIPCHECK(hipGetLastError());
  if (full) copy_out(out->sigma_c, dsig.p, (size_t)nc * nr * 2 * sizeof(double), s);
  copy_out(out->im_sigma_dec, dimd.p, (size_t)nc * nr * sizeof(double), s);
  copy_out(out->sigma_c_eps, dse.p, (size_t)nc * 2 * sizeof(double), s);
  copy_out(out->sigma_x, dsx.p, (size_t)nc * sizeof(double), s);
  copy_out(out->e_qp, deq.p, (size_t)nc * sizeof(double), s);
  std::vector<double> e_newton;
  std::vector<int> qp_it;
  if (in.qp) {
    std::vector<double> sx(nc);
    HIPCHECK(hipMemcpyAsync(sx.data(), dsx.p, nc * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    run_qp_newton(rs, mx, args, in, dWi.as<double2>(), d_wi, d_wwi, sx, e_newton, qp_it, status, s,
                  batch_bytes);
    copy_out(out->e_qp_newton, e_newton.data(), (size_t)nc * sizeof(double), s);
    copy_out(out->qp_iterations, qp_it.data(), (size_t)nc * sizeof(int), s);
  }
  HIPCHECK(hipStreamSynchronize(s));
}

size_t predict_cumulant_bytes(int n_real, int n_t, int n_out) {
  return (size_t)n_real * 4 * sizeof(double) + 2 * (size_t)n_t * sizeof(double2) +
         (size_t)n_out * sizeof(double) + 4096;
}

void run_cumulant(const gwc_cumulant_args *a, double *A_out, double *z_out, hipStream_t s) {
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

  DevBuf dw(s), dim(s), dnu(s), dc(s), dz(s), dA(s), dB(s), dAout(s);
  const double *d_w = upload(dw, w, s);
  const double *d_im = upload(dim, im, s);
  dnu.alloc(a->n_real * sizeof(double));
  dc.alloc(a->n_real * sizeof(double));
  dz.alloc(2 * sizeof(double));
  dA.alloc((size_t)nt * sizeof(double2));
  dB.alloc((size_t)nt * sizeof(double2));
  dAout.alloc((size_t)a->n_out * sizeof(double));
  launch_cumulant_weights(d_w, d_im, a->n_real, a->eps_n, dnu.as<double>(), dc.as<double>(),
                          dz.as<double>(), s);
  launch_cumulant_time(dnu.as<double>(), dc.as<double>(), a->n_real, nt, dt, a->e_qp,
                       a->omega_out_min, a->eta, dA.as<double2>(), s);
  double2 *res = nullptr;
  launch_fft_inverse(dA.as<double2>(), dB.as<double2>(), log2n, &res, s);
  launch_extract_spectrum(res, a->n_out, dAout.as<double>(), s);
  HIPCHECK(hipGetLastError());
  copy_out(A_out, dAout.p, (size_t)a->n_out * sizeof(double), s);
  if (z_out) copy_out(z_out, dz.p, 2 * sizeof(double), s);
  HIPCHECK(hipStreamSynchronize(s));
}

// Fully analytic G0W0 (kernels_analytic.hip): Casida matrix, block-Jacobi
// eigensolver with the rotations carried into Y = Delta^1/2 L, transition
// moments, pole sums, E_QP and the spectral functions.
struct AnalyticInputs {
  std::vector<int> core;
  std::vector<double> wr, vxc;
};

// Host-side checks of gwc_sigma_analytic's arguments (no device work).
AnalyticInputs check_analytic_args(int n_occ, long long n_ov, const gwc_analytic_args *args,
                                   const gwc_analytic_out *out, hipStream_t s) {
  if (!args || !out) fail(GWC_ERR_INVALID_ARG, "NULL args or out");
  if (!out->sigma_c) fail(GWC_ERR_INVALID_ARG, "sigma_c is required");
  const int nc = args->n_core, nr = args->n_real;
  if (nc < 1 || nr < 1) fail(GWC_ERR_SHAPE, "n_core, n_real must be >= 1");
  if (!args->core_idx || !args->omega_real) fail(GWC_ERR_INVALID_ARG, "NULL input array");
  if (!std::isfinite(args->eta)) fail(GWC_ERR_NONFINITE, "non-finite eta");
  if (!(args->eta > 0.0)) fail(GWC_ERR_INVALID_ARG, "eta must be > 0");
  if (n_ov > 65536) fail(GWC_ERR_SHAPE, "n_occ * n_virt = %lld exceeds 65536", n_ov);
  AnalyticInputs in;
  in.core = to_host(args->core_idx, nc, s);
  in.wr = to_host(args->omega_real, (size_t)nc * nr, s);
  in.vxc.assign(nc, 0.0);
  if (args->vxc) in.vxc = to_host(args->vxc, nc, s);
  if (!all_finite(in.wr) || !all_finite(in.vxc)) fail(GWC_ERR_NONFINITE, "non-finite value in omega_real or vxc");
  for (int c = 0; c < nc; ++c) {
    if (in.core[c] < 0 || in.core[c] >= n_occ) fail(GWC_ERR_SHAPE, "core_idx[%d] = %d not in [0, n_occ)", c, in.core[c]);
    for (int j = 1; j < nr; ++j)
      if (!(in.wr[(size_t)c * nr + j] > in.wr[(size_t)c * nr + j - 1]))
        fail(GWC_ERR_INVALID_ARG, "omega_real of core %d must increase", c);
  }
  return in;
}

// RPA excitations of a resident system (Eqs. rpa_casida, rpa_matrices, symmetric
// form): the Casida matrix C is built and diagonalised by block Jacobi with
// the rotations carried into Y = Delta^1/2 L.  On return dY holds R = Y Z
// (n_aux x n_pad, row stride n_pad), dOm the excitation energies Omega in the
// rotated order (n_pad, 1 on the padding) and dsort (if non-NULL) the n_ov
// energies in ascending order.  Returns n_pad.
int rpa_solve(ResidentSystem &rs, hipStream_t s, DevBuf &dY, DevBuf &dOm, DevBuf *dsort, int &sweeps) {
  const int N = rs.N, no = rs.no, nv = rs.nv, n = rs.n_ov;
  const int JB2 = 2 * jacobi_block();
  const int n_pad = (int)round_up(n, JB2), nblk = n_pad / jacobi_block(), np = nblk / 2;
  const long long ld = n_pad;

  DevBuf dC(s), dVt(s), dVp(s), dact(s), drot(s);
  dC.alloc((size_t)n_pad * n_pad * sizeof(double));
  dVt.alloc((size_t)N * n_pad * sizeof(double));
  dY.alloc((size_t)N * n_pad * sizeof(double));
  dVp.alloc((size_t)np * JB2 * JB2 * sizeof(double));
  dact.alloc((size_t)np * sizeof(int));
  drot.alloc(3 * sizeof(int));  // rotations, C tiles and Y tiles updated in a sweep
  dOm.alloc((size_t)n_pad * sizeof(double));
  if (dsort) dsort->alloc((size_t)n * sizeof(double));
  double *C = dC.as<double>(), *Y = dY.as<double>();
  // transitions ordered by Delta, so that near-degenerate ones share Jacobi blocks
  std::vector<int> perm(n);
  std::vector<double> delta(n), diag2(n);
  for (int i = 0; i < no; ++i)
    for (int a = 0; a < nv; ++a) delta[(size_t)i * nv + a] = rs.eps[no + a] - rs.eps[i];
  for (int k = 0; k < n; ++k) perm[k] = k;
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return delta[x] < delta[y]; });
  for (int k = 0; k < n; ++k) diag2[k] = delta[perm[k]] * delta[perm[k]];
  DevBuf dperm(s), ddiag(s);
  const int *d_perm = upload(dperm, perm, s);
  const double *d_diag2 = upload(ddiag, diag2, s);
  // C = Vt^T Vt + diag(Delta^2) over the padded order (the padding stays zero)
  launch_casida_operands(rs.d_Mov.as<double>(), rs.d_eps.as<double>(), d_perm, N, no, nv, n_pad,
                         dVt.as<double>(), Y, s);
  launch_gemm_tn(dVt.as<double>(), ld, dVt.as<double>(), ld, n_pad, n_pad, N, C, ld, d_diag2, n, s);
  HIPCHECK(hipGetLastError());
  dVt.release();

  std::vector<PendingTiming> pending;
  const bool timing = g_timing;
  const double tol = 1e-14;
  // flops of one updated tile: C tiles two 64^3 products, Y tiles one
  const double fl_ctile = 4.0 * JB2 * JB2 * JB2, fl_ytile = 2.0 * JB2 * JB2 * JB2;
  const double fl_pairs = (double)np * (JB2 - 1) * 18.0 * jacobi_block() * JB2;
  sweeps = 0;
  int counts[3] = {1, 0, 0};
  constexpr int kMaxSweeps = 60;
  while (counts[0] != 0) {
    if (sweeps == kMaxSweeps) fail(GWC_ERR_FACTORIZATION, "block Jacobi not converged after %d sweeps", kMaxSweeps);
    launch_zero_counters(drot.as<int>(), 3, s);
    for (int r = 0; r < nblk - 1; ++r) {
      hipEvent_t ea = timing ? timing_mark(s) : nullptr;
      launch_jacobi_pairs(C, ld, nblk, r, tol, dVp.as<double>(), dact.as<int>(), drot.as<int>(), s);
      hipEvent_t eb = timing ? timing_mark(s) : nullptr;
      hipEvent_t ec = timing ? timing_mark(s) : nullptr;
      launch_jacobi_apply(C, ld, nblk, r, dVp.as<double>(), dact.as<int>(), Y, ld, N,
                          drot.as<int>() + 1, s);
      if (timing) {
        pending.push_back({4, ea, eb, fl_pairs});
        pending.push_back({3, ec, timing_mark(s), 0.0});
      }
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(counts, drot.p, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    ++sweeps;
    // the sweep's executed tile flops, booked on its last apply launch
    if (timing) pending.back().flops = counts[1] * fl_ctile + counts[2] * fl_ytile;
    timing_resolve(pending);
  }

  launch_excitations(C, ld, n, n_pad, dOm.as<double>(), dsort ? dsort->as<double>() : nullptr, s);
  {
    DevBuf dflag(s);
    dflag.alloc(sizeof(int));
    HIPCHECK(hipMemsetAsync(dflag.p, 0, sizeof(int), s));
    launch_nonfinite(dOm.as<double>(), n_pad, dflag.as<int>(), s);
    int flag = 0;
    HIPCHECK(hipMemcpyAsync(&flag, dflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (flag) fail(GWC_ERR_FACTORIZATION, "non-positive eigenvalue of the Casida matrix");
  }
  dC.release();
  return n_pad;
}

void run_analytic(ResidentSystem &rs, const gwc_analytic_args *args, gwc_analytic_out *out,
                  hipStream_t s) {
  const AnalyticInputs in = check_analytic_args(rs.no, rs.n_ov, args, out, s);
  const std::vector<int> &core = in.core;
  const std::vector<double> &wr = in.wr, &vxc = in.vxc;
  const int nc = args->n_core, nr = args->n_real;
  const int N = rs.N, no = rs.no, nv = rs.nv, nbas = rs.nb, n = rs.n_ov;

  DevBuf dcore(s), dwr(s), dvxc(s), dY(s), dOm(s), dsort(s);
  const int *d_core = upload(dcore, core, s);
  const double *d_wr = upload(dwr, wr, s);
  const double *d_vxc = upload(dvxc, vxc, s);
  int sweeps = 0;
  const long long ld = rpa_solve(rs, s, dY, dOm, &dsort, sweeps);
  const double *Y = dY.as<double>();

  // Q[c nb + m][nu] = sum_P M^P_{n_c m} R[P][nu], R = Y after the rotations
  DevBuf dBp(s), dQ(s), dpart(s), dsig(s), dsx(s), dsc(s), dse(s), deq(s), dagw(s), dadh(s);
  const int cols = nc * nbas, npts = nr + 1;
  dBp.alloc((size_t)N * cols * sizeof(double));
  dQ.alloc((size_t)cols * n * sizeof(double));
  launch_pack_pairs(rs.d_Moo.as<double>(), rs.d_Mov.as<double>(), N, no, nv, d_core, nc,
                    dBp.as<double>(), s);
  launch_gemm_tn(dBp.as<double>(), cols, Y, ld, cols, n, N, dQ.as<double>(), n, nullptr, 0, s);
  dpart.alloc((size_t)pole_sum_blocks(n) * nc * npts * sizeof(double2));
  dsig.alloc((size_t)nc * npts * sizeof(double2));
  launch_pole_sum(dQ.as<double>(), n, dOm.as<double>(), n, rs.d_eps.as<double>(), no, nbas, d_core,
                  nc, d_wr, nr, args->eta, 0, nullptr, dpart.as<double2>(), dsig.as<double2>(), s);
  dsx.alloc(nc * sizeof(double));
  launch_sigma_x(rs.d_Moo.as<double>(), N, no, d_core, nc, dsx.as<double>(), s);
  dsc.alloc((size_t)nc * nr * 2 * sizeof(double));
  dse.alloc((size_t)nc * 2 * sizeof(double));
  deq.alloc(nc * sizeof(double));
  dagw.alloc((size_t)nc * nr * sizeof(double));
  dadh.alloc((size_t)nc * nr * sizeof(double));
  launch_analytic_finish(dsig.as<double2>(), nc, nr, rs.d_eps.as<double>(), d_core, d_wr,
                         dsx.as<double>(), d_vxc, dsc.as<double>(), dse.as<double>(),
                         deq.as<double>(), dagw.as<double>(), dadh.as<double>(), s);
  HIPCHECK(hipGetLastError());
  copy_out(out->sigma_c, dsc.p, (size_t)nc * nr * 2 * sizeof(double), s);
  copy_out(out->sigma_c_eps, dse.p, (size_t)nc * 2 * sizeof(double), s);
  copy_out(out->sigma_x, dsx.p, (size_t)nc * sizeof(double), s);
  copy_out(out->e_qp, deq.p, (size_t)nc * sizeof(double), s);
  copy_out(out->a_gw, dagw.p, (size_t)nc * nr * sizeof(double), s);
  copy_out(out->a_dh, dadh.p, (size_t)nc * nr * sizeof(double), s);
  copy_out(out->omega_exc, dsort.p, (size_t)n * sizeof(double), s);
  if (out->sweeps) copy_out(out->sweeps, &sweeps, sizeof(int32_t), s);
  HIPCHECK(hipStreamSynchronize(s));
}

struct EvgwInputs {
  std::vector<int> core;
  std::vector<double> wr, vxc;
  gwc_evgw_params p{100, 1e-8, 200, 1e-10};
};

// Host-side checks of gwc_evgw0's arguments (no device work).
EvgwInputs check_evgw_args(int n_occ, int n_basis, long long n_ov, const gwc_evgw_args *args,
                           const gwc_evgw_out *out, hipStream_t s) {
  if (!args || !out) fail(GWC_ERR_INVALID_ARG, "NULL args or out");
  if (!out->e_qp) fail(GWC_ERR_INVALID_ARG, "e_qp is required");
  if (!args->M_vv) fail(GWC_ERR_INVALID_ARG, "M_vv is required");
  const int nc = args->n_core, nr = args->n_real;
  if (nc < 1 || nr < 1) fail(GWC_ERR_SHAPE, "n_core, n_real must be >= 1");
  if (!args->core_idx || !args->omega_real) fail(GWC_ERR_INVALID_ARG, "NULL input array");
  if (!std::isfinite(args->eta)) fail(GWC_ERR_NONFINITE, "non-finite eta");
  if (!(args->eta > 0.0)) fail(GWC_ERR_INVALID_ARG, "eta must be > 0");
  if (n_ov > 65536) fail(GWC_ERR_SHAPE, "n_occ * n_virt = %lld exceeds 65536", n_ov);
  EvgwInputs in;
  if (args->params) {
    in.p = *args->params;
    if (!std::isfinite(in.p.tol_outer) || !std::isfinite(in.p.tol_newton))
      fail(GWC_ERR_NONFINITE, "non-finite evGW0 tolerance");
    if (in.p.max_outer < 1 || in.p.max_newton < 1 || !(in.p.tol_outer > 0.0) || !(in.p.tol_newton > 0.0))
      fail(GWC_ERR_INVALID_ARG, "evGW0 settings need max_outer, max_newton >= 1 and tolerances > 0");
  }
  in.core = to_host(args->core_idx, nc, s);
  in.wr = to_host(args->omega_real, (size_t)nc * nr, s);
  in.vxc.assign(n_basis, 0.0);
  if (args->vxc) in.vxc = to_host(args->vxc, n_basis, s);
  if (!all_finite(in.wr) || !all_finite(in.vxc)) fail(GWC_ERR_NONFINITE, "non-finite value in omega_real or vxc");
  for (int c = 0; c < nc; ++c) {
    if (in.core[c] < 0 || in.core[c] >= n_occ) fail(GWC_ERR_SHAPE, "core_idx[%d] = %d not in [0, n_occ)", c, in.core[c]);
    for (int j = 1; j < nr; ++j)
      if (!(in.wr[(size_t)c * nr + j] > in.wr[(size_t)c * nr + j - 1]))
        fail(GWC_ERR_INVALID_ARG, "omega_real of core %d must increase", c);
  }
  return in;
}

// evGW0 (kernels_evgw.hip): the RPA once, rho^2 for every pair of states, then
// the outer iteration over all states' quasiparticle equations.
void run_evgw0(ResidentSystem &rs, const gwc_evgw_args *args, gwc_evgw_out *out, hipStream_t s) {
  const EvgwInputs in = check_evgw_args(rs.no, rs.nb, rs.n_ov, args, out, s);
  const int nc = args->n_core, nr = args->n_real;
  const int N = rs.N, no = rs.no, nv = rs.nv, nbas = rs.nb, n = rs.n_ov;

  DevBuf dvv(s), dcore(s), dwr(s), dvxc(s), dY(s), dOm(s);
  const size_t n_vv = (size_t)N * nv * nv;
  dvv.alloc(n_vv * sizeof(double));
  HIPCHECK(hipMemcpyAsync(dvv.p, args->M_vv, n_vv * sizeof(double), hipMemcpyDefault, s));
  {
    DevBuf dflag(s);
    dflag.alloc(sizeof(int));
    HIPCHECK(hipMemsetAsync(dflag.p, 0, sizeof(int), s));
    launch_nonfinite(dvv.as<double>(), (long long)n_vv, dflag.as<int>(), s);
    int flag = 0;
    HIPCHECK(hipMemcpyAsync(&flag, dflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (flag) fail(GWC_ERR_NONFINITE, "non-finite value in M_vv");
  }
  const int *d_core = upload(dcore, in.core, s);
  const double *d_wr = upload(dwr, in.wr, s);
  const double *d_vxc = upload(dvxc, in.vxc, s);
  int sweeps = 0;
  const long long ld = rpa_solve(rs, s, dY, dOm, nullptr, sweeps);

  // rho^2[(n nb + m)][nu] for every pair of states
  const long long rows = (long long)nbas * nbas;
  DevBuf dR2(s), dsx(s);
  {
    DevBuf dBp(s);
    dBp.alloc((size_t)N * rows * sizeof(double));
    dR2.alloc((size_t)rows * n * sizeof(double));
    launch_pack_all_pairs(rs.d_Moo.as<double>(), rs.d_Mov.as<double>(), dvv.as<double>(), N, no, nv,
                          dBp.as<double>(), s);
    launch_gemm_tn(dBp.as<double>(), rows, dY.as<double>(), ld, (int)rows, n, N, dR2.as<double>(), n,
                   nullptr, 0, s);
    launch_square_moments(dR2.as<double>(), rows, n, dOm.as<double>(), s);
    HIPCHECK(hipGetLastError());
  }
  dY.release();
  dvv.release();
  dsx.alloc((size_t)nbas * sizeof(double));
  launch_exchange_all(rs.d_Moo.as<double>(), rs.d_Mov.as<double>(), N, no, nv, dsx.as<double>(), s);

  // outer iteration on the energies in G
  DevBuf de(s), denew(s), dsteps(s);
  de.alloc((size_t)nbas * sizeof(double));
  denew.alloc((size_t)nbas * sizeof(double));
  dsteps.alloc((size_t)nbas * sizeof(int));
  HIPCHECK(hipMemcpyAsync(de.p, rs.d_eps.p, (size_t)nbas * sizeof(double), hipMemcpyDeviceToDevice, s));
  std::vector<double> e_host(rs.eps), e_new(nbas), e_first;
  int outer = -1;
  for (int k = 0; k < in.p.max_outer; ++k) {
    launch_ev_solve(dR2.as<double>(), n, dOm.as<double>(), rs.d_eps.as<double>(), de.as<double>(),
                    dsx.as<double>(), d_vxc, nbas, no, args->eta, in.p.tol_newton, in.p.max_newton,
                    denew.as<double>(), dsteps.as<int>(), s);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(e_new.data(), denew.p, (size_t)nbas * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(de.p, denew.p, (size_t)nbas * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));
    double delta = 0.0;
    for (int m = 0; m < nbas; ++m) delta = std::max(delta, std::fabs(e_new[m] - e_host[m]));
    if (!all_finite(e_new)) fail(GWC_ERR_NONFINITE, "non-finite quasiparticle energy in evGW0");
    e_host = e_new;
    if (k == 0) e_first = e_new;
    if (delta < in.p.tol_outer) {
      outer = k + 1;
      break;
    }
  }

  // Sigma^c,ev and A of the core states with the final energies in G
  const int npts = nr + 1;
  DevBuf dpart(s), dsig(s), dsc(s), daev(s);
  dpart.alloc((size_t)pole_sum_blocks(n) * nc * npts * sizeof(double2));
  dsig.alloc((size_t)nc * npts * sizeof(double2));
  launch_pole_sum(dR2.as<double>(), n, dOm.as<double>(), n, de.as<double>(), no, nbas, d_core, nc,
                  d_wr, nr, args->eta, 1, d_core, dpart.as<double2>(), dsig.as<double2>(), s);
  dsc.alloc((size_t)nc * nr * 2 * sizeof(double));
  daev.alloc((size_t)nc * nr * sizeof(double));
  launch_ev_finish(dsig.as<double2>(), nc, nr, rs.d_eps.as<double>(), d_core, d_wr, dsx.as<double>(),
                   d_vxc, dsc.as<double>(), daev.as<double>(), s);
  HIPCHECK(hipGetLastError());
  copy_out(out->e_qp, de.p, (size_t)nbas * sizeof(double), s);
  copy_out(out->e_first, e_first.data(), (size_t)nbas * sizeof(double), s);
  copy_out(out->sigma_x, dsx.p, (size_t)nbas * sizeof(double), s);
  copy_out(out->sigma_c, dsc.p, (size_t)nc * nr * 2 * sizeof(double), s);
  copy_out(out->a_ev, daev.p, (size_t)nc * nr * sizeof(double), s);
  copy_out(out->newton, dsteps.p, (size_t)nbas * sizeof(int32_t), s);
  if (out->outer) copy_out(out->outer, &outer, sizeof(int32_t), s);
  HIPCHECK(hipStreamSynchronize(s));
}

}  // namespace gwc

namespace {

template <class F>
int guarded(F &&fn) {
  std::string &err = gwc::last_error();
  err.clear();
  try {
    return fn();
  } catch (const GwcError &e) {
    err = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    err = "host allocation failed";
    return GWC_ERR_OUT_OF_MEMORY;
  } catch (const std::exception &e) {
    err = e.what();
    return GWC_ERR_DEVICE;
  } catch (...) {
    err = "unknown error";
    return GWC_ERR_DEVICE;
  }
}

}  // namespace

struct gwc_resident_system_s {
  gwc::ResidentSystem *rs;
};

gwc::ResidentSystem *gwc_handle_system(gwc_system_handle h) { return h ? h->rs : nullptr; }

extern "C" {

int gwc_sigma_core(const gwc_system *sys, const gwc_sigma_args *args, gwc_sigma_out *out,
                   void *hip_stream) {
  return guarded([&] {
    if (!sys || !args || !out) fail(GWC_ERR_INVALID_ARG, "NULL system, args or out");
    hipStream_t s = (hipStream_t)hip_stream;
    // argument checks that need no device come first
    gwc::validate_sigma_args(sys->n_occ, sys->n_occ + sys->n_virt, args, out, s);
    std::unique_ptr<gwc::ResidentSystem> rs(gwc::create_resident(sys, s));
    gwc::run_sigma(*rs, args, out, s, 0);
    return GWC_OK;
  });
}

int gwc_system_create(const gwc_system *sys, gwc_system_handle *handle) {
  return guarded([&] {
    if (!handle) fail(GWC_ERR_INVALID_ARG, "NULL handle");
    *handle = nullptr;
    gwc::ResidentSystem *rs = gwc::create_resident(sys, nullptr);
    *handle = new gwc_resident_system_s{rs};
    return GWC_OK;
  });
}

int gwc_system_destroy(gwc_system_handle handle) {
  return guarded([&] {
    if (!handle) fail(GWC_ERR_INVALID_ARG, "NULL handle");
    HIPCHECK(hipDeviceSynchronize());
    gwc::destroy_resident(handle->rs);
    delete handle;
    return GWC_OK;
  });
}

int gwc_sigma_core_resident(gwc_system_handle handle, const gwc_sigma_args *args,
                            gwc_sigma_out *out, void *hip_stream) {
  return guarded([&] {
    if (!handle || !args || !out) fail(GWC_ERR_INVALID_ARG, "NULL handle, args or out");
    gwc::run_sigma(*handle->rs, args, out, (hipStream_t)hip_stream, 0);
    return GWC_OK;
  });
}

int gwc_sigma_analytic(const gwc_system *sys, const gwc_analytic_args *args, gwc_analytic_out *out,
                       void *hip_stream) {
  return guarded([&] {
    if (!sys || !args || !out) fail(GWC_ERR_INVALID_ARG, "NULL system, args or out");
    hipStream_t s = (hipStream_t)hip_stream;
    // argument checks that need no device come first
    (void)gwc::check_analytic_args(sys->n_occ, (long long)sys->n_occ * sys->n_virt, args, out, s);
    std::unique_ptr<gwc::ResidentSystem> rs(gwc::create_resident(sys, s));
    gwc::run_analytic(*rs, args, out, s);
    return GWC_OK;
  });
}

int gwc_evgw0(const gwc_system *sys, const gwc_evgw_args *args, gwc_evgw_out *out,
              void *hip_stream) {
  return guarded([&] {
    if (!sys || !args || !out) fail(GWC_ERR_INVALID_ARG, "NULL system, args or out");
    hipStream_t s = (hipStream_t)hip_stream;
    (void)gwc::check_evgw_args(sys->n_occ, sys->n_occ + sys->n_virt,
                               (long long)sys->n_occ * sys->n_virt, args, out, s);
    std::unique_ptr<gwc::ResidentSystem> rs(gwc::create_resident(sys, s));
    gwc::run_evgw0(*rs, args, out, s);
    return GWC_OK;
  });
}

int gwc_spectral_cumulant(const gwc_cumulant_args *args, double *A_out, double *z_out,
                          void *hip_stream) {
  return guarded([&] {
    gwc::run_cumulant(args, A_out, z_out, (hipStream_t)hip_stream);
    return GWC_OK;
  });
}

int gwc_timing_enable(int on) {
  std::lock_guard<std::mutex> lock(g_timing_mutex);
  for (int k = 0; k < kNumTimed; ++k) g_stats[k] = TimerStat{};
  g_timing = on != 0;
  return GWC_OK;
}

int gwc_timing_get(const char *kernel, double *total_ms, long long *launches, double *flops) {
  std::lock_guard<std::mutex> lock(g_timing_mutex);
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

const char *gwc_last_error(void) { return gwc::last_error().c_str(); }

int gwc_probe_peak(int kind, double *value, void *hip_stream) {
  return guarded([&] {
    if (!value || kind < 0 || kind > 5) fail(GWC_ERR_INVALID_ARG, "gwc_probe_peak: kind must be 0..5 and value non-NULL");
    HIPCHECK(gwc::probe_peak(kind, (hipStream_t)hip_stream, value));
    return GWC_OK;
  });
}

int gwc_version(void) { return GWC_VERSION; }

}  // extern "C"
