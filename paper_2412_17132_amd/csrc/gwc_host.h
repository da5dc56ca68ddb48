// Host-side internals shared by the C ABI entry points (gwc_api.hip) and the
// request server (gwc_server.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

#include "gwc.h"

namespace gwc {

struct GwcError {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const char *fmt, ...);

// A system whose RI coefficients, energies and packed L live on the device.
struct ResidentSystem;

// Validates `sys` and stages it on the current device (ordered on `s`).
ResidentSystem *create_resident(const gwc_system *sys, hipStream_t s);
void destroy_resident(ResidentSystem *rs);
int resident_n_occ(const ResidentSystem &rs);
int resident_n_basis(const ResidentSystem &rs);
double resident_eps(const ResidentSystem &rs, int m);

// The calling thread's message for gwc_last_error().
std::string &last_error();
size_t resident_bytes(const ResidentSystem &rs);

// Self-energy of the requested core states on a resident system.  Batched
// matrices of one launch use at most `batch_bytes` (0: min(48 GB, free / 2)).
void run_sigma(ResidentSystem &rs, const gwc_sigma_args *args, gwc_sigma_out *out, hipStream_t s,
               size_t batch_bytes);

// Host-side checks of the self-energy arguments (no device work).
void validate_sigma_args(int n_occ, int n_basis, const gwc_sigma_args *args,
                         const gwc_sigma_out *out, hipStream_t s);

// Upper bound of the device bytes run_sigma allocates for these arguments
// (besides the resident system), with the same batch budget.
size_t predict_sigma_bytes(const ResidentSystem &rs, const gwc_sigma_args *args,
                           size_t batch_bytes);

// Split operands of the mixed-precision Pi build (built on a resident
// system's first request at that precision and kept with the system):
// bytes they would take if not built yet (0 for FP64 or when built), and
// building them now, returning the bytes this call allocated (0 if they
// existed).
size_t mixed_operand_bytes(ResidentSystem &rs, int prec);
size_t prepare_mixed_operands(ResidentSystem &rs, int prec, hipStream_t s);

// Cumulant spectral function (all pointers host or device).
void run_cumulant(const gwc_cumulant_args *a, double *A_out, double *z_out, hipStream_t s);
size_t predict_cumulant_bytes(int n_real, int n_t, int n_out);

}  // namespace gwc
