// C ABI of the k-point AFQMC library: host-side validation, workspace sizing and dispatch.
// Every check runs before any HIP call, so argument errors are reported identically on a
// machine without a GPU.
#include <math.h>
#include <string.h>

#include <mutex>

#include "internal.h"

namespace afqmc {
size_t prepare_ws_bytes(const afqmc_kpt_problem& p);
size_t propagate_ws_bytes(const afqmc_kpt_problem& p);
size_t ortho_ws_bytes(const afqmc_kpt_problem& p);
size_t energy_ws_bytes(const afqmc_kpt_problem& p);
size_t backward_ws_bytes(const afqmc_kpt_problem& p);

size_t ws_bytes_entry(const afqmc_kpt_problem& p, int entry) {
  Dims d = dims_of(p);
  switch (entry) {
    case AFQMC_ENTRY_PREPARE: return prepare_ws_bytes(p);
    case AFQMC_ENTRY_GREENS: { Carve c(nullptr); GreensWs g; return carve_greens(c, d, g); }
    case AFQMC_ENTRY_VBIAS: { Carve c(nullptr); VbiasWs v; return carve_vbias(c, d, v); }
    case AFQMC_ENTRY_VHS: return align_up(16 * (size_t)d.W * d.nk * d.C);
    case AFQMC_ENTRY_PROPAGATE: {
      const size_t a = propagate_ws_bytes(p), b = ortho_ws_bytes(p);
      return a > b ? a : b;
    }
    case AFQMC_ENTRY_ORTHO: return ortho_ws_bytes(p);
    case AFQMC_ENTRY_ENERGY: return energy_ws_bytes(p);
    case AFQMC_ENTRY_ENERGY_BACKWARD: return backward_ws_bytes(p);
    default: return 0;
  }
}
}  // namespace afqmc

using namespace afqmc;

namespace {

enum Need : unsigned {
  N_L = 1u << 0, N_A = 1u << 1, N_LH = 1u << 2, N_H1H = 1u << 3, N_BHALF = 1u << 4,
  N_U = 1u << 5, N_GH = 1u << 6, N_LOGDET = 1u << 7, N_WEIGHT = 1u << 8, N_STATUS = 1u << 9,
  N_LD = 1u << 10, N_LHD = 1u << 11  // *D: the complex128 arrays in every precision
};

inline bool misaligned(const void* p, size_t a) { return ((uintptr_t)p) % a != 0; }

afqmc_status check_ptr(const void* p, size_t align) {
  if (!p) return AFQMC_ENULL;
  if (misaligned(p, align)) return AFQMC_EALIGN;
  return AFQMC_OK;
}

#define AFQMC_TRY(x)                      \
  do {                                    \
    afqmc_status st_ = (x);               \
    if (st_ != AFQMC_OK) return st_;      \
  } while (0)

afqmc_status check_dims(const afqmc_kpt_problem& p) {
  for (int i = 0; i < 3; ++i)
    if (p.mesh[i] < 1 || p.mesh[i] > 64) return AFQMC_EINVAL;
  if ((int64_t)p.mesh[0] * p.mesh[1] * p.mesh[2] != p.nk) return AFQMC_EINVAL;
  if (p.m < 1 || p.nocc < 1 || p.nocc > p.m || p.nchol < 1 || p.nwalk < 1) return AFQMC_EINVAL;
  if (p.prec != AFQMC_PREC_FP64 && p.prec != AFQMC_PREC_FP32) return AFQMC_EINVAL;
  if (!(p.dt > 0.0) || !isfinite(p.dt)) return AFQMC_EINVAL;
  // sizes the kernels implement
  if (p.m > 64 || p.nocc > 16) return AFQMC_EUNSUPPORTED;
  if ((int64_t)p.nk * p.nocc > 128) return AFQMC_EUNSUPPORTED;
  if ((int64_t)p.nk * p.nk * p.nk > (1 << 24)) return AFQMC_EUNSUPPORTED;
  // 32-bit row/column indices inside the GEMM tiles
  if ((int64_t)p.nk * p.m * p.m > 0x7fffffffLL || (int64_t)p.nk * p.m * p.nchol > 0x7fffffffLL)
    return AFQMC_EUNSUPPORTED;
  return AFQMC_OK;
}

afqmc_status check_fields(const afqmc_kpt_problem& p, unsigned need) {
  const bool f32 = (p.prec == AFQMC_PREC_FP32);
  if (need & N_L) AFQMC_TRY(check_ptr(f32 ? p.L32 : p.L, 16));
  if (need & N_A) AFQMC_TRY(check_ptr(p.A, 16));
  if (need & N_LH) AFQMC_TRY(check_ptr(f32 ? p.Lh32 : p.Lh, 16));
  if (need & N_LD) AFQMC_TRY(check_ptr(p.L, 16));
  if (need & N_LHD) AFQMC_TRY(check_ptr(p.Lh, 16));
  if (need & N_H1H) AFQMC_TRY(check_ptr(p.h1h, 16));
  if (need & N_BHALF) AFQMC_TRY(check_ptr(p.bhalf, 16));
  if (need & N_U) AFQMC_TRY(check_ptr(p.U, 16));
  if (need & N_GH) AFQMC_TRY(check_ptr(p.Gh, 16));
  if (need & N_LOGDET) AFQMC_TRY(check_ptr(p.logdet, 16));
  if (need & N_WEIGHT) AFQMC_TRY(check_ptr(p.weight, 8));
  if (need & N_STATUS) AFQMC_TRY(check_ptr(p.status, 4));
  return AFQMC_OK;
}

afqmc_status check_problems(const afqmc_kpt_problem* p, int nprob, unsigned need) {
  if (!p) return AFQMC_ENULL;
  if (nprob < 1) return AFQMC_EINVAL;
  for (int i = 0; i < nprob; ++i) {
    AFQMC_TRY(check_dims(p[i]));
    AFQMC_TRY(check_fields(p[i], need));
  }
  return AFQMC_OK;
}

afqmc_status check_ws(const afqmc_kpt_problem* p, int nprob, int entry, const void* ws,
                      size_t ws_bytes) {
  size_t need = 0;
  for (int i = 0; i < nprob; ++i) {
    const size_t b = ws_bytes_entry(p[i], entry);
    if (b > need) need = b;
  }
  if (need == 0) return AFQMC_OK;
  if (!ws || ws_bytes < need) return AFQMC_EWORKSPACE;
  if (misaligned(ws, 256)) return AFQMC_EALIGN;
  return AFQMC_OK;
}

// Device check, once per process: a gfx950 device must be current.
afqmc_status check_device() {
  static std::once_flag once;
  static afqmc_status st = AFQMC_ENODEV;
  std::call_once(once, [] {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) { st = AFQMC_ENODEV; return; }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { st = AFQMC_ENODEV; return; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) { st = AFQMC_ENODEV; return; }
    st = (strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? AFQMC_OK : AFQMC_ENODEV;
  });
  return st;
}

afqmc_status hip_status(hipError_t e) { return e == hipSuccess ? AFQMC_OK : AFQMC_EHIP; }

}  // namespace

extern "C" {

afqmc_status afqmc_kpt_workspace_bytes(const afqmc_kpt_problem* p, int nprob, int entry,
                                       size_t* bytes) {
  if (!bytes) return AFQMC_ENULL;
  if (!p) return AFQMC_ENULL;
  if (nprob < 1 || entry < AFQMC_ENTRY_PREPARE || entry > AFQMC_ENTRY_ENERGY_BACKWARD)
    return AFQMC_EINVAL;
  size_t need = 0;
  for (int i = 0; i < nprob; ++i) {
    AFQMC_TRY(check_dims(p[i]));
    const size_t b = ws_bytes_entry(p[i], entry);
    if (b > need) need = b;
  }
  *bytes = need;
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_prepare(const afqmc_kpt_problem* p, int nprob, const void* H1, void* ws,
                               size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, 0));
  for (int i = 0; i < nprob; ++i) {
    unsigned need = N_A | N_H1H | N_BHALF | N_LD | N_LHD;  // complex128 L and Lh always
    if (p[i].prec == AFQMC_PREC_FP32) need |= N_L | N_LH;  // plus the complex64 copies
    AFQMC_TRY(check_fields(p[i], need));
  }
  AFQMC_TRY(check_ptr(H1, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_PREPARE, ws, ws_bytes));
  AFQMC_TRY(check_device());
  for (int i = 0; i < nprob; ++i) AFQMC_TRY(hip_status(run_prepare(p[i], H1, ws, (hipStream_t)stream)));
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_greens(const afqmc_kpt_problem* p, int nprob, void* ws, size_t ws_bytes,
                              void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_A | N_U | N_GH | N_LOGDET | N_STATUS));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_GREENS, ws, ws_bytes));
  AFQMC_TRY(check_device());
  for (int i = 0; i < nprob; ++i) AFQMC_TRY(hip_status(run_greens(p[i], ws, false, (hipStream_t)stream)));
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_vbias(const afqmc_kpt_problem* p, int nprob, void* xbar, void* X, void* ws,
                             size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_LH | N_GH));
  AFQMC_TRY(check_ptr(xbar, 16));
  if (X) AFQMC_TRY(check_ptr(X, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_VBIAS, ws, ws_bytes));
  AFQMC_TRY(check_device());
  if (nprob > 1) return AFQMC_EUNSUPPORTED;  // per-problem output arrays are not expressible
  return hip_status(run_vbias(p[0], xbar, X, ws, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_vhs(const afqmc_kpt_problem* p, int nprob, const double* x,
                           const void* xbar, void* vhs, void* ws, size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_L));
  AFQMC_TRY(check_ptr(x, 8));
  AFQMC_TRY(check_ptr(xbar, 16));
  AFQMC_TRY(check_ptr(vhs, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_VHS, ws, ws_bytes));
  AFQMC_TRY(check_device());
  if (nprob > 1) return AFQMC_EUNSUPPORTED;
  return hip_status(run_vhs(p[0], x, xbar, vhs, ws, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_propagate(const afqmc_kpt_problem* p, int nprob, const void* vhs,
                                 const double* x, const void* xbar, int flags, void* ws,
                                 size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_A | N_BHALF | N_U | N_GH | N_LOGDET | N_WEIGHT | N_STATUS));
  AFQMC_TRY(check_ptr(vhs, 16));
  AFQMC_TRY(check_ptr(x, 8));
  AFQMC_TRY(check_ptr(xbar, 16));
  if (flags & ~AFQMC_PROPAGATE_ORTHO) return AFQMC_EINVAL;
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_PROPAGATE, ws, ws_bytes));
  AFQMC_TRY(check_device());
  if (nprob > 1) return AFQMC_EUNSUPPORTED;
  return hip_status(run_propagate(p[0], vhs, x, xbar, flags, ws, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_orthonormalize(const afqmc_kpt_problem* p, int nprob, void* ws,
                                      size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_A | N_U | N_GH | N_LOGDET | N_STATUS));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_ORTHO, ws, ws_bytes));
  AFQMC_TRY(check_device());
  for (int i = 0; i < nprob; ++i) AFQMC_TRY(hip_status(run_ortho(p[i], ws, (hipStream_t)stream)));
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_energy(const afqmc_kpt_problem* p, int nprob, void* E, void* ws,
                              size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_LH | N_H1H | N_GH));
  AFQMC_TRY(check_ptr(E, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_ENERGY, ws, ws_bytes));
  AFQMC_TRY(check_device());
  if (nprob > 1) return AFQMC_EUNSUPPORTED;
  return hip_status(run_energy(p[0], E, ws, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_energy_backward(const afqmc_kpt_problem* p, int nprob, const void* gE,
                                       void* gGh, void* ws, size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_LH | N_LHD | N_H1H | N_GH));
  if (gE) AFQMC_TRY(check_ptr(gE, 16));
  AFQMC_TRY(check_ptr(gGh, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_ENERGY_BACKWARD, ws, ws_bytes));
  AFQMC_TRY(check_device());
  if (nprob > 1) return AFQMC_EUNSUPPORTED;
  return hip_status(run_energy_backward(p[0], gE, gGh, ws, (hipStream_t)stream));
}

const char* afqmc_kpt_strerror(int status) {
  switch (status) {
    case AFQMC_OK: return "ok";
    case AFQMC_EINVAL: return "invalid dimension, time step or flag";
    case AFQMC_ENULL: return "required pointer is NULL";
    case AFQMC_EALIGN: return "pointer is not suitably aligned";
    case AFQMC_EWORKSPACE: return "workspace missing or too small";
    case AFQMC_ENODEV: return "no gfx950 device is current";
    case AFQMC_EHIP: return "HIP call or kernel launch failed";
    case AFQMC_EUNSUPPORTED: return "sizes outside what the kernels implement";
    default: return "unknown status";
  }
}

const char* afqmc_kpt_version(void) { return "afqmc_kpt 0.1 gfx950"; }

}  // extern "C"
