// C ABI of the k-point AFQMC library: host-side validation, workspace sizing and dispatch.
// Every check runs before any HIP call, so argument errors are reported identically on a
// machine without a GPU.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "internal.h"

namespace afqmc {
size_t prepare_ws_bytes(const afqmc_kpt_problem& p);
size_t propagate_ws_bytes(const afqmc_kpt_problem& p);
size_t ortho_ws_bytes(const afqmc_kpt_problem& p);
size_t energy_ws_bytes(const afqmc_kpt_problem& p);
size_t backward_ws_bytes(const afqmc_kpt_problem& p);
size_t population_ws_bytes(const afqmc_kpt_problem& p);
hipError_t run_population(const afqmc_kpt_problem* p, int nprob, const double* xi,
                          int32_t* const* parent, void* ws, hipStream_t s);
hipError_t run_update_etrial(const afqmc_kpt_problem* p, int nprob, const void* Emix,
                             double blend, hipStream_t s);
int reblock_host(const double* x, int64_t n, afqmc_reblock_level* levels, int max_levels,
                 int* optimal);
hipError_t run_dense_system(const afqmc_kpt_problem& p, const void* H1, void* Ld, void* H1d,
                            void* Ad, hipStream_t s);
hipError_t run_dense_fields(const afqmc_kpt_problem& p, const double* x, double* xd,
                            hipStream_t s);

size_t ws_bytes_entry(const afqmc_kpt_problem& p0, int entry) {
  // the step entry sizes each of its stages in that stage's precision
  const afqmc_kpt_problem p = stage_view(p0, energy_entry(entry));
  Dims d = dims_of(p);
  switch (entry) {
    case AFQMC_ENTRY_PREPARE: return prepare_ws_bytes(p);
    case AFQMC_ENTRY_GREENS: { Carve c(nullptr); GreensWs g; return carve_greens(c, d, g); }
    case AFQMC_ENTRY_VBIAS: { Carve c(nullptr); VbiasWs v; return carve_vbias(c, d, v); }
    case AFQMC_ENTRY_VHS: {  // the combined field, or its BF16 split planes
      const size_t cp = 32 * (size_t)((d.C + 31) / 32);
      const size_t a = 16 * (size_t)d.W * d.nk * d.C, b = 8 * (size_t)d.W * d.nk * cp;
      return align_up(a > b ? a : b);
    }
    case AFQMC_ENTRY_PROPAGATE: {
      const size_t a = propagate_ws_bytes(p), b = ortho_ws_bytes(p);
      return a > b ? a : b;
    }
    case AFQMC_ENTRY_ORTHO: return ortho_ws_bytes(p);
    case AFQMC_ENTRY_ENERGY: return energy_ws_bytes(p);
    case AFQMC_ENTRY_ENERGY_BACKWARD: return backward_ws_bytes(p);
    case AFQMC_ENTRY_POPULATION: return population_ws_bytes(p);
    case AFQMC_ENTRY_STEP: {
      size_t b = ws_bytes_entry(p0, AFQMC_ENTRY_VBIAS);
      const size_t e[3] = {ws_bytes_entry(p0, AFQMC_ENTRY_VHS), ws_bytes_entry(p0, AFQMC_ENTRY_PROPAGATE),
                           ws_bytes_entry(p0, AFQMC_ENTRY_ENERGY)};
      for (size_t v : e) b = v > b ? v : b;
      return b;
    }
    default: return 0;
  }
}
// Bytes of one problem's slice of a per-call buffer.
size_t buf_bytes(const afqmc_kpt_problem& p, int buf) {
  const size_t W = (size_t)p.nwalk, nk = (size_t)p.nk, C = (size_t)p.nchol;
  const size_t N = nk * p.m, n = nk * p.nocc;
  switch (buf) {
    case AFQMC_BUF_FIELDS: return 8 * W * nk * C * 2;
    case AFQMC_BUF_XBAR: return 16 * W * nk * C * 2;
    case AFQMC_BUF_X: return 16 * W * nk * C;
    case AFQMC_BUF_VHS: return (low_prec(step_prec(p.prec)) ? 8 : 16) * W * N * N;
    case AFQMC_BUF_ENERGY: return 16 * W * 3;
    case AFQMC_BUF_GE: return 16 * W;
    case AFQMC_BUF_GGH: return 16 * W * n * N;
    default: return 0;
  }
}

// offsets[i] (multiples of 256) and offsets[nprob] = end of the last slice.
void buf_offsets(const afqmc_kpt_problem* p, int nprob, int buf, size_t* off) {
  size_t o = 0;
  for (int i = 0; i < nprob; ++i) {
    off[i] = o;
    const size_t b = buf_bytes(p[i], buf);
    off[i + 1] = o + b;
    o = align_up(o + b);
  }
}

}  // namespace afqmc

using namespace afqmc;

namespace {

enum Need : unsigned {
  N_L = 1u << 0, N_A = 1u << 1, N_LH = 1u << 2, N_H1H = 1u << 3, N_BHALF = 1u << 4,
  N_U = 1u << 5, N_GH = 1u << 6, N_LOGDET = 1u << 7, N_WEIGHT = 1u << 8, N_STATUS = 1u << 9,
  N_LD = 1u << 10, N_LHD = 1u << 11,  // *D: the complex128 arrays in every precision
  N_LHS = 1u << 12, N_LS = 1u << 13,   // the BF16 split planes (BF16X3 problems only)
  N_ETRIAL = 1u << 14                  // the energy shift: optional, 8-byte aligned if set
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
  // an afqmc_prec value, or AFQMC_PREC_PLACE(step, energy)
  if ((p.prec & ~0x7f) != 0 || (p.prec & 15) > AFQMC_PREC_BF16X3 ||
      (p.prec >> 4) > AFQMC_PREC_INT8X4 + 1)
    return AFQMC_EINVAL;
  if (!(p.dt > 0.0) || !isfinite(p.dt)) return AFQMC_EINVAL;
  // sizes the kernels implement
  if (p.m > 64 || p.nocc > 16) return AFQMC_EUNSUPPORTED;
  if ((int64_t)p.nk * p.nocc > 256) return AFQMC_EUNSUPPORTED;
  if ((int64_t)p.nk * p.nk * p.nk > (1 << 24)) return AFQMC_EUNSUPPORTED;
  // 32-bit row/column indices inside the GEMM tiles
  if ((int64_t)p.nk * p.m * p.m > 0x7fffffffLL || (int64_t)p.nk * p.m * p.nchol > 0x7fffffffLL)
    return AFQMC_EUNSUPPORTED;
  return AFQMC_OK;
}

afqmc_status check_fields(const afqmc_kpt_problem& p, unsigned need) {
  const bool f32 = low_prec(p.prec);
  if ((need & N_L) && p.prec != AFQMC_PREC_BF16X3) AFQMC_TRY(check_ptr(f32 ? p.L32 : p.L, 16));
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
  if ((need & N_ETRIAL) && p.etrial && misaligned(p.etrial, 8)) return AFQMC_EALIGN;
  if ((need & N_LHS) && p.prec == AFQMC_PREC_BF16X3) AFQMC_TRY(check_ptr(p.Lhs, 16));
  if ((need & N_LS) && p.prec == AFQMC_PREC_BF16X3) AFQMC_TRY(check_ptr(p.Ls, 16));
  return AFQMC_OK;
}

// Two-determinant walkers: every up half directly followed by its down half, the two
// describing one system (sizes but nocc, precision, time step, the L pointer), with walker
// arrays of their own.
afqmc_status check_spins(const afqmc_kpt_problem* p, int nprob) {
  auto same = [](const void* a, const void* b) { return a && a == b; };
  for (int i = 0; i < nprob; ++i) {
    const int sp = p[i].spin;
    if (sp < AFQMC_SPIN_CLOSED || sp > AFQMC_SPIN_DOWN) return AFQMC_EINVAL;
    if (sp == AFQMC_SPIN_DOWN && (i == 0 || p[i - 1].spin != AFQMC_SPIN_UP)) return AFQMC_EINVAL;
    if (sp != AFQMC_SPIN_UP) continue;
    if (i + 1 >= nprob || p[i + 1].spin != AFQMC_SPIN_DOWN) return AFQMC_EINVAL;
    const afqmc_kpt_problem &a = p[i], &b = p[i + 1];
    for (int d = 0; d < 3; ++d)
      if (a.mesh[d] != b.mesh[d]) return AFQMC_EINVAL;
    if (a.m != b.m || a.nchol != b.nchol || a.nwalk != b.nwalk || a.prec != b.prec ||
        a.dt != b.dt || a.L != b.L)
      return AFQMC_EINVAL;
    if (same(a.U, b.U) || same(a.Gh, b.Gh) || same(a.logdet, b.logdet) ||
        same(a.weight, b.weight) || same(a.status, b.status) || same(a.Lh, b.Lh) ||
        same(a.h1h, b.h1h))
      return AFQMC_EINVAL;
  }
  return AFQMC_OK;
}

// need: the arrays the entry's stages read, checked in the precision of the step (energy =
// false) or of the local energy (energy = true).
afqmc_status check_problems(const afqmc_kpt_problem* p, int nprob, unsigned need,
                            bool energy = false) {
  if (!p) return AFQMC_ENULL;
  if (nprob < 1) return AFQMC_EINVAL;
  for (int i = 0; i < nprob; ++i) {
    AFQMC_TRY(check_dims(p[i]));
    AFQMC_TRY(check_fields(stage_view(p[i], energy), need));
  }
  return check_spins(p, nprob);
}

// The int8-split energies read the digits of Lh.
afqmc_status check_int8(const afqmc_kpt_problem* p, int nprob) {
  for (int i = 0; i < nprob; ++i)
    if (int8_digits(energy_prec(p[i].prec))) AFQMC_TRY(check_ptr(p[i].Lh8, 16));
  return AFQMC_OK;
}

// The re-orthonormalisation handles nk*nocc <= 256 (registers up to 128, L2 above).
afqmc_status check_ortho(const afqmc_kpt_problem* p, int nprob) {
  for (int i = 0; i < nprob; ++i)
    if ((int64_t)p[i].nk * p[i].nocc > 256) return AFQMC_EUNSUPPORTED;
  return AFQMC_OK;
}

afqmc_status check_ws(const afqmc_kpt_problem* p, int nprob, int entry, const void* ws,
                      size_t ws_bytes) {
  size_t need = 0;
  for (int i = 0; i < nprob; ++i) need += align_up(ws_bytes_entry(p[i], entry));
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

// Per-call buffer arguments of an entry (packed over the batch).
struct Bufs {
  const double* x = nullptr;
  void* xbar = nullptr;
  void* X = nullptr;
  void* vhs = nullptr;
  void* E = nullptr;
  const void* gE = nullptr;
  void* gGh = nullptr;
};

template <typename P>
P slice(P base, const afqmc_kpt_problem* p, int nprob, int buf, int i,
        std::vector<size_t>& off) {
  if (!base) return nullptr;
  off.resize(nprob + 1);
  buf_offsets(p, nprob, buf, off.data());
  return (P)((const char*)base + off[i]);
}

// Jobs of a batch: workspace regions and buffer slices.
std::vector<Job> make_jobs(const afqmc_kpt_problem* p, int nprob, int entry, void* ws,
                           const Bufs& b) {
  std::vector<Job> jobs(nprob);
  std::vector<size_t> off;
  size_t wo = 0;
  for (int i = 0; i < nprob; ++i) {
    Job& j = jobs[i];
    j.p = stage_view(p[i], energy_entry(entry));
    j.int8 = entry == AFQMC_ENTRY_ENERGY ? int8_digits(energy_prec(p[i].prec)) : 0;
    j.ws = ws ? (char*)ws + wo : nullptr;
    wo += align_up(ws_bytes_entry(p[i], entry));
    j.x = slice(b.x, p, nprob, AFQMC_BUF_FIELDS, i, off);
    j.xbar = slice(b.xbar, p, nprob, AFQMC_BUF_XBAR, i, off);
    j.X = slice(b.X, p, nprob, AFQMC_BUF_X, i, off);
    j.vhs = slice(b.vhs, p, nprob, AFQMC_BUF_VHS, i, off);
    j.E = slice(b.E, p, nprob, AFQMC_BUF_ENERGY, i, off);
    j.gE = slice(b.gE, p, nprob, AFQMC_BUF_GE, i, off);
    j.gGh = slice(b.gGh, p, nprob, AFQMC_BUF_GGH, i, off);
    // the down half of a two-determinant pair takes the up half's fields and cotangents
    if (p[i].spin == AFQMC_SPIN_DOWN) {
      j.x = jobs[i - 1].x;
      j.gE = jobs[i - 1].gE;
    }
  }
  return jobs;
}

// The step sequence; fields of step s at x + s * stride bytes.
hipError_t run_steps(std::vector<Job>& jobs, const int* orig_prec, const double* x,
                     size_t stride, int nsteps, int flags, hipStream_t s) {
  const int n = (int)jobs.size();
  std::vector<const double*> x0(n);
  for (int i = 0; i < n; ++i) x0[i] = jobs[i].x;
  // the halves of a two-determinant pair have one field and one force bias, hence one HS
  // potential: the down half propagates with the up half's
  std::vector<int> vh;
  for (int i = 0; i < n; ++i) {
    if (jobs[i].p.spin == AFQMC_SPIN_DOWN) jobs[i].vhs = jobs[i - 1].vhs;
    else vh.push_back(i);
  }
  std::vector<Job> vj(vh.size());
  hipError_t e = hipSuccess;
  for (int st = 0; st < nsteps && e == hipSuccess; ++st) {
    for (int i = 0; i < n; ++i)
      jobs[i].x = (const double*)((const char*)x0[i] + (size_t)st * stride);
    for (size_t q = 0; q < vh.size(); ++q) vj[q] = jobs[vh[q]];
    e = run_vbias(jobs.data(), n, s);
    if (e == hipSuccess) e = run_vhs(vj.data(), (int)vj.size(), s);
    // every Gh but that of a last step without re-orthonormalisation only feeds the next
    // force bias
    const bool last = st == nsteps - 1;
    const int pf = last ? (flags & AFQMC_PROPAGATE_ORTHO) : 0;
    const int rg = (!last || (flags & AFQMC_PROPAGATE_ORTHO)) ? AFQMC_PROPAGATE_REDUCED_GH : 0;
    if (e == hipSuccess) e = run_propagate(jobs.data(), n, pf | rg, s);
  }
  for (int i = 0; i < n; ++i) jobs[i].x = x0[i];
  if (e == hipSuccess && (flags & AFQMC_STEP_ENERGY)) {
    // the same workspace and buffers, with the problems in their energy precision
    std::vector<Job> ej(jobs);
    for (int i = 0; i < n; ++i) {
      const int ep = energy_prec(orig_prec[i]);
      ej[i].int8 = int8_digits(ep);
      ej[i].p.prec = ej[i].int8 ? AFQMC_PREC_FP64 : ep;
    }
    e = run_energy(ej.data(), n, s);
  }
  return e;
}

afqmc_status check_step_args(const afqmc_kpt_problem* p, int nprob, const double* x, int nsteps,
                             void* xbar, void* vhs, void* E, int flags, void* ws,
                             size_t ws_bytes) {
  // every step runs the force bias, whose BF16X3 kernel reads the split planes Lhs
  unsigned need = N_L | N_LS | N_LH | N_LHS | N_A | N_BHALF | N_U | N_GH | N_LOGDET | N_WEIGHT |
                  N_STATUS | N_ETRIAL;
  AFQMC_TRY(check_problems(p, nprob, need));
  if (flags & AFQMC_STEP_ENERGY) {
    AFQMC_TRY(check_problems(p, nprob, N_LH | N_LHS | N_H1H | N_GH, true));
    AFQMC_TRY(check_int8(p, nprob));
  }
  if (nsteps < 1) return AFQMC_EINVAL;
  if (flags & ~(AFQMC_PROPAGATE_ORTHO | AFQMC_STEP_ENERGY)) return AFQMC_EINVAL;
  if (flags & AFQMC_PROPAGATE_ORTHO) AFQMC_TRY(check_ortho(p, nprob));
  AFQMC_TRY(check_ptr(x, 8));
  AFQMC_TRY(check_ptr(xbar, 16));
  AFQMC_TRY(check_ptr(vhs, 16));
  if (flags & AFQMC_STEP_ENERGY) AFQMC_TRY(check_ptr(E, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_STEP, ws, ws_bytes));
  return AFQMC_OK;
}

}  // namespace

// Fixed scratch of the local energy for callers that cannot allocate: the Cholesky traces X,
// the split-K partials of the traces and the exchange partials of afqmc_kpt_energy live in
// this array instead of a caller workspace.  Each device holds its own copy (for the life
// of the process); host code uses only the per-device address from hipGetSymbolAddress,
// never the array's name.
static __device__ __align__(256) unsigned char scratch[AFQMC_ENERGY_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices];  // device address of scratch, per device; null until set up

// The current device's copy of scratch, resolved once per device with that device current.
afqmc_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return AFQMC_ENODEV;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return AFQMC_EHIP;
    scratch_dev[dev] = ptr;
  }
  *out = scratch_dev[dev];
  return AFQMC_OK;
}

}  // namespace

// Captured step block.
struct afqmc_kpt_graph_s {
  hipGraphExec_t exec;
};

extern "C" {

afqmc_status afqmc_kpt_workspace_bytes(const afqmc_kpt_problem* p, int nprob, int entry,
                                       size_t* bytes) {
  if (!bytes) return AFQMC_ENULL;
  if (!p) return AFQMC_ENULL;
  if (nprob < 1 || entry < AFQMC_ENTRY_PREPARE || entry > AFQMC_ENTRY_POPULATION)
    return AFQMC_EINVAL;
  size_t need = 0;
  for (int i = 0; i < nprob; ++i) {
    AFQMC_TRY(check_dims(p[i]));
    need += align_up(ws_bytes_entry(p[i], entry));
  }
  *bytes = need;
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_prepare(const afqmc_kpt_problem* p, int nprob, const void* H1, void* ws,
                               size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, 0));
  for (int i = 0; i < nprob; ++i) {
    // complex128 L and Lh always, plus the lower-precision copies each stage reads
    const unsigned need = N_A | N_H1H | N_BHALF | N_LD | N_LHD;
    AFQMC_TRY(check_fields(p[i], need));
    AFQMC_TRY(check_fields(stage_view(p[i], false), N_L | N_LH | N_LHS | N_LS));
    AFQMC_TRY(check_fields(stage_view(p[i], true), N_LH | N_LHS));
  }
  AFQMC_TRY(check_int8(p, nprob));
  AFQMC_TRY(check_ptr(H1, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_PREPARE, ws, ws_bytes));
  AFQMC_TRY(check_device());
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_PREPARE, ws, Bufs());
  for (int i = 0; i < nprob; ++i)
    AFQMC_TRY(hip_status(run_prepare(p[i], H1, jobs[i].ws, (hipStream_t)stream)));
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_greens(const afqmc_kpt_problem* p, int nprob, void* ws, size_t ws_bytes,
                              void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_A | N_U | N_GH | N_LOGDET | N_STATUS));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_GREENS, ws, ws_bytes));
  AFQMC_TRY(check_device());
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_GREENS, ws, Bufs());
  return hip_status(run_greens(jobs.data(), nprob, false, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_vbias(const afqmc_kpt_problem* p, int nprob, void* xbar, void* X, void* ws,
                             size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_LH | N_LHS | N_GH));
  AFQMC_TRY(check_ptr(xbar, 16));
  if (X) AFQMC_TRY(check_ptr(X, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_VBIAS, ws, ws_bytes));
  AFQMC_TRY(check_device());
  Bufs b;
  b.xbar = xbar;
  b.X = X;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_VBIAS, ws, b);
  return hip_status(run_vbias(jobs.data(), nprob, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_vhs(const afqmc_kpt_problem* p, int nprob, const double* x,
                           const void* xbar, void* vhs, void* ws, size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_L | N_LS));
  AFQMC_TRY(check_ptr(x, 8));
  AFQMC_TRY(check_ptr(xbar, 16));
  AFQMC_TRY(check_ptr(vhs, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_VHS, ws, ws_bytes));
  AFQMC_TRY(check_device());
  Bufs b;
  b.x = x;
  b.xbar = (void*)xbar;
  b.vhs = vhs;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_VHS, ws, b);
  return hip_status(run_vhs(jobs.data(), nprob, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_propagate(const afqmc_kpt_problem* p, int nprob, const void* vhs,
                                 const double* x, const void* xbar, int flags, void* ws,
                                 size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_A | N_BHALF | N_U | N_GH | N_LOGDET | N_WEIGHT | N_STATUS |
                                         N_ETRIAL));
  AFQMC_TRY(check_ptr(vhs, 16));
  AFQMC_TRY(check_ptr(x, 8));
  AFQMC_TRY(check_ptr(xbar, 16));
  if (flags & ~(AFQMC_PROPAGATE_ORTHO | AFQMC_PROPAGATE_REDUCED_GH)) return AFQMC_EINVAL;
  if (flags & AFQMC_PROPAGATE_ORTHO) AFQMC_TRY(check_ortho(p, nprob));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_PROPAGATE, ws, ws_bytes));
  AFQMC_TRY(check_device());
  Bufs b;
  b.x = x;
  b.xbar = (void*)xbar;
  b.vhs = (void*)vhs;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_PROPAGATE, ws, b);
  return hip_status(run_propagate(jobs.data(), nprob, flags, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_orthonormalize(const afqmc_kpt_problem* p, int nprob, void* ws,
                                      size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_A | N_U | N_GH | N_LOGDET | N_STATUS));
  AFQMC_TRY(check_ortho(p, nprob));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_ORTHO, ws, ws_bytes));
  AFQMC_TRY(check_device());
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_ORTHO, ws, Bufs());
  return hip_status(run_ortho(jobs.data(), nprob, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_energy(const afqmc_kpt_problem* p, int nprob, void* E, void* ws,
                              size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_LH | N_LHS | N_H1H | N_GH, true));
  AFQMC_TRY(check_int8(p, nprob));
  AFQMC_TRY(check_ptr(E, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_ENERGY, ws, ws_bytes));
  AFQMC_TRY(check_device());
  Bufs b;
  b.E = E;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_ENERGY, ws, b);
  return hip_status(run_energy(jobs.data(), nprob, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_energy_noalloc(const afqmc_kpt_problem* p, int nprob, void* E,
                                      void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_LH | N_LHS | N_H1H | N_GH, true));
  AFQMC_TRY(check_int8(p, nprob));
  AFQMC_TRY(check_ptr(E, 16));
  size_t need = 0;
  for (int i = 0; i < nprob; ++i) need += align_up(ws_bytes_entry(p[i], AFQMC_ENTRY_ENERGY));
  if (need > (size_t)AFQMC_ENERGY_NOALLOC_MAX_BYTES) return AFQMC_EWORKSPACE;
  AFQMC_TRY(check_device());
  void* ws = nullptr;
  AFQMC_TRY(scratch_address(&ws));
  Bufs b;
  b.E = E;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_ENERGY, ws, b);
  return hip_status(run_energy(jobs.data(), nprob, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_energy_backward(const afqmc_kpt_problem* p, int nprob, const void* gE,
                                       void* gGh, void* ws, size_t ws_bytes, void* stream) {
  // the Coulomb part of the adjoint needs X, whose BF16X3 trace reads Lhs
  AFQMC_TRY(check_problems(p, nprob, N_LH | N_LHD | N_LHS | N_H1H | N_GH, true));
  if (gE) AFQMC_TRY(check_ptr(gE, 16));
  AFQMC_TRY(check_ptr(gGh, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_ENERGY_BACKWARD, ws, ws_bytes));
  AFQMC_TRY(check_device());
  Bufs b;
  b.gE = gE;
  b.gGh = gGh;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_ENERGY_BACKWARD, ws, b);
  return hip_status(run_energy_backward(jobs.data(), nprob, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_mixed_energy(const afqmc_kpt_problem* p, int nprob, const void* E,
                                    void* Emix, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_WEIGHT));
  AFQMC_TRY(check_ptr(E, 16));
  AFQMC_TRY(check_ptr(Emix, 16));
  AFQMC_TRY(check_device());
  Bufs b;
  b.E = (void*)E;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_ENERGY, nullptr, b);
  return hip_status(run_mixed_energy(jobs.data(), nprob, Emix, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_population_control(const afqmc_kpt_problem* p, int nprob,
                                          const double* xi, int32_t* const* parent, void* ws,
                                          size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_U | N_GH | N_LOGDET | N_WEIGHT | N_STATUS));
  if (!xi) return AFQMC_ENULL;
  // the down half of a two-determinant pair draws with the up half's xi (equal weights and
  // equal xi give both halves the same copies)
  std::vector<double> xs(xi, xi + nprob);
  for (int i = 0; i < nprob; ++i) {
    if (p[i].spin == AFQMC_SPIN_DOWN) xs[i] = xs[i - 1];
    if (!(xs[i] >= 0.0 && xs[i] < 1.0)) return AFQMC_EINVAL;
    if (parent && parent[i] && misaligned(parent[i], 4)) return AFQMC_EALIGN;
  }
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_POPULATION, ws, ws_bytes));
  AFQMC_TRY(check_device());
  return hip_status(run_population(p, nprob, xs.data(), parent, ws, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_update_etrial(const afqmc_kpt_problem* p, int nprob, const void* Emix,
                                     double blend, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, 0));
  for (int i = 0; i < nprob; ++i) AFQMC_TRY(check_ptr(p[i].etrial, 8));
  AFQMC_TRY(check_ptr(Emix, 16));
  if (!(blend > 0.0 && blend <= 1.0)) return AFQMC_EINVAL;
  AFQMC_TRY(check_device());
  return hip_status(run_update_etrial(p, nprob, Emix, blend, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_reblock(const double* x, int64_t n, afqmc_reblock_level* levels,
                               int max_levels, int* nlevels, int* optimal) {
  if (!x || !nlevels || !optimal) return AFQMC_ENULL;
  if (n < 1 || max_levels < 0) return AFQMC_EINVAL;
  if (max_levels > 0 && !levels) return AFQMC_ENULL;
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(x[i])) return AFQMC_EINVAL;
  *nlevels = reblock_host(x, n, levels, max_levels, optimal);
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_dense_system(const afqmc_kpt_problem* p, int nprob, const void* H1,
                                    void* Ld, void* H1d, void* Ad, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_LD | N_A));
  if (nprob != 1) return AFQMC_EINVAL;
  // the dense problem (m = nk m, nocc = nk nocc on a 1x1x1 mesh) must be one the kernels run
  if ((int64_t)p[0].nk * p[0].m > 64 || (int64_t)p[0].nk * p[0].nocc > 16)
    return AFQMC_EUNSUPPORTED;
  AFQMC_TRY(check_ptr(H1, 16));
  AFQMC_TRY(check_ptr(Ld, 16));
  AFQMC_TRY(check_ptr(H1d, 16));
  AFQMC_TRY(check_ptr(Ad, 16));
  AFQMC_TRY(check_device());
  return hip_status(run_dense_system(p[0], H1, Ld, H1d, Ad, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_dense_fields(const afqmc_kpt_problem* p, int nprob, const double* x,
                                    double* xd, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, 0));
  if (nprob != 1) return AFQMC_EINVAL;
  AFQMC_TRY(check_ptr(x, 8));
  AFQMC_TRY(check_ptr(xd, 8));
  AFQMC_TRY(check_device());
  return hip_status(run_dense_fields(p[0], x, xd, (hipStream_t)stream));
}

}  // extern "C"

namespace {

// The padded problem and band counts of afqmc_kpt_pad_bands / afqmc_kpt_unpad_bands.
afqmc_status check_bands(const afqmc_kpt_problem* p, int nprob, const int32_t* mk) {
  if (!p || !mk) return AFQMC_ENULL;
  if (nprob != 1) return AFQMC_EINVAL;
  AFQMC_TRY(check_dims(p[0]));
  if (p[0].nk > AFQMC_PAD_MAX_NK) return AFQMC_EUNSUPPORTED;
  for (int k = 0; k < p[0].nk; ++k)
    if (mk[k] < p[0].nocc || mk[k] > p[0].m) return AFQMC_EINVAL;
  return AFQMC_OK;
}

// An input given requires its output.
afqmc_status check_pair_ptr(const void* in, const void* out) {
  if (!in) return AFQMC_OK;
  AFQMC_TRY(check_ptr(in, 16));
  return check_ptr(out, 16);
}

}  // namespace

extern "C" {

afqmc_status afqmc_kpt_pad_bands(const afqmc_kpt_problem* p, int nprob, const int32_t* mk,
                                 const void* L_r, const void* H1_r, const void* A_r,
                                 const void* U_r, void* L, void* H1, void* A, void* U,
                                 void* stream) {
  AFQMC_TRY(check_bands(p, nprob, mk));
  AFQMC_TRY(check_pair_ptr(L_r, L));
  AFQMC_TRY(check_pair_ptr(H1_r, H1));
  AFQMC_TRY(check_pair_ptr(A_r, A));
  AFQMC_TRY(check_pair_ptr(U_r, U));
  AFQMC_TRY(check_device());
  return hip_status(run_pad_bands(p[0], mk, L_r, H1_r, A_r, U_r, L, H1, A, U,
                                  (hipStream_t)stream));
}

afqmc_status afqmc_kpt_unpad_bands(const afqmc_kpt_problem* p, int nprob, const int32_t* mk,
                                   const void* U, const void* Gh, void* U_r, void* Gh_r,
                                   void* stream) {
  AFQMC_TRY(check_bands(p, nprob, mk));
  AFQMC_TRY(check_pair_ptr(U, U_r));
  AFQMC_TRY(check_pair_ptr(Gh, Gh_r));
  AFQMC_TRY(check_device());
  return hip_status(run_unpad_bands(p[0], mk, U, Gh, U_r, Gh_r, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_buffer_layout(const afqmc_kpt_problem* p, int nprob, int buf,
                                     size_t* offsets) {
  if (!p || !offsets) return AFQMC_ENULL;
  if (nprob < 1 || buf < AFQMC_BUF_FIELDS || buf > AFQMC_BUF_GGH) return AFQMC_EINVAL;
  for (int i = 0; i < nprob; ++i) AFQMC_TRY(check_dims(p[i]));
  buf_offsets(p, nprob, buf, offsets);
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_step(const afqmc_kpt_problem* p, int nprob, const double* x, int nsteps,
                            void* xbar, void* vhs, void* E, int flags, void* ws,
                            size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_step_args(p, nprob, x, nsteps, xbar, vhs, E, flags, ws, ws_bytes));
  AFQMC_TRY(check_device());
  Bufs b;
  b.x = x;
  b.xbar = xbar;
  b.vhs = vhs;
  b.E = E;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_STEP, ws, b);
  std::vector<size_t> off(nprob + 1);
  buf_offsets(p, nprob, AFQMC_BUF_FIELDS, off.data());
  std::vector<int> prec(nprob);
  for (int i = 0; i < nprob; ++i) prec[i] = p[i].prec;
  return hip_status(
      run_steps(jobs, prec.data(), x, off[nprob], nsteps, flags, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_autotune(const afqmc_kpt_problem* p, int nprob, void* vhs, void* ws,
                                size_t ws_bytes, void* stream) {
  AFQMC_TRY(check_problems(p, nprob, N_L | N_LS | N_LH | N_LHS | N_GH | N_U));
  AFQMC_TRY(check_ptr(vhs, 16));
  AFQMC_TRY(check_ws(p, nprob, AFQMC_ENTRY_STEP, ws, ws_bytes));
  AFQMC_TRY(check_device());
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  AFQMC_TRY(hip_status(hipStreamIsCapturing(s, &cs)));
  if (cs != hipStreamCaptureStatusNone) return AFQMC_EINVAL;
  Bufs b;
  b.vhs = vhs;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_STEP, ws, b);
  AFQMC_TRY(hip_status(tune_vbias(jobs.data(), nprob, s)));
  AFQMC_TRY(hip_status(tune_vhs(jobs.data(), nprob, s)));
  AFQMC_TRY(hip_status(tune_taylor(jobs.data(), nprob, s)));
  return hip_status(hipStreamSynchronize(s));
}

afqmc_status afqmc_kpt_graph_create(const afqmc_kpt_problem* p, int nprob, const double* x,
                                    int nsteps, void* xbar, void* vhs, void* E, int flags,
                                    void* ws, size_t ws_bytes, afqmc_kpt_graph* graph) {
  if (!graph) return AFQMC_ENULL;
  *graph = nullptr;
  AFQMC_TRY(check_step_args(p, nprob, x, nsteps, xbar, vhs, E, flags, ws, ws_bytes));
  AFQMC_TRY(check_device());
  Bufs b;
  b.x = x;
  b.xbar = xbar;
  b.vhs = vhs;
  b.E = E;
  std::vector<Job> jobs = make_jobs(p, nprob, AFQMC_ENTRY_STEP, ws, b);
  std::vector<size_t> off(nprob + 1);
  buf_offsets(p, nprob, AFQMC_BUF_FIELDS, off.data());
  std::vector<int> prec(nprob);
  for (int i = 0; i < nprob; ++i) prec[i] = p[i].prec;
  // record on a private stream (a capture cannot use the legacy default stream)
  hipStream_t cs;
  AFQMC_TRY(hip_status(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t er = run_steps(jobs, prec.data(), x, off[nprob], nsteps, flags, cs);
    e = hipStreamEndCapture(cs, &g);
    if (er != hipSuccess) e = er;
  }
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (exec) (void)hipGraphExecDestroy(exec);
    return AFQMC_EHIP;
  }
  *graph = new afqmc_kpt_graph_s{exec};
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_graph_launch(afqmc_kpt_graph graph, void* stream) {
  if (!graph) return AFQMC_ENULL;
  return hip_status(hipGraphLaunch(graph->exec, (hipStream_t)stream));
}

afqmc_status afqmc_kpt_graph_destroy(afqmc_kpt_graph graph) {
  if (!graph) return AFQMC_ENULL;
  const hipError_t e = hipGraphExecDestroy(graph->exec);
  delete graph;
  return hip_status(e);
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
