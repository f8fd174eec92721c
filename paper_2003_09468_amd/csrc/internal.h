// Host-side internal interface of the k-point AFQMC library: workspace layout, problem
// batches ("jobs") and the per-entry launch sequences.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/afqmc_kpt.h"
#include "batch.h"
#include "kcommon.h"
#include "timing.h"

namespace afqmc {

inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Dims {
  int64_t nk, m, nocc, C, W;
  int64_t N() const { return nk * m; }     // supercell orbitals
  int64_t n() const { return nk * nocc; }  // occupied orbitals per spin
};

inline Dims dims_of(const afqmc_kpt_problem& p) {
  return Dims{p.nk, p.m, p.nocc, p.nchol, p.nwalk};
}

// Number of K slices of the split-K force-bias contraction: at most 4, and at least two
// k-points per slice.
inline int vbias_splits(const Dims& d) {
  int s = 1;
  while (s * 2 <= d.nk && d.nk / (s * 2) >= 2 && s < 4) s *= 2;
  return s;
}

// Workspace carving: sequential 256-B aligned regions.
struct Carve {
  char* base;
  size_t off;
  explicit Carve(void* b) : base((char*)b), off(0) {}
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  }
};

// Regions used by several entries.
struct GreensWs { void* omat; void* oinvT; void* logdet_new; };
struct VbiasWs { void* parts; };

size_t carve_greens(Carve& c, const Dims& d, GreensWs& g);
size_t carve_vbias(Carve& c, const Dims& d, VbiasWs& v);

// Workspace of one problem for one entry (every entry's layout starts with the Green's
// function slots).  A placed precision sizes each stage in its own precision.
size_t ws_bytes_entry(const afqmc_kpt_problem& p, int entry);

// The half store of L's split planes (BF16X3 step): one slot per time-reversal pair, the Q
// whose index does not exceed that of -Q, in increasing Q.  -Q = Q exactly when every
// component of Q is 0 or half an even mesh dimension, so the slots number
// (nk + prod_d (1 + [mesh_d even])) / 2.
inline int ls_slots(const afqmc_kpt_problem& p) {
  int self = 1;
  for (int d = 0; d < 3; ++d) self *= (p.mesh[d] % 2 == 0) ? 2 : 1;
  return (p.nk + self) / 2;
}
// Bytes of the planes [slots][CP / 32][nk m m][4][32] (bf16); the int32 Q of each slot
// follows them.
inline size_t ls_plane_bytes(const afqmc_kpt_problem& p) {
  const size_t CP = 32 * (size_t)((p.nchol + 31) / 32);
  return (size_t)ls_slots(p) * CP * (size_t)p.nk * p.m * p.m * 4 * 2;
}

// The problem as a stage sees it: prec resolved to the energy precision for the local
// energy and its adjoint, to the step precision otherwise.
// The int8-split energies run as FP64 except for their exchange kernel (Job::int8).
inline afqmc_kpt_problem stage_view(const afqmc_kpt_problem& p, bool energy) {
  afqmc_kpt_problem q = p;
  q.prec = energy ? energy_prec(p.prec) : step_prec(p.prec);
  if (int8_digits(q.prec)) q.prec = AFQMC_PREC_FP64;
  return q;
}
inline bool energy_entry(int entry) {
  return entry == AFQMC_ENTRY_ENERGY || entry == AFQMC_ENTRY_ENERGY_BACKWARD;
}

// One problem of a batch with its workspace region and its slices of the packed per-call
// buffers (unused ones are null).
struct Job {
  afqmc_kpt_problem p;
  int int8;         // energy stage whose exchange runs on the int8 split: its digits per
                    // operand (4 or 5; p.prec is FP64), else 0
  void* ws;
  const double* x;  // fields of the current step [W][nk][C][2]
  void* xbar;       // [W][nk][C][2] complex128
  void* X;          // [W][nk][C] complex128
  void* vhs;        // [W][nk*m][nk*m] in the contraction precision
  void* E;          // [W][3] complex128
  const void* gE;   // [W] complex128
  void* gGh;        // like Gh
};

// Calls fn(ids, count) for groups of at most AFQMC_MAXP jobs with equal key(job index),
// in first-seen order; stops at the first error.
template <class KeyFn, class Fn>
hipError_t for_groups(int n, KeyFn key, Fn fn) {
  if (n <= 0) return hipSuccess;
  char done_small[64];
  char* done = n <= 64 ? done_small : new char[n];
  for (int i = 0; i < n; ++i) done[i] = 0;
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    if (done[i]) continue;
    const auto k = key(i);
    int ids[AFQMC_MAXP];
    int c = 0;
    for (int j = i; j < n && c < AFQMC_MAXP; ++j)
      if (!done[j] && key(j) == k) { ids[c++] = j; done[j] = 1; }
    e = fn(ids, c);
  }
  if (done != done_small) delete[] done;
  return e;
}

// Compute units of the current device (1 if the query fails).
inline int device_cus() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1;
  return ncu > 0 ? ncu : 1;
}

// Launch-group key of a problem in a batched GEMM stage: a problem whose own launch would
// give at least two workgroups per compute unit fills the device alone, and batching it
// with others only mixes tiles of different cost (and one tile shape for all), so it gets a
// key, and a launch, of its own; smaller problems share launches by their base key.
inline int solo_key(int base, int index, int64_t workgroups, int ncu) {
  return workgroups >= 2LL * ncu ? ((index + 1) << 12) | base : base;
}

// Launch sequences over a batch of jobs (arguments already validated).
hipError_t run_prepare(const afqmc_kpt_problem& p, const void* H1, void* ws, hipStream_t s);
hipError_t run_greens(const Job* jobs, int n, bool write_logdet_new_only, hipStream_t s,
                      bool reduced_gh = false);
hipError_t run_vbias(const Job* jobs, int n, hipStream_t s);
hipError_t run_vhs(const Job* jobs, int n, hipStream_t s);
hipError_t run_propagate(const Job* jobs, int n, int flags, hipStream_t s);
hipError_t run_ortho(const Job* jobs, int n, hipStream_t s);
hipError_t run_energy(const Job* jobs, int n, hipStream_t s);
hipError_t run_energy_backward(const Job* jobs, int n, hipStream_t s);
hipError_t run_mixed_energy(const Job* jobs, int n, void* Emix, hipStream_t s);

// Two-determinant walkers (AFQMC_SPIN_UP at job i, AFQMC_SPIN_DOWN at i + 1): the couplings
// between the halves' closed-shell stages.  run_spin_fields: xbar and X of each pair to the
// mean of the halves' (after the force bias); run_spin_energy: the pair's energy into both
// halves' rows from their closed-shell energies and traces X[job]; run_pair_mean: a = b =
// (a + b) / 2 over n[i] doubles; run_spin_adjoint_scale: gGh of every half times 1/2.
// Band padding (bands.hip): padded uniform arrays from packed ragged ones, and back.
hipError_t run_pad_bands(const afqmc_kpt_problem& p, const int32_t* mk, const void* Lr,
                         const void* H1r, const void* Ar, const void* Ur, void* L, void* H1,
                         void* A, void* U, hipStream_t s);
hipError_t run_unpad_bands(const afqmc_kpt_problem& p, const int32_t* mk, const void* U,
                           const void* Gh, void* Ur, void* Ghr, hipStream_t s);

bool has_pairs(const Job* jobs, int n);
hipError_t run_pair_mean(double* const* a, double* const* b, const int64_t* n, int cnt,
                         hipStream_t s);
hipError_t run_spin_fields(const Job* jobs, int n, hipStream_t s);
hipError_t run_spin_energy(const Job* jobs, int n, void* const* X, hipStream_t s);
hipError_t run_spin_adjoint_scale(const Job* jobs, int n, hipStream_t s);

// Kernels shared across translation units.  launch_cholesky_trace writes X (and xbar when
// requested) of every job; parts are the per-job split-K slices.
hipError_t launch_ortho_factor(const Job* jobs, int n, void* const* S, void* const* out,
                               hipStream_t s);
hipError_t launch_cholesky_trace(const Job* jobs, int n, void* const* X, void* const* xbar,
                                 void* const* parts, hipStream_t s);

// Autotuned tile shapes of the large contractions.  A stage's candidates are numbered
// from 0 (the built-in default); the cache maps (stage, precision, shapes of the batch) to
// the measured fastest candidate.
enum TuneStage { TS_TAYLOR = 0, TS_VHS = 1, TS_VBIAS = 2, TS_COUNT = 3 };
std::string tune_key(int stage, const Job* jobs, const int* ids, int c);
int tune_lookup(const std::string& key);
void tune_store(const std::string& key, int choice);
int tune_ncand(int stage, int prec);
// Times every candidate of a stage for one group (run(choice) launches it) and caches the
// fastest.  Synchronises the stream.
hipError_t tune_group(int stage, const Job* jobs, const int* ids, int c,
                      const std::function<hipError_t(int)>& run, hipStream_t s);
// Per-stage tuners over a batch, grouped exactly as the entries group their launches.
hipError_t tune_taylor(const Job* jobs, int n, hipStream_t s);
hipError_t tune_vhs(const Job* jobs, int n, hipStream_t s);
hipError_t tune_vbias(const Job* jobs, int n, hipStream_t s);

// One tile candidate of a stage for a group of jobs (the entries call these through the
// cache; the autotuner times them).
hipError_t launch_taylor_group(const Job* jobs, const int* ids, int c, int choice,
                               const void* const* tin, void* const* tout, void* const* acc,
                               double alpha_scale, hipStream_t s);
hipError_t launch_vhs_group(const Job* jobs, const int* ids, int c, int choice,
                            void* const* zeta, hipStream_t s);
hipError_t launch_vbias_group(const Job* jobs, const int* ids, int c, int choice,
                              void* const* parts, hipStream_t s);

// Workspace slots of the propagation used by the autotuner.
void propagate_slots(const Job& j, void** acc, void** t0, void** t1, void** tc);

}  // namespace afqmc
