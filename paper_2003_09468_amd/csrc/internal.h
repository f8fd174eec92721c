// Host-side internal interface of the k-point AFQMC library: workspace layout and the
// per-entry launch sequences (one problem at a time).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/afqmc_kpt.h"
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

// Number of K slices of the split-K force-bias contraction.
inline int vbias_splits(const Dims& d) {
  int s = 1;
  while (s * 2 <= d.nk && d.nk / (s * 2) >= 2 && s < 8) s *= 2;
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

size_t ws_bytes_entry(const afqmc_kpt_problem& p, int entry);

// Launch sequences (arguments already validated).
hipError_t run_prepare(const afqmc_kpt_problem& p, const void* H1, void* ws, hipStream_t s);
hipError_t run_greens(const afqmc_kpt_problem& p, void* ws, bool write_logdet_new_only,
                      hipStream_t s);
hipError_t run_vbias(const afqmc_kpt_problem& p, void* xbar, void* X, void* ws, hipStream_t s);
hipError_t run_vhs(const afqmc_kpt_problem& p, const double* x, const void* xbar, void* vhs,
                   void* ws, hipStream_t s);
hipError_t run_propagate(const afqmc_kpt_problem& p, const void* vhs, const double* x,
                         const void* xbar, int flags, void* ws, hipStream_t s);
hipError_t run_ortho(const afqmc_kpt_problem& p, void* ws, hipStream_t s);
hipError_t run_energy(const afqmc_kpt_problem& p, void* E, void* ws, hipStream_t s);
hipError_t run_energy_backward(const afqmc_kpt_problem& p, const void* gE, void* gGh, void* ws,
                               hipStream_t s);

// Kernels shared across translation units.
hipError_t launch_small_gj(const afqmc_kpt_problem& p, int mode, const void* S_in, void* out,
                           void* logdet_out, hipStream_t s);
hipError_t launch_greens_solve(const afqmc_kpt_problem& p, const void* oinvT, hipStream_t s);
hipError_t launch_cholesky_trace(const afqmc_kpt_problem& p, void* X, void* parts, hipStream_t s);

enum { GJ_MODE_GREENS = 0, GJ_MODE_CHOL_INV = 1 };

}  // namespace afqmc
