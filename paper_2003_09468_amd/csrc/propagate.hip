// Walker propagation (symmetric propagator with the 6th-order Taylor expansion of the
// two-body exponential) and re-orthonormalisation.
//
//   T_0 = bhalf U,   T_j = (-sqrt(dt) / j) vhs T_{j-1},   U' = bhalf sum_j T_j.
//
// Each Taylor term is one batched MFMA GEMM per walker ((nk*m)^2 x nk*nocc) whose epilogue
// writes T_j and adds it into an FP64 accumulator; the one-body half steps are batched over
// (walker, k) blocks and always run in FP64.  With FP32 contractions the Taylor terms are
// computed from complex64 vhs and T_{j-1} with FP32 MFMA accumulation, while the walker
// accumulator stays complex128.
#include <math.h>

#include "cgemm.h"
#include "internal.h"

namespace afqmc {

hipError_t launch_weights(const Job* jobs, int n, hipStream_t s);

// out[w][(k p)][j] = sum_q bhalf[k][p][q] in[w][(k q)][j]; optionally also acc = out and a
// copy in the contraction precision T.
template <typename TO>
struct OpBhalf {
  typedef double T;
  static constexpr bool A_KCONTIG = true;
  static constexpr bool B_NCONTIG = true;
  int M, N, K, nbatch;  // M = K = m, N = nk*nocc, nbatch = W * nk
  const cpx<double>* B;   // [nk][m][m]
  const cpx<double>* in;  // [W][nk*m][N]
  cpx<double>* out;       // [W][nk*m][N] (may be null)
  cpx<TO>* outT;          // copy in the Taylor precision (may be null)
  int nk;
  __device__ void load_a(int b, int row, int k, double& re, double& im) const {
    const int kp = b % nk;
    const cpx<double> v = B[((int64_t)kp * M + row) * K + k];
    re = v.re; im = v.im;
  }
  __device__ void load_b(int b, int k, int col, double& re, double& im) const {
    const cpx<double> v = in[((int64_t)b * K + k) * N + col];
    re = v.re; im = v.im;
  }
  __device__ void store(int b, int row, int col, double re, double im) const {
    const int64_t idx = ((int64_t)b * M + row) * N + col;
    if (out) out[idx] = cpx<double>{re, im};
    if (outT) outT[idx] = cpx<TO>{(TO)re, (TO)im};
  }
};

// T_j = alpha vhs T_{j-1}; acc += T_j
template <typename TT>
struct OpTaylor {
  typedef TT T;
  static constexpr bool A_KCONTIG = true;
  static constexpr bool B_NCONTIG = true;
  int M, N, K, nbatch;  // M = K = nk*m, N = nk*nocc, nbatch = W
  T alpha;
  const cpx<T>* V;     // [W][M][M]
  const cpx<T>* Tin;   // [W][M][N]
  cpx<T>* Tout;        // [W][M][N] (null for the last term)
  cpx<double>* acc;    // [W][M][N]
  __device__ void load_a(int b, int row, int k, T& re, T& im) const {
    const cpx<T> v = V[((int64_t)b * M + row) * K + k];
    re = v.re; im = v.im;
  }
  __device__ void load_b(int b, int k, int col, T& re, T& im) const {
    const cpx<T> v = Tin[((int64_t)b * K + k) * N + col];
    re = v.re; im = v.im;
  }
  __device__ void store(int b, int row, int col, T re, T im) const {
    const int64_t idx = ((int64_t)b * M + row) * N + col;
    const T r = alpha * re, i = alpha * im;
    if (Tout) Tout[idx] = cpx<T>{r, i};
    cpx<double> a = acc[idx];
    a.re += (double)r;
    a.im += (double)i;
    acc[idx] = a;
  }
};

// One-body half step of every job of a group; in/out/outT give each job's operands.
template <typename TO>
static hipError_t launch_bhalf(const Job* jobs, const int* ids, int c, void* const* in,
                               void* const* out, void* const* outT, hipStream_t s) {
  OpBhalf<TO> ops[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) {
    const afqmc_kpt_problem& p = jobs[ids[q]].p;
    OpBhalf<TO>& op = ops[q];
    op.M = p.m; op.K = p.m; op.N = p.nk * p.nocc;
    op.nbatch = p.nwalk * p.nk;
    op.nk = p.nk;
    op.B = (const cpx<double>*)p.bhalf;
    op.in = (const cpx<double>*)in[ids[q]];
    op.out = out ? (cpx<double>*)out[ids[q]] : nullptr;
    op.outT = outT ? (cpx<TO>*)outT[ids[q]] : nullptr;
  }
  TimedScope ts(KC_BHALF, s);
  int mmax = 0;
  for (int q = 0; q < c; ++q) mmax = jobs[ids[q]].p.m > mmax ? jobs[ids[q]].p.m : mmax;
  if (mmax <= 16) return launch_ops<16, 64, 16, 1, 4>(ops, c, s);
  return launch_ops<32, 64, 16, 2, 2>(ops, c, s);
}

// Taylor tile class of an FP32 problem: one column tile spans all nk*nocc columns
// (rounded up to 16), each of the 4 waves owning 16 rows x BN columns.
static int taylor_class(const afqmc_kpt_problem& p) {
  if (!low_prec(p.prec)) return 0;
  const int c = (p.nk * p.nocc + 15) / 16;
  return c <= 8 ? c : 9;
}

template <typename T>
static hipError_t taylor_tiles(const OpTaylor<T>* ops, int c, int cls, int choice,
                               hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    // 64 x 32 tiles: measured fastest for the 16x16x4 FP64 MFMA at 702 x 108 x 702
    switch (choice) {
      case 1: return launch_ops<64, 64, 16, 2, 2>(ops, c, s);
      case 2: return launch_ops<32, 64, 16, 2, 2>(ops, c, s);
      case 3: return launch_ops<32, 32, 16, 2, 2>(ops, c, s);
      // one column tile over nk*nocc <= 112 (less zero padding than 32-column tiles):
      // seven waves side by side, each 64 (or 2 x 64) rows x 16 columns
      case 4: return launch_ops<64, 112, 16, 1, 7>(ops, c, s);
      case 5: return launch_ops<128, 112, 16, 2, 7>(ops, c, s);
      default: return launch_ops<64, 32, 16, 4, 1>(ops, c, s);
    }
  } else {
    if (choice == 1) return launch_ops<64, 64, 16, 2, 2>(ops, c, s);
    if (choice == 2) return launch_ops<64, 32, 16, 4, 1>(ops, c, s);
    switch (cls) {
      case 1: return launch_ops<64, 16, 16, 4, 1>(ops, c, s);
      case 2: return launch_ops<64, 32, 16, 4, 1>(ops, c, s);
      case 3: return launch_ops<64, 48, 16, 4, 1>(ops, c, s);
      case 4: return launch_ops<64, 64, 16, 4, 1>(ops, c, s);
      case 5: return launch_ops<64, 80, 16, 4, 1>(ops, c, s);
      case 6: return launch_ops<64, 96, 16, 4, 1>(ops, c, s);
      case 7: return launch_ops<64, 112, 16, 4, 1>(ops, c, s);
      case 8: return launch_ops<64, 128, 16, 4, 1>(ops, c, s);
      default: return launch_ops<64, 64, 16, 2, 2>(ops, c, s);
    }
  }
}

// One Taylor term, T_j = alpha vhs T_{j-1}, acc += T_j, for a group of jobs of one
// precision and tile class; alpha = -sqrt(dt) * alpha_scale per job.
hipError_t launch_taylor_group(const Job* jobs, const int* ids, int c, int choice,
                               const void* const* tin, void* const* tout, void* const* acc,
                               double alpha_scale, hipStream_t s) {
  TimedScope ts(KC_TAYLOR, s);
  const int cls = taylor_class(jobs[ids[0]].p);
  if (low_prec(jobs[ids[0]].p.prec)) {
    OpTaylor<float> ops[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const Job& j = jobs[ids[q]];
      OpTaylor<float>& op = ops[q];
      op.M = j.p.nk * j.p.m; op.K = op.M; op.N = j.p.nk * j.p.nocc;
      op.nbatch = j.p.nwalk;
      op.alpha = (float)(-sqrt(j.p.dt) * alpha_scale);
      op.V = (const cpx<float>*)j.vhs;
      op.Tin = (const cpx<float>*)tin[ids[q]];
      op.Tout = tout ? (cpx<float>*)tout[ids[q]] : nullptr;
      op.acc = (cpx<double>*)acc[ids[q]];
    }
    return taylor_tiles<float>(ops, c, cls, choice, s);
  }
  OpTaylor<double> ops[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) {
    const Job& j = jobs[ids[q]];
    OpTaylor<double>& op = ops[q];
    op.M = j.p.nk * j.p.m; op.K = op.M; op.N = j.p.nk * j.p.nocc;
    op.nbatch = j.p.nwalk;
    op.alpha = -sqrt(j.p.dt) * alpha_scale;
    op.V = (const cpx<double>*)j.vhs;
    op.Tin = (const cpx<double>*)tin[ids[q]];
    op.Tout = tout ? (cpx<double>*)tout[ids[q]] : nullptr;
    op.acc = (cpx<double>*)acc[ids[q]];
  }
  return taylor_tiles<double>(ops, c, cls, choice, s);
}

// Layout: the Green's-function slots come first in every entry's workspace, so that
// run_greens (which carves from the start) and the weight update agree on them.
static size_t carve_propagate(Carve& c, const afqmc_kpt_problem& p, void** acc, void** t0,
                              void** t1, GreensWs& g) {
  Dims d = dims_of(p);
  const size_t tsz = low_prec(p.prec) ? 8 : 16;
  carve_greens(c, d, g);
  *acc = c.take(16 * (size_t)d.W * d.N() * d.n());
  *t0 = c.take(tsz * (size_t)d.W * d.N() * d.n());
  *t1 = c.take(tsz * (size_t)d.W * d.N() * d.n());
  return c.off;
}

size_t propagate_ws_bytes(const afqmc_kpt_problem& p) {
  Carve c(nullptr);
  void *a, *b, *t;
  GreensWs g;
  return carve_propagate(c, p, &a, &b, &t, g);
}

void propagate_slots(const Job& j, void** acc, void** t0, void** t1) {
  Carve c(j.ws);
  GreensWs g;
  carve_propagate(c, j.p, acc, t0, t1, g);
}

static int taylor_key(const afqmc_kpt_problem& p) { return p.prec * 16 + taylor_class(p); }

// U <- bhalf T6(-sqrt(dt) vhs) bhalf U for every job.
static hipError_t propagate_jobs(const Job* J, int c, hipStream_t s) {
  void *acc[AFQMC_MAXP], *t0[AFQMC_MAXP], *t1[AFQMC_MAXP], *U[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) {
    propagate_slots(J[q], &acc[q], &t0[q], &t1[q]);
    U[q] = J[q].p.U;
  }
  return for_groups(
      c, [&](int i) { return taylor_key(J[i].p); },
      [&](const int* ids, int g) -> hipError_t {
        const bool f32 = low_prec(J[ids[0]].p.prec);
        // T_0 = bhalf U (FP64), acc = T_0, t0 = T_0 in the Taylor precision
        hipError_t e = f32 ? launch_bhalf<float>(J, ids, g, U, acc, t0, s)
                           : launch_bhalf<double>(J, ids, g, U, acc, t0, s);
        if (e != hipSuccess) return e;
        const int choice = tune_lookup(tune_key(TS_TAYLOR, J, ids, g));
        void** tin = t0;
        void** tout = t1;
        for (int j = 1; j <= 6; ++j) {
          e = launch_taylor_group(J, ids, g, choice, tin, (j < 6) ? tout : nullptr, acc,
                                  1.0 / j, s);
          if (e != hipSuccess) return e;
          void** t = tin; tin = tout; tout = t;
        }
        // U = bhalf acc (FP64)
        return launch_bhalf<double>(J, ids, g, acc, U, nullptr, s);
      });
}

hipError_t tune_taylor(const Job* jobs, int n, hipStream_t s) {
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    const Job* J = jobs + c0;
    void *acc[AFQMC_MAXP], *t0[AFQMC_MAXP], *t1[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) propagate_slots(J[q], &acc[q], &t0[q], &t1[q]);
    const hipError_t e = for_groups(
        c, [&](int i) { return taylor_key(J[i].p); },
        [&](const int* ids, int g) -> hipError_t {
          return tune_group(
              TS_TAYLOR, J, ids, g,
              [&](int ch) { return launch_taylor_group(J, ids, g, ch, t0, t1, acc, 1.0, s); }, s);
        });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_propagate(const Job* jobs, int n, int flags, hipStream_t s) {
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    hipError_t e = propagate_jobs(jobs + c0, c, s);
    if (e != hipSuccess) return e;
  }
  // new overlap and Gh; weights from the old and new log overlaps
  hipError_t e = run_greens(jobs, n, true, s);
  if (e != hipSuccess) return e;
  e = launch_weights(jobs, n, s);
  if (e != hipSuccess) return e;
  if (flags & AFQMC_PROPAGATE_ORTHO) return run_ortho(jobs, n, s);
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Re-orthonormalisation by Cholesky-QR applied twice (FP64):
//   S = U^H U, S = L L^H, U <- U L^{-H}.

// S[w][i][j] = sum_R conj(U[w][R][i]) U[w][R][j]
struct OpGram {
  typedef double T;
  static constexpr bool A_KCONTIG = false;
  static constexpr bool B_NCONTIG = true;
  int M, N, K, nbatch;  // M = N = n, K = nk*m
  const cpx<double>* U;
  cpx<double>* S;
  __device__ void load_a(int b, int row, int k, double& re, double& im) const {
    const cpx<double> v = U[((int64_t)b * K + k) * M + row];
    re = v.re; im = -v.im;
  }
  __device__ void load_b(int b, int k, int col, double& re, double& im) const {
    const cpx<double> v = U[((int64_t)b * K + k) * N + col];
    re = v.re; im = v.im;
  }
  __device__ void store(int b, int row, int col, double re, double im) const {
    S[((int64_t)b * M + row) * N + col] = cpx<double>{re, im};
  }
};

// Uo[w] = U[w] Rinv[w]
struct OpRightMul {
  typedef double T;
  static constexpr bool A_KCONTIG = true;
  static constexpr bool B_NCONTIG = true;
  int M, N, K, nbatch;  // M = nk*m, N = K = n
  const cpx<double>* U;
  const cpx<double>* R;
  cpx<double>* Uo;
  __device__ void load_a(int b, int row, int k, double& re, double& im) const {
    const cpx<double> v = U[((int64_t)b * M + row) * K + k];
    re = v.re; im = v.im;
  }
  __device__ void load_b(int b, int k, int col, double& re, double& im) const {
    const cpx<double> v = R[((int64_t)b * K + k) * N + col];
    re = v.re; im = v.im;
  }
  __device__ void store(int b, int row, int col, double re, double im) const {
    Uo[((int64_t)b * M + row) * N + col] = cpx<double>{re, im};
  }
};

static size_t carve_ortho(Carve& c, const afqmc_kpt_problem& p, void** S, void** R, void** Ut,
                          GreensWs& g) {
  Dims d = dims_of(p);
  carve_greens(c, d, g);
  *S = c.take(16 * (size_t)d.W * d.n() * d.n());
  *R = c.take(16 * (size_t)d.W * d.n() * d.n());
  *Ut = c.take(16 * (size_t)d.W * d.N() * d.n());
  return c.off;
}

size_t ortho_ws_bytes(const afqmc_kpt_problem& p) {
  Carve c(nullptr);
  void *a, *b, *t;
  GreensWs g;
  return carve_ortho(c, p, &a, &b, &t, g);
}

hipError_t run_ortho(const Job* jobs, int n, hipStream_t s) {
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    const Job* J = jobs + c0;
    void *S[AFQMC_MAXP], *R[AFQMC_MAXP], *Ut[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      Carve cv(J[q].ws);
      GreensWs g;
      carve_ortho(cv, J[q].p, &S[q], &R[q], &Ut[q], g);
    }
    // pass 0: U -> Ut, pass 1: Ut -> U
    for (int pass = 0; pass < 2; ++pass) {
      TimedScope ts(KC_ORTHO, s);
      OpGram gm[AFQMC_MAXP];
      OpRightMul rm[AFQMC_MAXP];
      for (int q = 0; q < c; ++q) {
        const afqmc_kpt_problem& p = J[q].p;
        const int nn = p.nk * p.nocc, Nn = p.nk * p.m;
        const cpx<double>* src = (const cpx<double>*)(pass == 0 ? p.U : Ut[q]);
        cpx<double>* dst = (cpx<double>*)(pass == 0 ? Ut[q] : p.U);
        gm[q].M = nn; gm[q].N = nn; gm[q].K = Nn; gm[q].nbatch = p.nwalk;
        gm[q].U = src;
        gm[q].S = (cpx<double>*)S[q];
        rm[q].M = Nn; rm[q].N = nn; rm[q].K = nn; rm[q].nbatch = p.nwalk;
        rm[q].U = src;
        rm[q].R = (const cpx<double>*)R[q];
        rm[q].Uo = dst;
      }
      hipError_t e = launch_ops<32, 32, 16, 2, 2>(gm, c, s);
      if (e != hipSuccess) return e;
      e = launch_small_gj(J, c, GJ_MODE_CHOL_INV, S, R, nullptr, s);
      if (e != hipSuccess) return e;
      e = launch_ops<64, 64, 16, 2, 2>(rm, c, s);
      if (e != hipSuccess) return e;
    }
  }
  // Gh and the log overlap of the re-orthonormalised walkers
  return run_greens(jobs, n, false, s);
}

}  // namespace afqmc
