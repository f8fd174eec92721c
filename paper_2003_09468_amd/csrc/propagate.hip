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

hipError_t launch_weights(const afqmc_kpt_problem& p, const double* x, const void* xbar,
                          const void* logdet_new, hipStream_t s);

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

template <typename TO>
static hipError_t launch_bhalf(const afqmc_kpt_problem& p, const void* in, void* out, void* outT,
                               hipStream_t s) {
  OpBhalf<TO> op;
  op.M = p.m; op.K = p.m; op.N = p.nk * p.nocc;
  op.nbatch = p.nwalk * p.nk;
  op.nk = p.nk;
  op.B = (const cpx<double>*)p.bhalf;
  op.in = (const cpx<double>*)in;
  op.out = (cpx<double>*)out;
  op.outT = (cpx<TO>*)outT;
  TimedScope ts(KC_BHALF, s);
  if (p.m <= 16) return launch_cgemm<16, 64, 16, 1, 4>(op, s);
  return launch_cgemm<32, 64, 16, 2, 2>(op, s);
}

template <typename T>
static hipError_t launch_taylor(const afqmc_kpt_problem& p, const void* vhs, const void* tin,
                                void* tout, void* acc, double alpha, hipStream_t s) {
  OpTaylor<T> op;
  op.M = p.nk * p.m; op.K = p.nk * p.m; op.N = p.nk * p.nocc;
  op.nbatch = p.nwalk;
  op.alpha = (T)alpha;
  op.V = (const cpx<T>*)vhs;
  op.Tin = (const cpx<T>*)tin;
  op.Tout = (cpx<T>*)tout;
  op.acc = (cpx<double>*)acc;
  TimedScope ts(KC_TAYLOR, s);
  // FP32: one column tile spans all nk*nocc columns (rounded up to 16), each of the 4 waves
  // owning 16 rows x BN columns.  FP64: 64 x 32 tiles (measured fastest for the 16x16x4
  // FP64 MFMA at 702 x 108 x 702).
  if (sizeof(T) == 8) return launch_cgemm<64, 32, 16, 4, 1>(op, s);
  switch ((op.N + 15) / 16) {
    case 1: return launch_cgemm<64, 16, 16, 4, 1>(op, s);
    case 2: return launch_cgemm<64, 32, 16, 4, 1>(op, s);
    case 3: return launch_cgemm<64, 48, 16, 4, 1>(op, s);
    case 4: return launch_cgemm<64, 64, 16, 4, 1>(op, s);
    case 5: return launch_cgemm<64, 80, 16, 4, 1>(op, s);
    case 6: return launch_cgemm<64, 96, 16, 4, 1>(op, s);
    case 7: return launch_cgemm<64, 112, 16, 4, 1>(op, s);
    case 8: return launch_cgemm<64, 128, 16, 4, 1>(op, s);
    default: return launch_cgemm<64, 64, 16, 2, 2>(op, s);
  }
}

// Layout: the Green's-function slots come first in every entry's workspace, so that
// run_greens (which carves from the start) and the weight update agree on them.
static size_t carve_propagate(Carve& c, const afqmc_kpt_problem& p, void** acc, void** t0,
                              void** t1, GreensWs& g) {
  Dims d = dims_of(p);
  const size_t tsz = (p.prec == AFQMC_PREC_FP32) ? 8 : 16;
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

template <typename T>
static hipError_t propagate_typed(const afqmc_kpt_problem& p, const void* vhs, void* acc, void* t0,
                                  void* t1, hipStream_t s) {
  hipError_t e;
  // T_0 = bhalf U (FP64), acc = T_0, t0 = T_0 in the Taylor precision
  e = launch_bhalf<T>(p, p.U, acc, t0, s);
  if (e != hipSuccess) return e;
  const double sdt = sqrt(p.dt);
  void* tin = t0;
  void* tout = t1;
  for (int j = 1; j <= 6; ++j) {
    e = launch_taylor<T>(p, vhs, tin, (j < 6) ? tout : nullptr, acc, -sdt / j, s);
    if (e != hipSuccess) return e;
    void* t = tin; tin = tout; tout = t;
  }
  // U = bhalf acc (FP64)
  return launch_bhalf<double>(p, acc, p.U, nullptr, s);
}

hipError_t run_propagate(const afqmc_kpt_problem& p, const void* vhs, const double* x,
                         const void* xbar, int flags, void* ws, hipStream_t s) {
  Carve c(ws);
  void *acc, *t0, *t1;
  GreensWs g;
  carve_propagate(c, p, &acc, &t0, &t1, g);
  hipError_t e = (p.prec == AFQMC_PREC_FP32) ? propagate_typed<float>(p, vhs, acc, t0, t1, s)
                                             : propagate_typed<double>(p, vhs, acc, t0, t1, s);
  if (e != hipSuccess) return e;
  // new overlap and Gh; weights from the old and new log overlaps
  e = run_greens(p, ws, true, s);
  if (e != hipSuccess) return e;
  e = launch_weights(p, x, xbar, g.logdet_new, s);
  if (e != hipSuccess) return e;
  if (flags & AFQMC_PROPAGATE_ORTHO) return run_ortho(p, ws, s);
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

hipError_t run_ortho(const afqmc_kpt_problem& p, void* ws, hipStream_t s) {
  Carve c(ws);
  void *S, *R, *Ut;
  GreensWs g;
  carve_ortho(c, p, &S, &R, &Ut, g);
  const int n = p.nk * p.nocc;
  const int Nn = p.nk * p.m;
  hipError_t e;
  // pass 0: U -> Ut, pass 1: Ut -> U
  for (int pass = 0; pass < 2; ++pass) {
    TimedScope ts(KC_ORTHO, s);
    const cpx<double>* src = (const cpx<double>*)(pass == 0 ? p.U : Ut);
    cpx<double>* dst = (cpx<double>*)(pass == 0 ? Ut : p.U);
    OpGram gm;
    gm.M = n; gm.N = n; gm.K = Nn; gm.nbatch = p.nwalk;
    gm.U = src;
    gm.S = (cpx<double>*)S;
    e = launch_cgemm<32, 32, 16, 2, 2>(gm, s);
    if (e != hipSuccess) return e;
    e = launch_small_gj(p, GJ_MODE_CHOL_INV, S, R, nullptr, s);
    if (e != hipSuccess) return e;
    OpRightMul r;
    r.M = Nn; r.N = n; r.K = n; r.nbatch = p.nwalk;
    r.U = src;
    r.R = (const cpx<double>*)R;
    r.Uo = dst;
    e = launch_cgemm<64, 64, 16, 2, 2>(r, s);
    if (e != hipSuccess) return e;
  }
  // Gh and the log overlap of the re-orthonormalised walkers
  return run_greens(p, ws, false, s);
}

}  // namespace afqmc
