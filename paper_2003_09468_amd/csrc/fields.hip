// Force bias and HS potential (k-point force-bias and HS-matrix equations).
//
// Force bias: X[w][Q][g] = 2 sum_k sum_{a,r} Lh[Q][k][a][r][g] Gh[w][(k a), ((k-Q) r)].
// For each Q this is a (nchol x W) GEMM with K = nk*nocc*m running over the half-rotated
// Cholesky vectors; the K range is split over k-point groups so that the launch fills the
// chip, and a deterministic reduction forms X and the +/- force biases.
//
// HS potential: every (k1, k2) block of the dense walker potential is filled by exactly
// one Q = k1 - k2, so vhs[w][(k p), ((k-Q) r)] = sum_g L[Q][k][p][r][g] zeta[w][Q][g] is,
// per Q, a (W x nk*m*m) GEMM with K = nchol.  L is streamed once with the Cholesky index
// contiguous; walkers are the MFMA rows so that each 16-lane group writes consecutive r.
#include <math.h>

#include "cgemm.h"
#include "internal.h"

namespace afqmc {

// partial X: part[s][w][Q][g] = sum over the k of slice s of sum_{a,r} Lh Gh
template <typename TT>
struct OpVbias {
  typedef TT T;
  static constexpr bool A_KCONTIG = false;  // A(row=g, k) = Lh[...][g]: contiguous along g
  static constexpr bool B_NCONTIG = false;  // B(k, col=w): contiguous along r inside k
  int M, N, K, nbatch;
  int nk, m, nocc, C, S, kper;  // kper k-points per slice
  KMesh mesh;
  const cpx<T>* Lh;             // [nk][nk][nocc][m][C]
  const cpx<double>* Gh;        // [W][nk*nocc][nk*m]
  cpx<double>* part;            // [S][W][nk][C]
  __device__ void load_a(int b, int row, int k, T& re, T& im) const {
    const int Q = b / S, s = b % S;
    const int64_t kk = (int64_t)s * kper * nocc * m + k;  // global (k, a, r) index
    if (kk >= (int64_t)nk * nocc * m) { re = 0; im = 0; return; }
    const cpx<T> v = Lh[((int64_t)Q * nk * nocc * m + kk) * C + row];
    re = v.re; im = v.im;
  }
  __device__ void load_b(int b, int k, int col, T& re, T& im) const {
    const int Q = b / S, s = b % S;
    const int64_t kk = (int64_t)s * kper * nocc * m + k;
    if (kk >= (int64_t)nk * nocc * m) { re = 0; im = 0; return; }
    const int kp = (int)(kk / (nocc * m));
    const int ar = (int)(kk % (nocc * m));
    const int a = ar / m, r = ar % m;
    const int k2 = mesh.kmq(kp, Q);
    const int64_t Nn = (int64_t)nk * m;
    const cpx<double> v = Gh[((int64_t)col * nk * nocc + (int64_t)kp * nocc + a) * Nn + (int64_t)k2 * m + r];
    re = (T)v.re; im = (T)v.im;
  }
  __device__ void store(int b, int row, int col, T re, T im) const {
    const int Q = b / S, s = b % S;
    part[(((int64_t)s * N + col) * nk + Q) * C + row] = cpx<double>{(double)re, (double)im};
  }
};

struct VredArgs {
  int W, nk, C, S;
  KMesh mesh;
  double sdt;
  const cpx<double>* part;  // [S][W][nk][C]
  cpx<double>* X;           // [W][nk][C] (may be null)
  cpx<double>* xbar;        // [W][nk][C][2] (may be null)
};

__global__ __launch_bounds__(256) void vbias_reduce_kernel(const Batch<VredArgs> B) {
  long long bloc;
  const int pb = batch_find(B, blockIdx.x, bloc);
  const int W = B.a[pb].W, nk = B.a[pb].nk, C = B.a[pb].C, S = B.a[pb].S;
  const KMesh mesh = B.a[pb].mesh;
  const double sdt = B.a[pb].sdt;
  const cpx<double>* __restrict__ part = B.a[pb].part;
  cpx<double>* __restrict__ X = B.a[pb].X;
  cpx<double>* __restrict__ xbar = B.a[pb].xbar;
  const int64_t idx = bloc * 256 + threadIdx.x;
  const int64_t total = (int64_t)W * nk * C;
  if (idx >= total) return;
  const int g = (int)(idx % C);
  const int Q = (int)((idx / C) % nk);
  const int w = (int)(idx / ((int64_t)C * nk));
  const int mQ = mesh.neg(Q);
  double xr = 0, xi = 0, yr = 0, yi = 0;
  for (int s = 0; s < S; ++s) {
    const cpx<double> a = part[(((int64_t)s * W + w) * nk + Q) * C + g];
    const cpx<double> b = part[(((int64_t)s * W + w) * nk + mQ) * C + g];
    xr += a.re; xi += a.im; yr += b.re; yi += b.im;
  }
  xr *= 2.0; xi *= 2.0; yr *= 2.0; yi *= 2.0;  // both spins
  if (X) X[idx] = cpx<double>{xr, xi};
  if (xbar) {
    // xbar+ = -sqrt(dt) (i/2)(X_Q + X_-Q);  xbar- = -sqrt(dt) (1/2)(X_Q - X_-Q)
    const double sr = xr + yr, si = xi + yi;
    const double dr = xr - yr, di = xi - yi;
    xbar[2 * idx + 0] = cpx<double>{0.5 * sdt * si, -0.5 * sdt * sr};
    xbar[2 * idx + 1] = cpx<double>{-0.5 * sdt * dr, -0.5 * sdt * di};
  }
}

size_t carve_vbias(Carve& c, const Dims& d, VbiasWs& v) {
  v.parts = c.take(sizeof(double) * 2 * (size_t)vbias_splits(d) * d.W * d.nk * d.C);
  return c.off;
}

template <typename T>
static OpVbias<T> vbias_op(const afqmc_kpt_problem& p, void* parts) {
  Dims d = dims_of(p);
  OpVbias<T> op;
  op.nk = p.nk; op.m = p.m; op.nocc = p.nocc; op.C = p.nchol;
  op.S = vbias_splits(d);
  op.kper = (p.nk + op.S - 1) / op.S;
  op.mesh = make_mesh(p);
  op.M = p.nchol;
  op.N = p.nwalk;
  op.K = op.kper * p.nocc * p.m;
  op.nbatch = p.nk * op.S;
  op.Lh = (const cpx<T>*)(sizeof(T) == 8 ? p.Lh : p.Lh32);
  op.Gh = (const cpx<double>*)p.Gh;
  op.part = (cpx<double>*)parts;
  return op;
}

template <typename T>
static hipError_t vbias_tiles(const OpVbias<T>* ops, int c, int choice, hipStream_t s) {
  switch (choice) {
    case 1: return launch_ops<32, 64, 16, 2, 2>(ops, c, s);
    case 2: return launch_ops<64, 32, 16, 4, 1>(ops, c, s);
    default: return launch_ops<64, 64, 16, 2, 2>(ops, c, s);
  }
}

// Split-K partial traces of a group of jobs of one precision.
hipError_t launch_vbias_group(const Job* jobs, const int* ids, int c, int choice,
                              void* const* parts, hipStream_t s) {
  if (low_prec(jobs[ids[0]].p.prec)) {
    OpVbias<float> ops[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) ops[q] = vbias_op<float>(jobs[ids[q]].p, parts[ids[q]]);
    return vbias_tiles<float>(ops, c, choice, s);
  }
  OpVbias<double> ops[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) ops[q] = vbias_op<double>(jobs[ids[q]].p, parts[ids[q]]);
  return vbias_tiles<double>(ops, c, choice, s);
}

// X (and xbar where requested) for the current Gh of every job.
hipError_t launch_cholesky_trace(const Job* jobs, int n, void* const* X, void* const* xbar,
                                 void* const* parts, hipStream_t s) {
  TimedScope ts(KC_VBIAS, s);
  hipError_t e = for_groups(
      n, [&](int i) { return jobs[i].p.prec; },
      [&](const int* ids, int c) -> hipError_t {
        const int choice = tune_lookup(tune_key(TS_VBIAS, jobs, ids, c));
        return launch_vbias_group(jobs, ids, c, choice, parts, s);
      });
  if (e != hipSuccess) return e;
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    Batch<VredArgs> B;
    B.nprob = c;
    long long cnt[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const afqmc_kpt_problem& p = jobs[c0 + q].p;
      VredArgs& a = B.a[q];
      a.W = p.nwalk; a.nk = p.nk; a.C = p.nchol;
      a.S = vbias_splits(dims_of(p));
      a.mesh = make_mesh(p);
      a.sdt = sqrt(p.dt);
      a.part = (const cpx<double>*)parts[c0 + q];
      a.X = X ? (cpx<double>*)X[c0 + q] : nullptr;
      a.xbar = xbar ? (cpx<double>*)xbar[c0 + q] : nullptr;
      cnt[q] = ((int64_t)p.nwalk * p.nk * p.nchol + 255) / 256;
    }
    const long long g = batch_close(B, cnt);
    if (g < 0) return hipErrorInvalidValue;
    if (g == 0) continue;
    hipLaunchKernelGGL(vbias_reduce_kernel, dim3((unsigned)g), dim3(256), 0, s, B);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_vbias(const Job* jobs, int n, hipStream_t s) {
  void* X[64];
  void* xb[64];
  void* parts[64];
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int c = (n - c0 < 64) ? n - c0 : 64;
    for (int q = 0; q < c; ++q) {
      const Job& j = jobs[c0 + q];
      Carve cv(j.ws);
      VbiasWs v;
      carve_vbias(cv, dims_of(j.p), v);
      X[q] = j.X;
      xb[q] = j.xbar;
      parts[q] = v.parts;
    }
    hipError_t e = launch_cholesky_trace(jobs + c0, c, X, xb, parts, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t tune_vbias(const Job* jobs, int n, hipStream_t s) {
  void* parts[64];
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int c = (n - c0 < 64) ? n - c0 : 64;
    const Job* J = jobs + c0;
    for (int q = 0; q < c; ++q) {
      Carve cv(J[q].ws);
      VbiasWs v;
      carve_vbias(cv, dims_of(J[q].p), v);
      parts[q] = v.parts;
    }
    const hipError_t e = for_groups(
        c, [&](int i) { return J[i].p.prec; },
        [&](const int* ids, int g) -> hipError_t {
          return tune_group(
              TS_VBIAS, J, ids, g,
              [&](int ch) { return launch_vbias_group(J, ids, g, ch, parts, s); }, s);
        });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// combined field: zeta = -xi, xi = 1/2 [ i (xt+_Q + xt+_-Q) + (xt-_Q - xt-_-Q) ]
struct FieldArgs {
  int W, nk, C;
  KMesh mesh;
  const double* x;           // [W][nk][C][2]
  const cpx<double>* xbar;   // [W][nk][C][2]
  void* zeta;                // [W][nk][C] in the contraction precision
};

template <typename T>
__global__ __launch_bounds__(256) void field_kernel(const Batch<FieldArgs> B) {
  long long bloc;
  const int pb = batch_find(B, blockIdx.x, bloc);
  const int W = B.a[pb].W, nk = B.a[pb].nk, C = B.a[pb].C;
  const KMesh mesh = B.a[pb].mesh;
  const double* __restrict__ x = B.a[pb].x;
  const cpx<double>* __restrict__ xbar = B.a[pb].xbar;
  cpx<T>* __restrict__ zeta = (cpx<T>*)B.a[pb].zeta;
  const int64_t idx = bloc * 256 + threadIdx.x;
  const int64_t total = (int64_t)W * nk * C;
  if (idx >= total) return;
  const int g = (int)(idx % C);
  const int Q = (int)((idx / C) % nk);
  const int w = (int)(idx / ((int64_t)C * nk));
  const int64_t jdx = ((int64_t)w * nk + mesh.neg(Q)) * C + g;
  // xt = x - xbar
  const double apr = x[2 * idx] - xbar[2 * idx].re, api = -xbar[2 * idx].im;
  const double amr = x[2 * idx + 1] - xbar[2 * idx + 1].re, ami = -xbar[2 * idx + 1].im;
  const double bpr = x[2 * jdx] - xbar[2 * jdx].re, bpi = -xbar[2 * jdx].im;
  const double bmr = x[2 * jdx + 1] - xbar[2 * jdx + 1].re, bmi = -xbar[2 * jdx + 1].im;
  const double sr = apr + bpr, si = api + bpi;  // xt+_Q + xt+_-Q
  const double dr = amr - bmr, di = ami - bmi;  // xt-_Q - xt-_-Q
  // xi = 0.5 (i s + d)
  const double xr = 0.5 * (-si + dr), xi = 0.5 * (sr + di);
  zeta[idx] = cpx<T>{(T)(-xr), (T)(-xi)};
}

template <typename TT>
struct OpVhs {
  typedef TT T;
  static constexpr bool A_KCONTIG = true;   // zeta[w][Q][g]
  static constexpr bool B_NCONTIG = false;  // L[Q][(k p r)][g]: contiguous along g
  int M, N, K, nbatch;
  int nk, m;
  KMesh mesh;
  const cpx<T>* zeta;  // [W][nk][C]
  const cpx<T>* L;     // [nk][nk][m][m][C]
  cpx<T>* vhs;         // [W][nk*m][nk*m]
  __device__ void load_a(int b, int row, int k, T& re, T& im) const {
    const cpx<T> v = zeta[((int64_t)row * nk + b) * K + k];
    re = v.re; im = v.im;
  }
  __device__ void load_b(int b, int k, int col, T& re, T& im) const {
    const cpx<T> v = L[((int64_t)b * N + col) * K + k];
    re = v.re; im = v.im;
  }
  __device__ void store(int b, int row, int col, T re, T im) const {
    const int mm = m * m;
    const int kp = col / mm, pr = col % mm;
    const int p = pr / m, r = pr % m;
    const int k2 = mesh.kmq(kp, b);
    const int64_t Nn = (int64_t)nk * m;
    vhs[((int64_t)row * Nn + (int64_t)kp * m + p) * Nn + (int64_t)k2 * m + r] = cpx<T>{re, im};
  }
};

template <typename T>
static OpVhs<T> vhs_op(const Job& j, void* zeta) {
  const afqmc_kpt_problem& p = j.p;
  OpVhs<T> op;
  op.nk = p.nk; op.m = p.m; op.mesh = make_mesh(p);
  op.M = p.nwalk;
  op.N = p.nk * p.m * p.m;
  op.K = p.nchol;
  op.nbatch = p.nk;
  op.zeta = (const cpx<T>*)zeta;
  op.L = (const cpx<T>*)(sizeof(T) == 8 ? p.L : p.L32);
  op.vhs = (cpx<T>*)j.vhs;
  return op;
}

// Rows = walkers, (k p r) columns.  Default tiles measured at 27 x 64 x 18252 x 208.
template <typename T>
static hipError_t vhs_tiles(const OpVhs<T>* ops, int c, int choice, hipStream_t s) {
  // the default follows the walker count (the rows): 32-row tiles for W <= 32
  int mmax = 0;
  for (int q = 0; q < c; ++q) mmax = ops[q].M > mmax ? ops[q].M : mmax;
  if (choice == 0 && mmax <= 32) return launch_ops<32, 64, 16, 2, 2>(ops, c, s);
  if constexpr (sizeof(T) == 8) {
    switch (choice) {
      case 1: return launch_ops<64, 64, 16, 2, 2>(ops, c, s);
      case 2: return launch_ops<32, 64, 16, 2, 2>(ops, c, s);
      default: return launch_ops<64, 32, 16, 4, 1>(ops, c, s);
    }
  } else {
    switch (choice) {
      case 1: return launch_ops<64, 32, 16, 4, 1>(ops, c, s);
      case 2: return launch_ops<64, 128, 16, 2, 2>(ops, c, s);
      default: return launch_ops<64, 64, 16, 2, 2>(ops, c, s);
    }
  }
}

hipError_t launch_vhs_group(const Job* jobs, const int* ids, int c, int choice,
                            void* const* zeta, hipStream_t s) {
  if (low_prec(jobs[ids[0]].p.prec)) {
    OpVhs<float> ops[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) ops[q] = vhs_op<float>(jobs[ids[q]], zeta[ids[q]]);
    return vhs_tiles<float>(ops, c, choice, s);
  }
  OpVhs<double> ops[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) ops[q] = vhs_op<double>(jobs[ids[q]], zeta[ids[q]]);
  return vhs_tiles<double>(ops, c, choice, s);
}

// Launch groups of the HS potential: precision and walker-count class (the rows of its
// tiles), so that every problem gets its default tile shape.
static int vhs_key(const afqmc_kpt_problem& p) { return p.prec * 2 + (p.nwalk <= 32 ? 1 : 0); }

hipError_t run_vhs(const Job* jobs, int n, hipStream_t s) {
  TimedScope ts(KC_VHS, s);
  void* zeta[64];
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int c = (n - c0 < 64) ? n - c0 : 64;
    const Job* J = jobs + c0;
    for (int q = 0; q < c; ++q) {
      Carve cv(J[q].ws);
      zeta[q] = cv.take(sizeof(double) * 2 * (size_t)J[q].p.nwalk * J[q].p.nk * J[q].p.nchol);
    }
    hipError_t e = for_groups(
        c, [&](int i) { return vhs_key(J[i].p); },
        [&](const int* ids, int g) -> hipError_t {
          Batch<FieldArgs> B;
          B.nprob = g;
          long long cnt[AFQMC_MAXP];
          for (int q = 0; q < g; ++q) {
            const Job& j = J[ids[q]];
            FieldArgs& a = B.a[q];
            a.W = j.p.nwalk; a.nk = j.p.nk; a.C = j.p.nchol;
            a.mesh = make_mesh(j.p);
            a.x = j.x;
            a.xbar = (const cpx<double>*)j.xbar;
            a.zeta = zeta[ids[q]];
            cnt[q] = ((int64_t)j.p.nwalk * j.p.nk * j.p.nchol + 255) / 256;
          }
          const long long grid = batch_close(B, cnt);
          if (grid < 0) return hipErrorInvalidValue;
          if (grid > 0) {
            if (low_prec(J[ids[0]].p.prec))
              hipLaunchKernelGGL(field_kernel<float>, dim3((unsigned)grid), dim3(256), 0, s, B);
            else
              hipLaunchKernelGGL(field_kernel<double>, dim3((unsigned)grid), dim3(256), 0, s, B);
            const hipError_t e2 = hipGetLastError();
            if (e2 != hipSuccess) return e2;
          }
          const int choice = tune_lookup(tune_key(TS_VHS, J, ids, g));
          return launch_vhs_group(J, ids, g, choice, zeta, s);
        });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t tune_vhs(const Job* jobs, int n, hipStream_t s) {
  void* zeta[64];
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int c = (n - c0 < 64) ? n - c0 : 64;
    const Job* J = jobs + c0;
    for (int q = 0; q < c; ++q) {
      Carve cv(J[q].ws);
      zeta[q] = cv.take(sizeof(double) * 2 * (size_t)J[q].p.nwalk * J[q].p.nk * J[q].p.nchol);
    }
    const hipError_t e = for_groups(
        c, [&](int i) { return vhs_key(J[i].p); },
        [&](const int* ids, int g) -> hipError_t {
          return tune_group(
              TS_VHS, J, ids, g, [&](int ch) { return launch_vhs_group(J, ids, g, ch, zeta, s); },
              s);
        });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace afqmc
