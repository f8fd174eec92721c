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

__global__ void vbias_reduce_kernel(int W, int nk, int C, int S, KMesh mesh, double sdt,
                                    const cpx<double>* __restrict__ part,
                                    cpx<double>* __restrict__ X, cpx<double>* __restrict__ xbar) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
static hipError_t launch_vbias_gemm(const afqmc_kpt_problem& p, void* parts, hipStream_t s) {
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
  return launch_cgemm<64, 64, 16, 2, 2>(op, s);
}

// X (and optionally xbar) for the current Gh.
hipError_t launch_cholesky_trace_x(const afqmc_kpt_problem& p, void* X, void* xbar, void* parts,
                                   hipStream_t s) {
  TimedScope ts(KC_VBIAS, s);
  hipError_t e = (p.prec == AFQMC_PREC_FP32) ? launch_vbias_gemm<float>(p, parts, s)
                                             : launch_vbias_gemm<double>(p, parts, s);
  if (e != hipSuccess) return e;
  Dims d = dims_of(p);
  const int64_t total = d.W * d.nk * d.C;
  const int S = vbias_splits(d);
  hipLaunchKernelGGL(vbias_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     p.nwalk, p.nk, p.nchol, S, make_mesh(p), sqrt(p.dt),
                     (const cpx<double>*)parts, (cpx<double>*)X, (cpx<double>*)xbar);
  return hipGetLastError();
}

hipError_t launch_cholesky_trace(const afqmc_kpt_problem& p, void* X, void* parts, hipStream_t s) {
  return launch_cholesky_trace_x(p, X, nullptr, parts, s);
}

hipError_t run_vbias(const afqmc_kpt_problem& p, void* xbar, void* X, void* ws, hipStream_t s) {
  Carve c(ws);
  VbiasWs v;
  carve_vbias(c, dims_of(p), v);
  return launch_cholesky_trace_x(p, X, xbar, v.parts, s);
}

// ---------------------------------------------------------------------------
// combined field: zeta = -xi, xi = 1/2 [ i (xt+_Q + xt+_-Q) + (xt-_Q - xt-_-Q) ]
template <typename T>
__global__ void field_kernel(int W, int nk, int C, KMesh mesh, const double* __restrict__ x,
                             const cpx<double>* __restrict__ xbar, cpx<T>* __restrict__ zeta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
static hipError_t launch_vhs_typed(const afqmc_kpt_problem& p, const double* x, const void* xbar,
                                   void* vhs, void* zeta, hipStream_t s) {
  TimedScope ts(KC_VHS, s);
  const int64_t total = (int64_t)p.nwalk * p.nk * p.nchol;
  hipLaunchKernelGGL(field_kernel<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     p.nwalk, p.nk, p.nchol, make_mesh(p), x, (const cpx<double>*)xbar,
                     (cpx<T>*)zeta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  OpVhs<T> op;
  op.nk = p.nk; op.m = p.m; op.mesh = make_mesh(p);
  op.M = p.nwalk;
  op.N = p.nk * p.m * p.m;
  op.K = p.nchol;
  op.nbatch = p.nk;
  op.zeta = (const cpx<T>*)zeta;
  op.L = (const cpx<T>*)(sizeof(T) == 8 ? p.L : p.L32);
  op.vhs = (cpx<T>*)vhs;
  // rows = walkers, (k p r) columns; tiles measured at 27 x 64 x 18252 x 208
  if (sizeof(T) == 8) return launch_cgemm<64, 32, 16, 4, 1>(op, s);
  return launch_cgemm<64, 64, 16, 2, 2>(op, s);
}

hipError_t run_vhs(const afqmc_kpt_problem& p, const double* x, const void* xbar, void* vhs,
                   void* ws, hipStream_t s) {
  Carve c(ws);
  void* zeta = c.take(sizeof(double) * 2 * (size_t)p.nwalk * p.nk * p.nchol);
  if (p.prec == AFQMC_PREC_FP32) return launch_vhs_typed<float>(p, x, xbar, vhs, zeta, s);
  return launch_vhs_typed<double>(p, x, xbar, vhs, zeta, s);
}

}  // namespace afqmc
