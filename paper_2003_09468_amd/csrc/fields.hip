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

// The combined field as BF16 split planes for the three-pass HS potential:
//   zs[w][Q][plane][g], planes (re hi, re lo, im hi, im lo) of the FP32-rounded zeta,
//   g contiguous and zero-padded to CP = 32 ceil(C / 32).
__global__ __launch_bounds__(256) void field_split_kernel(const Batch<FieldArgs> B) {
  long long bloc;
  const int pb = batch_find(B, blockIdx.x, bloc);
  const int W = B.a[pb].W, nk = B.a[pb].nk, C = B.a[pb].C;
  const int CP = 32 * ((C + 31) / 32);
  const KMesh mesh = B.a[pb].mesh;
  const double* __restrict__ x = B.a[pb].x;
  const cpx<double>* __restrict__ xbar = B.a[pb].xbar;
  unsigned short* __restrict__ zs = (unsigned short*)B.a[pb].zeta;
  const int64_t idx = bloc * 256 + threadIdx.x;
  const int64_t total = (int64_t)W * nk * CP;
  if (idx >= total) return;
  const int g = (int)(idx % CP);
  const int64_t wq = idx / CP;  // w nk + Q
  const int Q = (int)(wq % nk), w = (int)(wq / nk);
  float zr = 0.f, zi = 0.f;
  if (g < C) {
    const int64_t i = wq * C + g;
    const int64_t j = ((int64_t)w * nk + mesh.neg(Q)) * C + g;
    const double apr = x[2 * i] - xbar[2 * i].re, api = -xbar[2 * i].im;
    const double amr = x[2 * i + 1] - xbar[2 * i + 1].re, ami = -xbar[2 * i + 1].im;
    const double bpr = x[2 * j] - xbar[2 * j].re, bpi = -xbar[2 * j].im;
    const double bmr = x[2 * j + 1] - xbar[2 * j + 1].re, bmi = -xbar[2 * j + 1].im;
    const double sr = apr + bpr, si = api + bpi, dr = amr - bmr, di = ami - bmi;
    zr = (float)(-0.5 * (-si + dr));
    zi = (float)(-0.5 * (sr + di));
  }
  unsigned short rh, rl, ih, il;
  bf16_split(zr, rh, rl);
  bf16_split(zi, ih, il);
  unsigned short* o = zs + wq * 4 * CP + g;
  o[0] = rh;
  o[CP] = rl;
  o[2 * CP] = ih;
  o[3 * CP] = il;
}

// HS potential on the three-pass BF16 split:
//   vhs[w][(k p), ((k-Q) r)] = sum_g zeta[w][Q][g] L[Q][k][p][r][g]
// per Q a (W x nk m m) product with K = nchol, 64 x 64 tiles of four waves (2 x 2, each
// 32 x 32), K in chunks of 32; both operands come as split planes with g contiguous and
// are staged into LDS with 16-byte copies; 12 BF16 MFMAs per complex 16 x 16 x 32 block.
struct VhsBfArgs {
  int W, nk, m, C, tiles_m, tiles_n;
  KMesh mesh;
  const unsigned short* zs;  // [W][nk][4][CP]
  const unsigned short* Ls;  // [nk][nk m m][4][CP]
  cpx<float>* vhs;           // [W][nk m][nk m]
};

__global__ __launch_bounds__(256) void vhs_bf16x3_kernel(const Batch<VhsBfArgs> B) {
  constexpr int BM = 64, BN = 64, BKC = 32, RS = BKC + 8;
  __shared__ __attribute__((aligned(16))) unsigned short sA[2][4][BM][RS];
  __shared__ __attribute__((aligned(16))) unsigned short sB[2][4][BN][RS];
  long long bloc;
  const int pb = batch_find(B, blockIdx.x, bloc);
  const VhsBfArgs& a = B.a[pb];
  const int W = a.W, nk = a.nk, m = a.m, C = a.C;
  const int CP = 32 * ((C + 31) / 32);
  const int ncol = nk * m * m;
  const int per_q = a.tiles_m * a.tiles_n;
  const int Q = (int)(bloc / per_q);
  const int rem = (int)(bloc % per_q);
  const int row0 = (rem / a.tiles_n) * BM, col0 = (rem % a.tiles_n) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const unsigned short* __restrict__ zs = a.zs;
  const unsigned short* __restrict__ Ls = a.Ls + (int64_t)Q * ncol * 4 * CP;

  // 16-byte units of a chunk: u = (row 4 + plane) 4 + c8; 64 rows x 4 planes x 4 = 1024
  uint4 pa[4], pbu[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = tid + 256 * e;
      const int r = u >> 4, pl = (u >> 2) & 3, c8 = u & 3;
      uint4 va = {0u, 0u, 0u, 0u}, vb = {0u, 0u, 0u, 0u};
      const int w = row0 + r;
      if (w < W)
        va = *reinterpret_cast<const uint4*>(
            zs + (((int64_t)w * nk + Q) * 4 + pl) * CP + k0 + 8 * c8);
      const int col = col0 + r;
      if (col < ncol)
        vb = *reinterpret_cast<const uint4*>(Ls + ((int64_t)col * 4 + pl) * CP + k0 + 8 * c8);
      pa[e] = va;
      pbu[e] = vb;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = tid + 256 * e;
      const int r = u >> 4, pl = (u >> 2) & 3, c8 = u & 3;
      *reinterpret_cast<uint4*>(&sA[buf][pl][r][8 * c8]) = pa[e];
      *reinterpret_cast<uint4*>(&sB[buf][pl][r][8 * c8]) = pbu[e];
    }
  };

  v4f acr[2][2], aci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acr[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      aci[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  const u16x8 sgn = {0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000};
  const int nch = CP / BKC;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) fetch((c + 1) * BKC);
    const int kq = 8 * (lane >> 4);
    u16x8 fa[2][4], fb[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        fa[i][pl] = *reinterpret_cast<const u16x8*>(&sA[buf][pl][wm * 32 + i * 16 + (lane & 15)][kq]);
        fb[i][pl] = *reinterpret_cast<const u16x8*>(&sB[buf][pl][wn * 32 + i * 16 + (lane & 15)][kq]);
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // re += Ar Br - Ai Bi,  im += Ar Bi + Ai Br
        acr[i][j] = mul3(fa[i][0], fa[i][1], fb[j][0], fb[j][1], acr[i][j]);
        acr[i][j] = mul3(fa[i][2] ^ sgn, fa[i][3] ^ sgn, fb[j][2], fb[j][3], acr[i][j]);
        aci[i][j] = mul3(fa[i][0], fa[i][1], fb[j][2], fb[j][3], aci[i][j]);
        aci[i][j] = mul3(fa[i][2], fa[i][3], fb[j][0], fb[j][1], aci[i][j]);
      }
    if (c + 1 < nch) stash(buf ^ 1);
    __syncthreads();
  }
  // scatter: column (k p r) of Q to vhs[w][(k p)][((k - Q) r)]
  const int64_t Nn = (int64_t)nk * m;
  const int mm = m * m;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int w = row0 + wm * 32 + i * 16 + mfma16<float>::drow(lane, v);
        const int col = col0 + wn * 32 + j * 16 + (lane & 15);
        if (w >= W || col >= ncol) continue;
        const int kp = col / mm, pr = col % mm;
        const int p = pr / m, r = pr % m;
        const int k2 = a.mesh.kmq(kp, Q);
        a.vhs[((int64_t)w * Nn + (int64_t)kp * m + p) * Nn + (int64_t)k2 * m + r] =
            cpx<float>{acr[i][j][v], aci[i][j][v]};
      }
}

static hipError_t launch_vhs_bf16x3(const Job* J, const int* ids, int g, void* const* zeta,
                                    hipStream_t s) {
  Batch<FieldArgs> F;
  Batch<VhsBfArgs> V;
  F.nprob = V.nprob = g;
  long long cf[AFQMC_MAXP], cv[AFQMC_MAXP];
  for (int q = 0; q < g; ++q) {
    const Job& j = J[ids[q]];
    const afqmc_kpt_problem& p = j.p;
    const int CP = 32 * ((p.nchol + 31) / 32);
    FieldArgs& fa = F.a[q];
    fa.W = p.nwalk; fa.nk = p.nk; fa.C = p.nchol;
    fa.mesh = make_mesh(p);
    fa.x = j.x;
    fa.xbar = (const cpx<double>*)j.xbar;
    fa.zeta = zeta[ids[q]];
    cf[q] = ((int64_t)p.nwalk * p.nk * CP + 255) / 256;
    VhsBfArgs& va = V.a[q];
    va.W = p.nwalk; va.nk = p.nk; va.m = p.m; va.C = p.nchol;
    va.tiles_m = (p.nwalk + 63) / 64;
    va.tiles_n = (p.nk * p.m * p.m + 63) / 64;
    va.mesh = make_mesh(p);
    va.zs = (const unsigned short*)zeta[ids[q]];
    va.Ls = (const unsigned short*)p.Ls;
    va.vhs = (cpx<float>*)j.vhs;
    cv[q] = (long long)p.nk * va.tiles_m * va.tiles_n;
  }
  long long gf = batch_close(F, cf), gv = batch_close(V, cv);
  if (gf < 0 || gv < 0) return hipErrorInvalidValue;
  if (gf > 0) hipLaunchKernelGGL(field_split_kernel, dim3((unsigned)gf), dim3(256), 0, s, F);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || gv == 0) return e;
  hipLaunchKernelGGL(vhs_bf16x3_kernel, dim3((unsigned)gv), dim3(256), 0, s, V);
  return hipGetLastError();
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

// Workspace of the combined field: complex values, or the BF16 split planes.
static size_t zeta_bytes(const afqmc_kpt_problem& p) {
  const size_t cp = 32 * (size_t)((p.nchol + 31) / 32);
  const size_t a = 16 * (size_t)p.nwalk * p.nk * p.nchol, b = 8 * (size_t)p.nwalk * p.nk * cp;
  return a > b ? a : b;
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
      zeta[q] = cv.take(zeta_bytes(J[q].p));
    }
    hipError_t e = for_groups(
        c, [&](int i) { return vhs_key(J[i].p); },
        [&](const int* ids, int g) -> hipError_t {
          if (J[ids[0]].p.prec == AFQMC_PREC_BF16X3) return launch_vhs_bf16x3(J, ids, g, zeta, s);
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
      zeta[q] = cv.take(zeta_bytes(J[q].p));
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
