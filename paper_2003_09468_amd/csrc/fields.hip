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

// K slices of the force bias of one problem: at most 4.  At c1 the BF16X3 kernel's 432
// workgroups then fill the chip in one round, where 8 slices take 864 in 1.7 rounds (0.108
// instead of 0.135 ms); the FP64 GEMM gains 5% (0.29 instead of 0.31 ms).
static int vbias_slices(const afqmc_kpt_problem& p) { return vbias_splits(dims_of(p)); }

template <typename T>
static OpVbias<T> vbias_op(const afqmc_kpt_problem& p, void* parts) {
  OpVbias<T> op;
  op.nk = p.nk; op.m = p.m; op.nocc = p.nocc; op.C = p.nchol;
  op.S = vbias_slices(p);
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

// Split-K partial traces on the three-pass BF16 split (BF16X3 mode):
//   part[s][w][Q][g] = sum over the k of slice s of sum_{a,r} Lh[Q][k][a][r][g] Gh[w][(k a)][(k-Q) r]
// one 256-thread workgroup per (Q, slice, 64 g, 64 walkers); the K stream runs over
// (k, a, 32 r) chunks.  Lh comes as split planes Lhs[Q][k][g][a][plane][r] (r padded to
// KP with zeros); the FP64 Gh rows are rounded to FP32 and split while staged.  Two chunks
// in flight in registers (unconditional, clamped loads), two LDS stages, four waves in
// 2 x 2 (32 g x 32 walkers each, 12 BF16 MFMAs per complex 16 x 16 x 32 block).
struct VbBfArgs {
  int W, nk, m, nocc, C, KP, S, kper, tiles_g, tiles_w;
  KMesh mesh;
  const unsigned short* Lhs;  // [nk][nk][C][nocc][4][KP]
  const cpx<double>* Gh;      // [W][nk nocc][nk m]
  cpx<double>* part;          // [S][W][nk][C]
};

__global__ __launch_bounds__(256) void vbias_bf16x3_kernel(const Batch<VbBfArgs> B) {
  constexpr int BG = 64, BW = 64, RS = 32;
  // planes padded by 64 bytes (a 16-byte staging store of 16 lanes covers 4 planes x 4
  // units); the two stages take 66 KB, two workgroups per CU
  constexpr int PS = 64 * RS + 32;
  __shared__ __attribute__((aligned(16))) unsigned short sA[2][4][PS];
  __shared__ __attribute__((aligned(16))) unsigned short sB[2][4][PS];
  // 16-byte slot of the 8 k at k8 = k / 8 in row r: k8 ^ ((r / 4) % 4), so that the 16 rows
  // of a fragment read (and the four lane groups at one row) fall in distinct banks
  auto sw = [](int r, int k) { return ((((k >> 3) ^ (r >> 2)) & 3) << 3) | (k & 7); };
  // the g tiles of one (Q, slice) read the same Gh rows: consecutive tiles, which
  // xcd_remap keeps on one XCD, share them in its L2
  long long loc;
  const int pb = batch_find(B, xcd_remap(blockIdx.x, gridDim.x), loc);
  const VbBfArgs& a = B.a[pb];
  const int tw = (int)(loc % a.tiles_w);
  long long rest = loc / a.tiles_w;
  const int tg = (int)(rest % a.tiles_g);
  rest /= a.tiles_g;
  const int sl = (int)(rest % a.S), Q = (int)(rest / a.S);
  const int g0 = tg * BG, w0 = tw * BW;
  const int W = a.W, nk = a.nk, m = a.m, nocc = a.nocc, C = a.C, KP = a.KP;
  const int kb = sl * a.kper, ke = min(nk, kb + a.kper);
  const int nrc = KP / 32;
  const int nch = ke > kb ? (ke - kb) * nocc * nrc : 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t n = (int64_t)nk * nocc, Nn = (int64_t)nk * m;
  cpx<double>* __restrict__ part = a.part + (int64_t)sl * W * nk * C;
  if (nch == 0) {  // empty slice: zero partial
    for (int u = tid; u < BG * BW; u += 256) {
      const int g = g0 + (u & 63), w = w0 + (u >> 6);
      if (g < C && w < W) part[((int64_t)w * nk + Q) * C + g] = cpx<double>{0.0, 0.0};
    }
    return;
  }
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 ra[2][4];
  cpx<double> rb[2][4][2];
  // unit u = tid + 256 e: A: g = u >> 4, plane (u >> 2) & 3, 8 r at 8 (u & 3);
  // B: walker u >> 4, r pair u & 15
  auto issue = [&](int c, u4 (&xa)[4], cpx<double> (&xb)[4][2]) {
    c = c < nch ? c : nch - 1;
    const int kk = kb + c / (nocc * nrc), aa = (c / nrc) % nocc, r0 = 32 * (c % nrc);
    const int k2 = a.mesh.kmq(kk, Q);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = tid + 256 * e;
      const int g = min(g0 + (u >> 4), C - 1);
      xa[e] = *reinterpret_cast<const u4*>(
          a.Lhs + (((((int64_t)Q * nk + kk) * C + g) * nocc + aa) * 4 + ((u >> 2) & 3)) * KP +
          r0 + 8 * (u & 3));
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = tid + 256 * e;
      const int w = min(w0 + (u >> 4), W - 1);
      const int r = r0 + 2 * (u & 15);
      const cpx<double>* row = a.Gh + ((int64_t)w * n + (int64_t)kk * nocc + aa) * Nn + (int64_t)k2 * m;
      xb[e][0] = row[min(r, m - 1)];
      xb[e][1] = row[min(r + 1, m - 1)];
    }
  };
  auto stash = [&](int c, int st, const u4 (&xa)[4], const cpx<double> (&xb)[4][2]) {
    const int r0 = 32 * ((c < nch ? c : nch - 1) % nrc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = tid + 256 * e;
      *reinterpret_cast<u4*>(&sA[st][(u >> 2) & 3][(u >> 4) * RS + sw(u >> 4, 8 * (u & 3))]) = xa[e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = tid + 256 * e;
      const int r = r0 + 2 * (u & 15);
      const bool ok0 = r < m, ok1 = r + 1 < m;
      unsigned int h[4];
      bf16_split2(ok0 ? (float)xb[e][0].re : 0.f, ok1 ? (float)xb[e][1].re : 0.f, h[0], h[1]);
      bf16_split2(ok0 ? (float)xb[e][0].im : 0.f, ok1 ? (float)xb[e][1].im : 0.f, h[2], h[3]);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        *reinterpret_cast<unsigned int*>(&sB[st][pl][(u >> 4) * RS + sw(u >> 4, 2 * (u & 15))]) = h[pl];
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
  issue(0, ra[0], rb[0]);
  issue(1, ra[1], rb[1]);
  stash(0, 0, ra[0], rb[0]);
  issue(2, ra[0], rb[0]);
  __syncthreads();
  // iteration c: chunk c from stage c & 1; chunk c + 1 (slot (c + 1) & 1) to the other
  // stage; chunk c + 3 requested into the freed slot
  for (int c0 = 0; c0 < nch; c0 += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int c = c0 + d;
      if (c < nch) {
        const int st = c & 1;
        const int kq = 8 * (lane >> 4);
        u16x8 fa[2][4], fb[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int pl = 0; pl < 4; ++pl) {
            fa[i][pl] = *reinterpret_cast<const u16x8*>(
                &sA[st][pl][(wm * 32 + i * 16 + (lane & 15)) * RS + sw(lane & 15, kq)]);
            fb[i][pl] = *reinterpret_cast<const u16x8*>(
                &sB[st][pl][(wn * 32 + i * 16 + (lane & 15)) * RS + sw(lane & 15, kq)]);
          }
        const u16x8 fn[2][2] = {{bf16_neg(fa[0][2]), bf16_neg(fa[0][3])},
                                {bf16_neg(fa[1][2]), bf16_neg(fa[1][3])}};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            // re += Lr Gr - Li Gi,  im += Lr Gi + Li Gr  (fn: -Li)
            acr[i][j] = mul3(fa[i][0], fa[i][1], fb[j][0], fb[j][1], acr[i][j]);
            acr[i][j] = mul3(fn[i][0], fn[i][1], fb[j][2], fb[j][3], acr[i][j]);
            aci[i][j] = mul3(fa[i][0], fa[i][1], fb[j][2], fb[j][3], aci[i][j]);
            aci[i][j] = mul3(fa[i][2], fa[i][3], fb[j][0], fb[j][1], aci[i][j]);
          }
      }
      stash(c + 1, (c + 1) & 1, ra[(d + 1) & 1], rb[(d + 1) & 1]);
      issue(c + 3, ra[(d + 1) & 1], rb[(d + 1) & 1]);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int g = g0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int w = w0 + wn * 32 + j * 16 + (lane & 15);
        if (g < C && w < W)
          part[((int64_t)w * nk + Q) * C + g] = cpx<double>{(double)acr[i][j][v], (double)aci[i][j][v]};
      }
}

static hipError_t launch_vbias_bf16x3(const Job* jobs, const int* ids, int c, void* const* parts,
                                      hipStream_t s) {
  Batch<VbBfArgs> Bv;
  Bv.nprob = c;
  long long cnt[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) {
    const afqmc_kpt_problem& p = jobs[ids[q]].p;
    VbBfArgs& v = Bv.a[q];
    v.W = p.nwalk; v.nk = p.nk; v.m = p.m; v.nocc = p.nocc; v.C = p.nchol;
    v.KP = 32 * ((p.m + 31) / 32);
    v.S = vbias_slices(p);
    v.kper = (p.nk + v.S - 1) / v.S;
    v.tiles_g = (p.nchol + 63) / 64;
    v.tiles_w = (p.nwalk + 63) / 64;
    v.mesh = make_mesh(p);
    v.Lhs = (const unsigned short*)p.Lhs;
    v.Gh = (const cpx<double>*)p.Gh;
    v.part = (cpx<double>*)parts[ids[q]];
    cnt[q] = (long long)p.nk * v.S * v.tiles_g * v.tiles_w;
  }
  const long long g = batch_close(Bv, cnt);
  if (g < 0) return hipErrorInvalidValue;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(vbias_bf16x3_kernel, dim3((unsigned)g), dim3(256), 0, s, Bv);
  return hipGetLastError();
}

// Split-K partial traces of a group of jobs of one precision.
hipError_t launch_vbias_group(const Job* jobs, const int* ids, int c, int choice,
                              void* const* parts, hipStream_t s) {
  if (jobs[ids[0]].p.prec == AFQMC_PREC_BF16X3)
    return launch_vbias_bf16x3(jobs, ids, c, parts, s);
  if (low_prec(jobs[ids[0]].p.prec)) {
    OpVbias<float> ops[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) ops[q] = vbias_op<float>(jobs[ids[q]].p, parts[ids[q]]);
    return vbias_tiles<float>(ops, c, choice, s);
  }
  OpVbias<double> ops[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) ops[q] = vbias_op<double>(jobs[ids[q]].p, parts[ids[q]]);
  return vbias_tiles<double>(ops, c, choice, s);
}

// Launch group of job i of the force-bias contraction: its precision, or a launch of its own
// when its output tiles (W nk C entries in 64 x 32 tiles, times the K slices) alone fill
// the device.
static int vbias_group(const Job* J, int i, int ncu) {
  const afqmc_kpt_problem& p = J[i].p;
  const int64_t tiles = ((int64_t)p.nwalk * p.nk * p.nchol + 2047) / 2048;
  return solo_key(p.prec, i, tiles * vbias_splits(dims_of(p)), ncu);
}

// X (and xbar where requested) for the current Gh of every job.
hipError_t launch_cholesky_trace(const Job* jobs, int n, void* const* X, void* const* xbar,
                                 void* const* parts, hipStream_t s) {
  TimedScope ts(KC_VBIAS, s);
  const int ncu = device_cus();
  hipError_t e = for_groups(
      n, [&](int i) { return vbias_group(jobs, i, ncu); },
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
      a.S = vbias_slices(p);
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
  // two-determinant walkers: the pair's force bias from both halves' traces
  return run_spin_fields(jobs, n, s);
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
    const int ncu = device_cus();
    const hipError_t e = for_groups(
        c, [&](int i) { return vbias_group(J, i, ncu); },
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
  // zs[Q][g / 32][w][plane][g % 32]: one chunk of the walkers is one contiguous block
  unsigned short* o = zs + ((((int64_t)Q * (CP / 32) + g / 32) * W + w) * 4) * 32 + (g % 32);
  o[0] = rh;
  o[32] = rl;
  o[64] = ih;
  o[96] = il;
}

// HS potential on the three-pass BF16 split, from the half store of L:
//   vhs[w][(k p), ((k-Q) r)] = sum_g zeta[w][Q][g] L[Q][k][p][r][g]
// per Q a (W x nk m m) product with K = nchol; both operands come as split planes with g
// contiguous.  L holds one member of each time-reversal pair: the Q whose index does not
// exceed that of -Q (slots in increasing Q).  For a slot with Q != -Q the same L tile also
// gives the partner blocks, L[-Q][k-Q][r][p] = conj(L[Q][k][p][r]):
//   vhs[w][((k-Q) r), (k p)] = sum_g zeta[w][-Q][g] conj(L[Q][k][p][r][g]),
// a second product on the same B operand.  The product streams the half store once from
// HBM, so the kernel is persistent and pipelined: each 512-thread workgroup walks its tiles
// (64 walkers x 96 columns of a slot, tile index b0 + i gridDim.x over every problem of
// the batch, b0 a per-XCD regrouping of blockIdx.x) as one stream of K chunks of 32.
// Waves 4-7 produce: they keep DEPTH chunks of the operands (zeta of Q, of -Q for a paired
// slot, and L) in flight in registers and copy the oldest into one of two LDS stages;
// waves 0-3 consume, in 2 x 2 (each 32 walkers x 48 columns, 12 BF16 MFMAs per complex
// 16 x 16 x 32 block and product, FP32 accumulation) and scatter a finished tile straight
// from registers (the partner block transposed).  One block barrier per chunk; loads are
// unconditional (clamped addresses, zeros selected afterwards).
struct VhsBfArgs {
  int W, nk, m, C, CP, tiles_m, tiles_n;
  KMesh mesh;
  const unsigned short* zs;  // [nk][CP / 32][W][4][32]
  const unsigned short* Ls;  // [nq][CP / 32][nk m m][4][32], then int32 Q of each slot
  const int* slotq;          // [nq]: the Q of each slot (the tail of Ls)
  cpx<float>* vhs;           // [W][nk m][nk m]
};

// Position of a workgroup in its stream of (tile, chunk) pairs, with the tile decoded
// once when the stream reaches it (the decode takes a batch lookup and 64-bit divisions,
// too slow to repeat for every chunk).
struct VhsPos {
  long long tile;  // global tile index (past the end: decoded as the last tile)
  int chunk;
  int p, nchk, slot, Q, nQ, row0, col0;  // nQ = -Q, or -1 for a self-paired slot
};

__global__ __launch_bounds__(512) void vhs_bf16x3_kernel(const Batch<VhsBfArgs> B) {
  // 96 columns per tile: the stages of both fields and of L then fit the 160 KB of LDS
  constexpr int BM = 64, BN = 96, BKC = 32, RS = BKC, DEPTH = 2;
  constexpr int NUB = BN / 16;   // B units per producer thread
  constexpr int NJ = BN / 32;    // 16-column blocks per consumer wave
  // planes padded by 64 bytes: a 16-byte staging store of 16 lanes covers 4 planes x 4
  // units, which unpadded plane strides (multiples of 256 bytes) put in one bank group
  constexpr int PSA = BM * RS + 32, PSB = BN * RS + 32;
  // 16-byte slot of the 8 k at k8 = k / 8 in row r of a stage: k8 ^ ((r / 4) % 4).  A
  // fragment read takes rows r0 .. r0 + 15 at one k8 (lanes 0-15) and the next k8 in each
  // further group of 16 lanes: 64-byte rows put the 16 lanes of a group, and the four lanes
  // of equal lane % 16 across the groups, in distinct banks.
  auto sw = [](int r, int k) { return ((((k >> 3) ^ (r >> 2)) & 3) << 3) | (k & 7); };
  __shared__ __attribute__((aligned(16))) unsigned short sA[2][2][4][PSA];  // [stage][Q / -Q]
  __shared__ __attribute__((aligned(16))) unsigned short sB[2][4][PSB];
  const long long ntiles = B.first[B.nprob];
  const long long G = gridDim.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // first tile of this workgroup: the workgroups of one XCD take consecutive tiles at every
  // pass, so the fields of Q and -Q that neighbouring column tiles share stay in its L2
  const long long b0 = xcd_remap(blockIdx.x, G);
  if (b0 >= ntiles) return;
  auto decode = [&](long long t, VhsPos& ps) {
    ps.tile = t;
    ps.chunk = 0;
    long long loc;
    ps.p = batch_find(B, t < ntiles ? t : ntiles - 1, loc);
    const VhsBfArgs& a = B.a[ps.p];
    const int per_q = a.tiles_m * a.tiles_n;
    ps.slot = (int)(loc / per_q);
    ps.Q = a.slotq[ps.slot];
    const int nq = a.mesh.neg(ps.Q);
    ps.nQ = nq == ps.Q ? -1 : nq;
    const int rem = (int)(loc % per_q);
    ps.row0 = (rem / a.tiles_n) * BM;
    ps.col0 = (rem % a.tiles_n) * BN;
    ps.nchk = a.CP / BKC;
  };
  // the stream length of this workgroup
  long long total = 0;
  for (long long t = b0; t < ntiles; t += G) {
    long long loc;
    total += B.a[batch_find(B, t, loc)].CP / BKC;
  }
  auto advance = [&](VhsPos& ps) {
    if (++ps.chunk == ps.nchk) decode(ps.tile + G, ps);
  };

  if (wave >= 4) {
    // ---------------- producers: unit u = pt + 256 e: row / column u >> 4, plane
    // (u >> 2) & 3, 8 k at 8 (u & 3); A: 4 units per field (Q and -Q), B: NUB units
    const int pt = threadIdx.x - 256;
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4 ra[DEPTH][8], rb[DEPTH][NUB];
    VhsPos ip, sp;
    decode(b0, ip);
    sp = ip;
    long long issued = 0;
    auto issue = [&](u4 (&xa)[8], u4 (&xb)[NUB]) {
      // past the end of the stream: chunk 0 of the last tile again (never stored)
      const VhsBfArgs& a = B.a[ip.p];
      const int row0 = ip.row0, col0 = ip.col0;
      const int ncol = a.nk * a.m * a.m, CP = a.CP;
      const int k0 = (issued < total ? ip.chunk : 0) * BKC;
      const unsigned short* __restrict__ Lq = a.Ls + (int64_t)ip.slot * ncol * 4 * CP;
      const int q2 = ip.nQ >= 0 ? ip.nQ : ip.Q;  // a self-paired slot loads Q twice (unused)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int u = pt + 256 * (e & 3);
        const int Qf = e < 4 ? ip.Q : q2;
        const int w = min(row0 + (u >> 4), a.W - 1);
        xa[e] = *reinterpret_cast<const u4*>(
            a.zs + ((((int64_t)Qf * (CP / BKC) + k0 / BKC) * a.W + w) * 4 + ((u >> 2) & 3)) * BKC +
            8 * (u & 3));
      }
#pragma unroll
      for (int e = 0; e < NUB; ++e) {
        const int u = pt + 256 * e;
        const int col = min(col0 + (u >> 4), ncol - 1);
        xb[e] = *reinterpret_cast<const u4*>(
            Lq + (((int64_t)(k0 / BKC) * ncol + col) * 4 + ((u >> 2) & 3)) * BKC + 8 * (u & 3));
      }
      if (issued < total) advance(ip);
      ++issued;
    };
    auto stash = [&](int st, const u4 (&xa)[8], const u4 (&xb)[NUB]) {
      // rows past W: zeros (their loads were clamped); columns past ncol are not stored
      const VhsBfArgs& a = B.a[sp.p];
      const int row0 = sp.row0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int u = pt + 256 * (e & 3);
        const u4 z = {0u, 0u, 0u, 0u};
        *reinterpret_cast<u4*>(&sA[st][e >> 2][(u >> 2) & 3][(u >> 4) * RS + sw(u >> 4, 8 * (u & 3))]) =
            row0 + (u >> 4) < a.W ? xa[e] : z;
      }
#pragma unroll
      for (int e = 0; e < NUB; ++e) {
        const int u = pt + 256 * e;
        *reinterpret_cast<u4*>(&sB[st][(u >> 2) & 3][(u >> 4) * RS + sw(u >> 4, 8 * (u & 3))]) = xb[e];
      }
    };
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) issue(ra[d], rb[d]);
    stash(0, ra[0], rb[0]);
    advance(sp);
    issue(ra[0], rb[0]);
    __syncthreads();
    // iteration s: the consumers work on chunk s; chunk s + 1 (slot (s + 1) % DEPTH) goes
    // to stage (s + 1) & 1 and the next chunk is requested into the freed slot
    for (long long s0 = 0; s0 < total; s0 += DEPTH) {
#pragma unroll
      for (int d = 0; d < DEPTH; ++d) {
        const int sl = (d + 1) % DEPTH;
        stash((int)((s0 + d + 1) & 1), ra[sl], rb[sl]);
        if (sp.tile < ntiles) advance(sp);
        issue(ra[sl], rb[sl]);
        __syncthreads();
      }
    }
    return;
  }

  // ---------------- consumers
  const int wm = wave >> 1, wn = wave & 1;
  v4f acr[2][NJ], aci[2][NJ], bcr[2][NJ], bci[2][NJ];  // products with zeta of Q and of -Q
  auto zero = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        acr[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        aci[i][j] = acr[i][j]; bcr[i][j] = acr[i][j]; bci[i][j] = acr[i][j];
      }
  };
  zero();
  VhsPos cp;
  decode(b0, cp);
  __syncthreads();
  for (long long s0 = 0; s0 < total; s0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      if (s0 + d < total) {
        const int st = (int)((s0 + d) & 1);
        const int kq = 8 * (lane >> 4);
        const bool paired = cp.nQ >= 0;
        u16x8 fa[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int pl = 0; pl < 4; ++pl)
            fa[i][pl] = *reinterpret_cast<const u16x8*>(&sA[st][0][pl][(wm * 32 + i * 16 + (lane & 15)) * RS + sw(lane & 15, kq)]);
        const u16x8 fn[2][2] = {{bf16_neg(fa[0][2]), bf16_neg(fa[0][3])},
                                {bf16_neg(fa[1][2]), bf16_neg(fa[1][3])}};
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          u16x8 fb[4];
#pragma unroll
          for (int pl = 0; pl < 4; ++pl)
            fb[pl] = *reinterpret_cast<const u16x8*>(&sB[st][pl][(wn * (BN / 2) + j * 16 + (lane & 15)) * RS + sw(lane & 15, kq)]);
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            // re += Zr Lr - Zi Li,  im += Zr Li + Zi Lr  (fn: -Zi)
            acr[i][j] = mul3(fa[i][0], fa[i][1], fb[0], fb[1], acr[i][j]);
            acr[i][j] = mul3(fn[i][0], fn[i][1], fb[2], fb[3], acr[i][j]);
            aci[i][j] = mul3(fa[i][0], fa[i][1], fb[2], fb[3], aci[i][j]);
            aci[i][j] = mul3(fa[i][2], fa[i][3], fb[0], fb[1], aci[i][j]);
          }
        }
        if (paired) {
          // with conj(L): re += Zr Lr + Zi Li,  im += Zi Lr - Zr Li
          u16x8 ga[2][4];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
              ga[i][pl] = *reinterpret_cast<const u16x8*>(&sA[st][1][pl][(wm * 32 + i * 16 + (lane & 15)) * RS + sw(lane & 15, kq)]);
          const u16x8 gn[2][2] = {{bf16_neg(ga[0][0]), bf16_neg(ga[0][1])},
                                  {bf16_neg(ga[1][0]), bf16_neg(ga[1][1])}};
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            u16x8 fb[4];
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
              fb[pl] = *reinterpret_cast<const u16x8*>(&sB[st][pl][(wn * (BN / 2) + j * 16 + (lane & 15)) * RS + sw(lane & 15, kq)]);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              bcr[i][j] = mul3(ga[i][0], ga[i][1], fb[0], fb[1], bcr[i][j]);
              bcr[i][j] = mul3(ga[i][2], ga[i][3], fb[2], fb[3], bcr[i][j]);
              bci[i][j] = mul3(ga[i][2], ga[i][3], fb[0], fb[1], bci[i][j]);
              bci[i][j] = mul3(gn[i][0], gn[i][1], fb[2], fb[3], bci[i][j]);
            }
          }
        }
        if (cp.chunk + 1 == cp.nchk) {
          // tile done: column (k p r) of Q to vhs[w][(k p)][((k - Q) r)], and for a paired
          // slot the partner product to vhs[w][((k - Q) r)][(k p)]
          const VhsBfArgs& a = B.a[cp.p];
          const int Q = cp.Q, row0 = cp.row0, col0 = cp.col0;
          const int m = a.m, mm = m * m, ncol = a.nk * mm;
          const int64_t Nn = (int64_t)a.nk * m;
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int col = col0 + wn * (BN / 2) + j * 16 + (lane & 15);
            if (col >= ncol) continue;
            const int kp = col / mm, pr = col % mm;
            const int pp = pr / m, r = pr % m;
            const int kq = a.mesh.kmq(kp, Q);
            const int64_t off = ((int64_t)kp * m + pp) * Nn + (int64_t)kq * m + r;
            const int64_t offt = ((int64_t)kq * m + r) * Nn + (int64_t)kp * m + pp;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int w = row0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
                if (w < a.W) {
                  a.vhs[(int64_t)w * Nn * Nn + off] = cpx<float>{acr[i][j][v], aci[i][j][v]};
                  if (paired)
                    a.vhs[(int64_t)w * Nn * Nn + offt] = cpx<float>{bcr[i][j][v], bci[i][j][v]};
                }
              }
          }
          zero();
        }
        advance(cp);
      }
      __syncthreads();
    }
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
    va.W = p.nwalk; va.nk = p.nk; va.m = p.m; va.C = p.nchol; va.CP = CP;
    va.tiles_m = (p.nwalk + 63) / 64;
    va.tiles_n = (p.nk * p.m * p.m + 95) / 96;
    va.mesh = make_mesh(p);
    va.zs = (const unsigned short*)zeta[ids[q]];
    va.Ls = (const unsigned short*)p.Ls;
    va.slotq = (const int*)((const char*)p.Ls + ls_plane_bytes(p));
    va.vhs = (cpx<float>*)j.vhs;
    cv[q] = (long long)ls_slots(p) * va.tiles_m * va.tiles_n;  // tiles
  }
  long long gf = batch_close(F, cf), gv = batch_close(V, cv);
  if (gf < 0 || gv < 0) return hipErrorInvalidValue;
  if (gf > 0) hipLaunchKernelGGL(field_split_kernel, dim3((unsigned)gf), dim3(256), 0, s, F);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || gv == 0) return e;
  // persistent: one workgroup per CU (the LDS stages take 145 KB), at most one per tile
  int dev = 0, ncu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const long long grid = gv < ncu ? gv : ncu;
  hipLaunchKernelGGL(vhs_bf16x3_kernel, dim3((unsigned)grid), dim3(512), 0, s, V);
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

// Launch group of job i of the HS potential: its key, or a launch of its own when its
// 64 x 64 output tiles (W nk^2 m^2 entries) alone fill the device.
static int vhs_group(const Job* J, int i, int ncu) {
  const afqmc_kpt_problem& p = J[i].p;
  const int64_t ent = (int64_t)p.nwalk * p.nk * p.nk * p.m * p.m;
  return solo_key(vhs_key(p), i, (ent + 4095) / 4096, ncu);
}

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
    const int ncu = device_cus();
    hipError_t e = for_groups(
        c, [&](int i) { return vhs_group(J, i, ncu); },
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
    const int ncu = device_cus();
    const hipError_t e = for_groups(
        c, [&](int i) { return vhs_group(J, i, ncu); },
        [&](const int* ids, int g) -> hipError_t {
          // the BF16X3 HS potential has a single variant
          if (J[ids[0]].p.prec == AFQMC_PREC_BF16X3) return hipSuccess;
          return tune_group(
              TS_VHS, J, ids, g, [&](int ch) { return launch_vhs_group(J, ids, g, ch, zeta, s); },
              s);
        });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace afqmc
