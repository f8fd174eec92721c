// Walker propagation (symmetric propagator with the 6th-order Taylor expansion of the
// two-body exponential) and re-orthonormalisation.
//
//   T_0 = bhalf U,   T_j = (-sqrt(dt) / j) vhs T_{j-1},   U' = bhalf sum_j T_j.
//
// Each Taylor term is one batched MFMA GEMM per walker ((nk*m)^2 x nk*nocc) whose epilogue
// writes T_j and adds it into an FP64 accumulator; the one-body half steps are batched over
// (walker, k) blocks and always run in FP64.  With FP32 contractions the Taylor terms are
// computed from complex64 vhs and T_{j-1} with FP32 MFMA accumulation, while the walker
// accumulator stays complex128.  In the BF16X3 mode the Taylor terms run on the three-pass
// BF16 split of the same complex64 operands.
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

// ---------------------------------------------------------------------------
// The Taylor polynomial on the three-pass BF16 split (BF16X3 mode), in nested (Horner)
// form: with X = -sqrt(dt) vhs,
//   R_6 = T_0,  R_{j-1} = T_0 + (X / j) R_j  (j = 6 .. 1),  T6(X) T_0 = R_0,
// the same polynomial as the sum of the terms X^j T_0 / j!.  Each step is one batched
// product whose epilogue forms R_{j-1} directly: the intermediate R are only ever read as
// BF16 operands, so they are formed in FP32 from the complex64 T_0 and stored as planes;
// the last step adds X R_1 to the FP64 T_0.  The walker-side operand is kept as BF16
// planes Rp[w][k / 32][n][plane][k % 32] (planes re hi, re lo, im hi, im lo; k = row of R,
// zero for M <= k < KP = 32 ceil(M / 32)): K-contiguous for the MFMA B operand, and one
// K chunk of all columns is one contiguous block.

__host__ __device__ __forceinline__ int kpad32(int m) { return 32 * ((m + 31) / 32); }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Tp[w][k / 32][n][pl][k % 32] from T[w][k][n] (complex64), 64 k x 64 n tiles transposed
// through LDS.
struct TSplitArgs {
  int W, M, N, KP, tk, tn;  // tk = ceil(KP / 64), tn = ceil(N / 64)
  const cpx<float>* T;
  unsigned short* Tp;
};

__global__ __launch_bounds__(256) void t_split_kernel(const Batch<TSplitArgs> B) {
  __shared__ float2 tile[64][65];
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const TSplitArgs& a = B.a[pb];
  const int per_w = a.tk * a.tn;
  const int w = (int)(loc / per_w), rem = (int)(loc % per_w);
  const int k0 = (rem / a.tn) * 64, n0 = (rem % a.tn) * 64;
  const int tid = threadIdx.x;
  const cpx<float>* __restrict__ T = a.T + (int64_t)w * a.M * a.N;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int u = tid + 256 * e, kk = u >> 6, nn = u & 63;
    const int k = k0 + kk, n = n0 + nn;
    float2 v = {0.f, 0.f};
    if (k < a.M && n < a.N) {
      const cpx<float> t = T[(int64_t)k * a.N + n];
      v = float2{t.re, t.im};
    }
    tile[kk][nn] = v;
  }
  __syncthreads();
  unsigned short* __restrict__ Tp = a.Tp + (int64_t)w * a.N * 4 * a.KP;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int u = tid + 256 * e, nn = u >> 4, kq = 4 * (u & 15);
    const int n = n0 + nn, k = k0 + kq;
    if (n >= a.N || k >= a.KP) continue;
    unsigned int h0[4], h1[4];
    bf16_split2(tile[kq][nn].x, tile[kq + 1][nn].x, h0[0], h0[1]);
    bf16_split2(tile[kq][nn].y, tile[kq + 1][nn].y, h0[2], h0[3]);
    bf16_split2(tile[kq + 2][nn].x, tile[kq + 3][nn].x, h1[0], h1[1]);
    bf16_split2(tile[kq + 2][nn].y, tile[kq + 3][nn].y, h1[2], h1[3]);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      *reinterpret_cast<uint2*>(Tp + ((((int64_t)(k >> 5) * a.N + n) * 4 + pl) << 5) + (k & 31)) =
          uint2{h0[pl], h1[pl]};
  }
}

static hipError_t launch_t_split(const Job* jobs, const int* ids, int c, void* const* T,
                                 void* const* Tp, hipStream_t s) {
  Batch<TSplitArgs> Bs;
  Bs.nprob = c;
  long long cnt[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) {
    const afqmc_kpt_problem& p = jobs[ids[q]].p;
    TSplitArgs& t = Bs.a[q];
    t.W = p.nwalk; t.M = p.nk * p.m; t.N = p.nk * p.nocc; t.KP = kpad32(t.M);
    t.tk = (t.KP + 63) / 64; t.tn = (t.N + 63) / 64;
    t.T = (const cpx<float>*)T[ids[q]];
    t.Tp = (unsigned short*)Tp[ids[q]];
    cnt[q] = (long long)t.W * t.tk * t.tn;
  }
  const long long g = batch_close(Bs, cnt);
  if (g < 0) return hipErrorInvalidValue;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(t_split_kernel, dim3((unsigned)g), dim3(256), 0, s, Bs);
  return hipGetLastError();
}

// One step, R_{j-1} = T_0 + alpha vhs R_j, one workgroup per (walker, BM-row tile (64 or
// 96), column tile of 16 NB columns) with NCW consumer waves and 4 producer waves.  The
// producers (the last four waves) stream the complex64 rows of vhs (from HBM) with DEPTH
// chunks of K in flight in registers and split them into BF16 planes, and copy the chunk's
// R_j planes (from L2), into two LDS stages.  The consumers sit in a 2 x NCW/2 grid: wave
// (wm, wn) owns rows BM/2 wm .. BM/2 (wm + 1) - 1 and 16-column blocks CB wn .. CB (wn + 1)
// - 1 (CB = ceil(NB / (NCW / 2))), with 12 BF16 MFMAs per complex 16 x 16 x 32 block and
// FP32 accumulation.  One block barrier per K chunk.  In the epilogue the consumers leave
// alpha (vhs R_j) in LDS (over the stages) and all waves add T_0 to it: from complex64 into
// the planes of R_{j-1}, or, in the last step, into the FP64 accumulator that holds T_0
// (every load issued before the first store).  Workgroups of one walker are placed on one
// XCD, where its planes stay in L2.
// Producer loads are unconditional (clamped addresses, zeros selected afterwards) so that
// each wait covers exactly the oldest chunk.
struct TaylorBfArgs {
  int W, M, N, KP, tiles_m, tiles_n;  // M = K = nk*m, N = nk*nocc
  int last;                           // 1: R_0 into acc (FP64), else planes of R_{j-1}
  float alpha;                        // -sqrt(dt) / j
  const cpx<float>* V;        // [W][M][M]
  const unsigned short* Tin;  // [W][KP / 32][N][4][32] planes of R_j
  unsigned short* Tout;       // [W][KP / 32][N][4][32] planes of R_{j-1} (not last)
  const cpx<float>* T0;       // [W][M][N] T_0 as complex64 (not last)
  cpx<double>* acc;           // [W][M][N] T_0 in FP64; R_0 after the last step
};

template <int BM, int NB, bool VEC, int NCW>
__global__ __launch_bounds__(64 * NCW + 256) void taylor_bf16x3_kernel(const Batch<TaylorBfArgs> B) {
  constexpr int BN = 16 * NB, BKC = 32, RS = BKC;
  // NCW consumer waves in a 2 x NCW / 2 grid, then 4 producer waves
  constexpr int NT = 64 * NCW + 256, GM = 2, GN = NCW / GM;
  constexpr int RB = BM / (16 * GM);  // 16-row blocks per consumer wave
  static_assert(RB * 16 * GM == BM, "row tile must split evenly over the consumer rows");
  constexpr int NUA = BM / 16;      // A units per producer thread
  // chunks in flight in the producers' registers: the register budget of 3 waves per SIMD
  // leaves room for one with 8 consumer waves
  constexpr int DEPTH = NCW > 4 ? 1 : ((NB >= 6 || BM > 64) ? 2 : 3);
  constexpr int CB = (NB + GN - 1) / GN;  // 16-column blocks per consumer wave
  // B planes padded by 64 bytes: a 16-byte staging store of 16 lanes covers 4 planes x 4
  // units, and unpadded plane strides (a multiple of 256 bytes) would put them in one bank
  // group
  constexpr int PSB = BN * RS + 32;
  // 16-byte slot of the 8 k at k8 = k / 8 in row (or column) r of a stage: k8 ^ ((r / 4) % 4).
  // A fragment read takes rows r0 .. r0 + 15 at one k8 (lanes 0-15) and the next k8 in
  // each further group of 16 lanes: 64-byte rows put the 16 lanes of a group, and the four
  // lanes of equal lane % 16 across the groups, in distinct banks.
  auto sw = [](int r, int k) { return ((((k >> 3) ^ (r >> 2)) & 3) << 3) | (k & 7); };
  constexpr int SA_BYTES = 2 * 4 * BM * RS * 2, SB_BYTES = 2 * 4 * PSB * 2;
  constexpr int RST = BN + 1;  // row stride of the result tile (float2)
  constexpr int RES_BYTES = BM * RST * 8;
  constexpr int LDS_BYTES =
      SA_BYTES + SB_BYTES > RES_BYTES ? SA_BYTES + SB_BYTES : RES_BYTES;
  __shared__ __attribute__((aligned(16))) unsigned char lds[LDS_BYTES];
  auto sA = reinterpret_cast<unsigned short (*)[4][BM][RS]>(lds);
  auto sB = reinterpret_cast<unsigned short (*)[4][PSB]>(lds + SA_BYTES);
  auto res = reinterpret_cast<float2 (*)[RST]>(lds);  // after the K loop
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const TaylorBfArgs& a = B.a[pb];
  const long long per_w = (long long)a.tiles_m * a.tiles_n;
  const long long total = per_w * a.W;
  const long long lt = xcd_remap(loc, (total + 7) & ~7LL);
  if (lt >= total) return;
  const int w = (int)(lt / per_w);
  const int rem = (int)(lt % per_w);
  const int row0 = (rem / a.tiles_n) * BM, col0 = (rem % a.tiles_n) * BN;
  const int M = a.M, N = a.N, K = a.M, KP = a.KP;
  const int nch = KP / BKC;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;

  if (wave >= NCW) {
    // ---------------- producers
    const int pt = threadIdx.x - 64 * NCW;
    const cpx<float>* __restrict__ V = a.V + (int64_t)w * M * K;
    const unsigned short* __restrict__ Tp = a.Tin + (int64_t)w * N * 4 * KP;
    float4 ra[DEPTH][NUA];  // A unit e: row pt / 16 + 16 e, k pair pt % 16
    u32x4 rb[DEPTH][NB];  // B unit e: u = pt + 256 e: column u / 16, plane (u / 4) % 4,
                          // 8 k at 8 (u % 4)
    auto issue = [&](int q, float4 (&xa)[NUA], u32x4 (&xb)[NB]) {
      const int k0 = (q < nch ? q : nch - 1) * BKC;
#pragma unroll
      for (int e = 0; e < NUA; ++e) {
        const int row = min(row0 + (pt >> 4) + 16 * e, M - 1);
        const int k = k0 + 2 * (pt & 15);
        if constexpr (VEC) {
          xa[e] = *reinterpret_cast<const float4*>(V + (int64_t)row * K + min(k, K - 2));
        } else {
          const cpx<float> v0 = V[(int64_t)row * K + min(k, K - 1)];
          const cpx<float> v1 = V[(int64_t)row * K + min(k + 1, K - 1)];
          xa[e] = float4{v0.re, v0.im, v1.re, v1.im};
        }
      }
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int u = pt + 256 * e;
        const int col = min(col0 + (u >> 4), N - 1);
        xb[e] = *reinterpret_cast<const u32x4*>(
            Tp + ((((int64_t)(k0 >> 5) * N + col) * 4 + ((u >> 2) & 3)) << 5) + 8 * (u & 3));
      }
    };
    auto stash = [&](int q, int st, const float4 (&xa)[NUA], const u32x4 (&xb)[NB]) {
      const int k0 = q * BKC;
#pragma unroll
      for (int e = 0; e < NUA; ++e) {
        const int r = (pt >> 4) + 16 * e, kk = 2 * (pt & 15);
        const bool rok = row0 + r < M;
        const float4 v = xa[e];
        const bool ok0 = rok && k0 + kk < K, ok1 = rok && k0 + kk + 1 < K;
        unsigned int h[4];
        bf16_split2(ok0 ? v.x : 0.f, ok1 ? v.z : 0.f, h[0], h[1]);
        bf16_split2(ok0 ? v.y : 0.f, ok1 ? v.w : 0.f, h[2], h[3]);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
          *reinterpret_cast<unsigned int*>(&sA[st][pl][r][sw(r, kk)]) = h[pl];
      }
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int u = pt + 256 * e;
        *reinterpret_cast<u32x4*>(&sB[st][(u >> 2) & 3][(u >> 4) * RS + sw(u >> 4, 8 * (u & 3))]) = xb[e];
      }
    };
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) issue(d, ra[d], rb[d]);
    stash(0, 0, ra[0], rb[0]);
    issue(DEPTH, ra[0], rb[0]);
    __syncthreads();
    // iteration c: the consumers work on chunk c; chunk c + 1 (slot (c + 1) % DEPTH) goes
    // to stage (c + 1) & 1 and chunk c + 1 + DEPTH is requested into the freed slot.  The
    // body has no branches (past the last chunk it stores into the stage nobody reads), so
    // the compiler's wait before each store covers only the oldest chunk.
    for (int c0 = 0; c0 < nch; c0 += DEPTH) {
#pragma unroll
      for (int d = 0; d < DEPTH; ++d) {
        const int c = c0 + d;
        const int sl = (d + 1) % DEPTH;
        stash(c + 1, (c + 1) & 1, ra[sl], rb[sl]);
        issue(c + 1 + DEPTH, ra[sl], rb[sl]);
        __syncthreads();
      }
    }
  } else {
    // ---------------- consumers
    const int wm = wave / GN, wn = wave % GN;
    v4f acr[RB][CB], aci[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        acr[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        aci[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      }
    const int cb0 = wn * CB, ncb = NB - cb0 < CB ? NB - cb0 : CB;
    __syncthreads();
    // as many barriers as the producers: ceil(nch / DEPTH) DEPTH iterations
    for (int c0 = 0; c0 < nch; c0 += DEPTH) {
#pragma unroll
      for (int d = 0; d < DEPTH; ++d) {
        const int c = c0 + d;
        if (c < nch) {
          const int st = c & 1;
          const int kq = 8 * (lane >> 4);
          u16x8 fa[RB][4], fn[RB][2];
#pragma unroll
          for (int i = 0; i < RB; ++i) {
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
              fa[i][pl] = *reinterpret_cast<const u16x8*>(&sA[st][pl][wm * 16 * RB + i * 16 + (lane & 15)][sw(lane & 15, kq)]);
            fn[i][0] = bf16_neg(fa[i][2]);
            fn[i][1] = bf16_neg(fa[i][3]);
          }
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            if (j < ncb) {
              u16x8 fb[4];
#pragma unroll
              for (int pl = 0; pl < 4; ++pl)
                fb[pl] = *reinterpret_cast<const u16x8*>(&sB[st][pl][(16 * (cb0 + j) + (lane & 15)) * RS + sw(lane & 15, kq)]);
#pragma unroll
              for (int i = 0; i < RB; ++i) {
                // re += Vr Tr - Vi Ti,  im += Vr Ti + Vi Tr  (fn: -Vi)
                acr[i][j] = mul3(fa[i][0], fa[i][1], fb[0], fb[1], acr[i][j]);
                acr[i][j] = mul3(fn[i][0], fn[i][1], fb[2], fb[3], acr[i][j]);
                aci[i][j] = mul3(fa[i][0], fa[i][1], fb[2], fb[3], aci[i][j]);
                aci[i][j] = mul3(fa[i][2], fa[i][3], fb[0], fb[1], aci[i][j]);
              }
            }
          }
        }
        __syncthreads();
      }
    }
    // the stages are free: alpha T to the result tile (lane: rows 4 (lane / 16) + v of
    // column lane % 16 of each 16 x 16 block)
    const float alpha = a.alpha;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        if (j >= ncb) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          res[wm * 16 * RB + i * 16 + 4 * (lane >> 4) + v][16 * (cb0 + j) + (lane & 15)] =
              float2{alpha * acr[i][j][v], alpha * aci[i][j][v]};
      }
  }
  __syncthreads();

  // ---------------- epilogue, all waves
  const int tid = threadIdx.x;
  constexpr int NE = (BM * BN + 2 * NT - 1) / (2 * NT);  // tile entries per thread and half
  if (a.last) {
    // acc = T_0 + X R_1 (FP64), in two halves: every load of a half first, then its stores
    cpx<double>* __restrict__ acc = a.acc + (int64_t)w * M * N;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      cpx<double> av[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int u = tid + NT * (2 * e + h), row = row0 + u / BN, col = col0 + u % BN;
        const bool ok = u < BM * BN && row < M && col < N;
        av[e] = acc[ok ? (int64_t)row * N + col : 0];
      }
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int u = tid + NT * (2 * e + h), row = row0 + u / BN, col = col0 + u % BN;
        if (u < BM * BN && row < M && col < N) {
          const float2 t = res[u / BN][u % BN];
          acc[(int64_t)row * N + col] =
              cpx<double>{av[e].re + (double)t.x, av[e].im + (double)t.y};
        }
      }
    }
    return;
  }
  // R_{j-1} = T_0 + X R_j in the tile (rows past M stay zero), then its planes: four
  // consecutive rows of one column per unit
  {
    const cpx<float>* __restrict__ T0 = a.T0 + (int64_t)w * M * N;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float2 tv[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int u = tid + NT * (2 * e + h), row = row0 + u / BN, col = col0 + u % BN;
        const bool ok = u < BM * BN && row < M && col < N;
        const cpx<float> t = T0[ok ? (int64_t)row * N + col : 0];
        tv[e] = ok ? float2{t.re, t.im} : float2{0.f, 0.f};
      }
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int u = tid + NT * (2 * e + h);
        if (u < BM * BN) {
          float2& r = res[u / BN][u % BN];
          r = float2{r.x + tv[e].x, r.y + tv[e].y};
        }
      }
    }
  }
  __syncthreads();
  unsigned short* __restrict__ To = a.Tout + (int64_t)w * N * 4 * KP;
  constexpr int QPC = BM / 4;                        // row quads per column
  constexpr int NQ = (QPC * BN + NT - 1) / NT;
  static_assert(BM % 32 == 0, "row tile of whole 32-row chunks");
#pragma unroll
  for (int e = 0; e < NQ; ++e) {
    // eight consecutive units: the eight row quads of one 32-row chunk of one column (64
    // contiguous bytes of each plane; their result rows fall in distinct LDS banks), then
    // the next column
    const int u = tid + NT * e;
    const int t = u >> 3;
    const int cl = t % BN, rq = 32 * (t / BN) + 4 * (u & 7);
    const int col = col0 + cl, rb = row0 + rq;
    if (u >= QPC * BN || col >= N || rb >= KP) continue;
    const float2 t0 = res[rq][cl], t1 = res[rq + 1][cl], t2 = res[rq + 2][cl],
                 t3 = res[rq + 3][cl];
    unsigned int h0[4], h1[4];
    bf16_split2(t0.x, t1.x, h0[0], h0[1]);
    bf16_split2(t0.y, t1.y, h0[2], h0[3]);
    bf16_split2(t2.x, t3.x, h1[0], h1[1]);
    bf16_split2(t2.y, t3.y, h1[2], h1[3]);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      *reinterpret_cast<uint2*>(To + ((((int64_t)(rb >> 5) * N + col) * 4 + pl) << 5) + (rb & 31)) =
          uint2{h0[pl], h1[pl]};
  }
}

// One Horner step for a group of BF16X3 jobs: R_{j-1} = T_0 + (-sqrt(dt) / j) vhs R_j
// (planes tin -> planes tout, T_0 from t0c), or with tout null the last step into acc.
static hipError_t launch_taylor_bf16x3(const Job* jobs, const int* ids, int c, int j,
                                       const void* const* tin, void* const* tout,
                                       const void* const* t0c, void* const* acc,
                                       hipStream_t s) {
  TimedScope ts(KC_TAYLOR, s);
  Batch<TaylorBfArgs> Bt;
  Bt.nprob = c;
  int nb = 0;
  bool vec = true;
  for (int q = 0; q < c; ++q) {
    const Job& jb = jobs[ids[q]];
    TaylorBfArgs& t = Bt.a[q];
    t.W = jb.p.nwalk;
    t.M = jb.p.nk * jb.p.m;
    t.N = jb.p.nk * jb.p.nocc;
    t.KP = kpad32(t.M);
    const int nbq = (t.N + 15) / 16 < 8 ? (t.N + 15) / 16 : 8;
    if (q == 0) nb = nbq;
    if (nbq != nb) return hipErrorInvalidValue;  // one column-tile width per group
    t.tiles_n = (t.N + 16 * nb - 1) / (16 * nb);
    vec = vec && (t.M % 2 == 0) && (((uintptr_t)jb.vhs & 15) == 0);
    t.last = tout ? 0 : 1;
    t.alpha = (float)(-sqrt(jb.p.dt) / j);
    t.V = (const cpx<float>*)jb.vhs;
    t.Tin = (const unsigned short*)tin[ids[q]];
    t.Tout = tout ? (unsigned short*)tout[ids[q]] : nullptr;
    t.T0 = (const cpx<float>*)t0c[ids[q]];
    t.acc = (cpx<double>*)acc[ids[q]];
  }
  // row-tile height: 64 or 96, whichever costs less over the rounds of workgroups (one
  // workgroup per CU at a time: the LDS stages take 50-145 KB), a round costing its rows
  // plus a fixed share equal to 64 rows (the per-chunk latencies do not grow with BM)
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (ncu < 1) ncu = 1;
  auto cost = [&](int bm) {
    long long tiles = 0;
    for (int q = 0; q < c; ++q)
      tiles += (long long)Bt.a[q].W * ((Bt.a[q].M + bm - 1) / bm) * Bt.a[q].tiles_n;
    return ((tiles + ncu - 1) / ncu) * (bm + 64);
  };
  const int bm = cost(96) < cost(64) ? 96 : 64;
  long long cnt[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) {
    TaylorBfArgs& t = Bt.a[q];
    t.tiles_m = (t.M + bm - 1) / bm;
    cnt[q] = ((long long)t.W * t.tiles_m * t.tiles_n + 7) & ~7LL;
  }
  const long long g = batch_close(Bt, cnt);
  if (g < 0) return hipErrorInvalidValue;
  if (g == 0) return hipSuccess;
  // 8 consumer waves (2 x 4): two per SIMD, so one wave's LDS reads and barrier waits
  // overlap the other's MFMAs (with 4 consumers the MFMA pipe idled two thirds of the time)
  constexpr int NCWL = 8;
  const dim3 grid((unsigned)g), block(64 * NCWL + 256);
#define AFQMC_TBF(BMV, NBV)                                                              \
  if (vec) hipLaunchKernelGGL((taylor_bf16x3_kernel<BMV, NBV, true, NCWL>), grid, block, 0, s, Bt); \
  else hipLaunchKernelGGL((taylor_bf16x3_kernel<BMV, NBV, false, NCWL>), grid, block, 0, s, Bt);
#define AFQMC_TBF_NB(BMV)     \
  switch (nb) {               \
    case 1: AFQMC_TBF(BMV, 1) break; \
    case 2: AFQMC_TBF(BMV, 2) break; \
    case 3: AFQMC_TBF(BMV, 3) break; \
    case 4: AFQMC_TBF(BMV, 4) break; \
    case 5: AFQMC_TBF(BMV, 5) break; \
    case 6: AFQMC_TBF(BMV, 6) break; \
    case 7: AFQMC_TBF(BMV, 7) break; \
    default: AFQMC_TBF(BMV, 8) break; \
  }
  if (bm == 96) {
    AFQMC_TBF_NB(96)
  } else {
    AFQMC_TBF_NB(64)
  }
#undef AFQMC_TBF_NB
#undef AFQMC_TBF
  return hipGetLastError();
}

// One Taylor term, T_j = alpha vhs T_{j-1}, acc += T_j, for a group of FP64 or FP32 jobs
// of one tile class; alpha = -sqrt(dt) * alpha_scale per job.
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
                              void** t1, void** tc, GreensWs& g) {
  Dims d = dims_of(p);
  // Taylor operands: complex128 or complex64 [W][N][n]; in the BF16X3 mode they hold
  // BF16 planes [W][n][4][KP] and tc the complex64 T_0
  const bool bf = p.prec == AFQMC_PREC_BF16X3;
  const size_t tbytes = bf ? 8 * (size_t)d.W * d.n() * kpad32(d.N())
                           : (low_prec(p.prec) ? 8 : 16) * (size_t)d.W * d.N() * d.n();
  carve_greens(c, d, g);
  *acc = c.take(16 * (size_t)d.W * d.N() * d.n());
  *t0 = c.take(tbytes);
  *t1 = c.take(tbytes);
  *tc = c.take(bf ? 8 * (size_t)d.W * d.N() * d.n() : 0);
  return c.off;
}

size_t propagate_ws_bytes(const afqmc_kpt_problem& p) {
  Carve c(nullptr);
  void *a, *b, *t, *tc;
  GreensWs g;
  return carve_propagate(c, p, &a, &b, &t, &tc, g);
}

void propagate_slots(const Job& j, void** acc, void** t0, void** t1, void** tc) {
  Carve c(j.ws);
  GreensWs g;
  carve_propagate(c, j.p, acc, t0, t1, tc, g);
}

static int taylor_key(const afqmc_kpt_problem& p) { return p.prec * 16 + taylor_class(p); }

// Launch group of job i of a Taylor stage: its tile class, or a launch of its own when its
// 64 x 32 output tiles alone fill the device.
static int taylor_group(const Job* J, int i, int ncu) {
  const afqmc_kpt_problem& p = J[i].p;
  const int64_t M = (int64_t)p.nk * p.m, N = (int64_t)p.nk * p.nocc;
  return solo_key(taylor_key(p), i, (int64_t)p.nwalk * ((M + 63) / 64) * ((N + 31) / 32), ncu);
}

// U <- bhalf T6(-sqrt(dt) vhs) bhalf U for every job.
static hipError_t propagate_jobs(const Job* J, int c, hipStream_t s) {
  void *acc[AFQMC_MAXP], *t0[AFQMC_MAXP], *t1[AFQMC_MAXP], *tc[AFQMC_MAXP], *U[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) {
    propagate_slots(J[q], &acc[q], &t0[q], &t1[q], &tc[q]);
    U[q] = J[q].p.U;
  }
  const int ncu = device_cus();
  return for_groups(
      c, [&](int i) { return taylor_group(J, i, ncu); },
      [&](const int* ids, int g) -> hipError_t {
        const bool f32 = low_prec(J[ids[0]].p.prec);
        hipError_t e;
        if (J[ids[0]].p.prec == AFQMC_PREC_BF16X3) {
          // T_0 = bhalf U: acc (FP64) and tc (complex64), R_6 = T_0 as planes in t0;
          // Horner steps j = 6 .. 1 alternate between the plane buffers
          e = launch_bhalf<float>(J, ids, g, U, acc, tc, s);
          if (e == hipSuccess) e = launch_t_split(J, ids, g, tc, t0, s);
          void** rin = t0;
          void** rout = t1;
          for (int j = 6; j >= 1 && e == hipSuccess; --j) {
            e = launch_taylor_bf16x3(J, ids, g, j, rin, (j > 1) ? rout : nullptr, tc, acc, s);
            void** t = rin; rin = rout; rout = t;
          }
          if (e != hipSuccess) return e;
          return launch_bhalf<double>(J, ids, g, acc, U, nullptr, s);
        }
        // T_0 = bhalf U (FP64), acc = T_0, t0 = T_0 in the Taylor precision
        e = f32 ? launch_bhalf<float>(J, ids, g, U, acc, t0, s)
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
    void *acc[AFQMC_MAXP], *t0[AFQMC_MAXP], *t1[AFQMC_MAXP], *tc[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) propagate_slots(J[q], &acc[q], &t0[q], &t1[q], &tc[q]);
    const int ncu = device_cus();
    const hipError_t e = for_groups(
        c, [&](int i) { return taylor_group(J, i, ncu); },
        [&](const int* ids, int g) -> hipError_t {
          // the BF16X3 steps have a single variant
          if (J[ids[0]].p.prec == AFQMC_PREC_BF16X3) return hipSuccess;
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
  hipError_t e = run_greens(jobs, n, true, s, (flags & AFQMC_PROPAGATE_REDUCED_GH) != 0);
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
      e = launch_ortho_factor(J, c, S, R, s);
      if (e != hipSuccess) return e;
      e = launch_ops<64, 64, 16, 2, 2>(rm, c, s);
      if (e != hipSuccess) return e;
    }
  }
  // Gh and the log overlap of the re-orthonormalised walkers
  return run_greens(jobs, n, false, s);
}

}  // namespace afqmc
