// Batched complex GEMM core on gfx950 MFMA (16x16x4, FP64 or FP32 accumulate).
//
// C[b](BM x BN tile) = sum_k A[b](row, k) B[b](k, col): operands are reached through an
// operation functor Op that maps (batch, row, k) / (batch, k, col) to memory and owns the
// epilogue, so that each hot contraction of the k-point step (force bias, HS potential,
// Taylor terms, one-body half steps, Green's function solve, Gram matrices, half rotation)
// is one instantiation with its own index map and fused epilogue.
//
// Tiles are staged through two LDS stages of complex-interleaved elements; the next K slice
// is prefetched into registers while the MFMAs of the current one run, with one barrier per
// K slice.  Complex products take
// four real MFMAs (Dre += Are Bre - Aim Bim, Dim += Are Bim + Aim Bre).  The 1-D grid is
// remapped so that consecutive logical tiles (same batch) land on the same XCD, which keeps
// the shared operand of a batch in one L2.
#pragma once

#include "batch.h"

namespace afqmc {

// Op requirements (device, by value in kernel arguments):
//   typedef T;                        storage/compute type of the MFMA (double or float)
//   static constexpr bool A_KCONTIG;  A(row, k) contiguous along k (else along row)
//   static constexpr bool B_NCONTIG;  B(k, col) contiguous along col (else along k)
//   int M, N, K, nbatch;
//   void load_a(int b, int row, int k, T& re, T& im) const;   // 0 <= row < M, 0 <= k < K
//   void load_b(int b, int k, int col, T& re, T& im) const;   // 0 <= k < K, 0 <= col < N
//   void store(int b, int row, int col, T re, T im) const;    // 0 <= row < M, 0 <= col < N

template <class Op, int BM, int BN, int BK, int WM, int WN>
__device__ __forceinline__ void cgemm_tile(const Op& op, int b, int tm, int tn) {
  typedef typename Op::T T;
  typedef typename mfma16<T>::acc_t acc_t;
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / (WM * 16);
  constexpr int TN = BN / (WN * 16);
  constexpr int EA = (BM * BK + NT - 1) / NT;
  constexpr int EB = (BK * BN + NT - 1) / NT;
  static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile must split into 16x16 blocks");
  static_assert(BK % 4 == 0, "BK multiple of the MFMA K");

  // complex-interleaved tiles (one 8/16-byte LDS read per complex operand), two stages
  __shared__ cpx<T> sA[2][BK][BM + 1];
  __shared__ cpx<T> sB[2][BK][BN + 1];

  const int row0 = tm * BM, col0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int M = op.M, N = op.N, K = op.K;

  acc_t accr[TM][TN], acci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      accr[i][j] = mfma16<T>::zero();
      acci[i][j] = mfma16<T>::zero();
    }

  cpx<T> pa[EA], pb[EB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * NT;
      int r, kk;
      if (Op::A_KCONTIG) { r = idx / BK; kk = idx % BK; }
      else { kk = idx / BM; r = idx % BM; }
      const int row = row0 + r, k = k0 + kk;
      T re = 0, im = 0;
      if (idx < BM * BK && row < M && k < K) op.load_a(b, row, k, re, im);
      pa[e] = cpx<T>{re, im};
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * NT;
      int c, kk;
      if (Op::B_NCONTIG) { kk = idx / BN; c = idx % BN; }
      else { c = idx / BK; kk = idx % BK; }
      const int col = col0 + c, k = k0 + kk;
      T re = 0, im = 0;
      if (idx < BK * BN && col < N && k < K) op.load_b(b, k, col, re, im);
      pb[e] = cpx<T>{re, im};
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * NT;
      int r, kk;
      if (Op::A_KCONTIG) { r = idx / BK; kk = idx % BK; }
      else { kk = idx / BM; r = idx % BM; }
      if (idx < BM * BK) sA[buf][kk][r] = pa[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * NT;
      int c, kk;
      if (Op::B_NCONTIG) { kk = idx / BN; c = idx % BN; }
      else { c = idx / BK; kk = idx % BK; }
      if (idx < BK * BN) sB[buf][kk][c] = pb[e];
    }
  };

  const int rbase = wm * TM * 16 + (lane & 15);
  const int cbase = wn * TN * 16 + (lane & 15);
  const int klane = lane >> 4;

  // stage s is computed while stage s+1 is fetched into registers; one barrier per K slice
  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = (k0 + BK < K);
    if (more) fetch(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      cpx<T> a[TM], bb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = sA[buf][ks + klane][rbase + i * 16];
#pragma unroll
      for (int j = 0; j < TN; ++j) bb[j] = sB[buf][ks + klane][cbase + j * 16];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) cmfma<T>(a[i].re, a[i].im, bb[j].re, bb[j].im, accr[i][j], acci[i][j]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wm * TM * 16 + i * 16 + mfma16<T>::drow(lane, v);
        const int col = col0 + wn * TN * 16 + j * 16 + (lane & 15);
        if (row < M && col < N) op.store(b, row, col, accr[i][j][v], acci[i][j][v]);
      }
      // one 16x16 tile of the epilogue at a time (read-modify-write epilogues)
      __builtin_amdgcn_sched_barrier(0);
    }
}

// Up to AFQMC_MAXP problems (systems) in one launch: each problem's index map, its tile
// grid and the first global tile index of each problem.  Problems are enumerated in the
// order given (callers put the longest-K problems first).
template <class Op>
struct OpSet {
  Op op[AFQMC_MAXP];
  int tiles_m[AFQMC_MAXP], tiles_n[AFQMC_MAXP];
  long long first[AFQMC_MAXP + 1];
  int nprob;
};

// One problem: one workgroup per tile.  Workgroups are dealt round-robin over the 8 XCDs
// (block i on XCD i % 8); the remap gives each XCD a contiguous range of tiles, so tiles
// sharing an operand (same batch) stay in one L2.
template <class Op, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void cgemm_kernel(Op op, int tiles_m, int tiles_n) {
  const int ntiles = tiles_m * tiles_n;
  const long long total = (long long)ntiles * op.nbatch;
  const long long bid = xcd_remap(blockIdx.x, total);
  const int b = (int)(bid / ntiles);
  const int rem = (int)(bid % ntiles);
  cgemm_tile<Op, BM, BN, BK, WM, WN>(op, b, rem / tiles_n, rem % tiles_n);
}

// Several problems in one launch.  Each problem's workgroup range starts at a multiple of
// 8 and is padded to one (spare workgroups exit), so every XCD receives an equal share of
// every problem (tiles of different problems differ in K, hence in cost), and inside a
// problem the same remap as above keeps each XCD on a contiguous range of tiles.
template <class Op, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void cgemm_set_kernel(const OpSet<Op> set) {
  const long long gid = blockIdx.x;
  int p = 0;
  while (p + 1 < set.nprob && gid >= set.first[p + 1]) ++p;
  p = __builtin_amdgcn_readfirstlane(p);
  const long long loc = gid - set.first[p];
  const long long lt = xcd_remap(loc, set.first[p + 1] - set.first[p]);
  const int ntiles = set.tiles_m[p] * set.tiles_n[p];
  if (lt >= (long long)ntiles * set.op[p].nbatch) return;
  const int b = (int)(lt / ntiles);
  const int rem = (int)(lt % ntiles);
  cgemm_tile<Op, BM, BN, BK, WM, WN>(set.op[p], b, rem / set.tiles_n[p], rem % set.tiles_n[p]);
}

// Host launcher for a set of problems.
template <int BM, int BN, int BK, int WM, int WN, class Op>
hipError_t launch_cgemm_set(OpSet<Op>& set, hipStream_t s) {
  long long total = 0;
  for (int p = 0; p < set.nprob; ++p) {
    const Op& op = set.op[p];
    set.first[p] = total;
    if (op.M <= 0 || op.N <= 0 || op.K <= 0 || op.nbatch <= 0) {
      set.tiles_m[p] = set.tiles_n[p] = 1;
      set.op[p].nbatch = 0;  // no tiles: every workgroup of the (empty) range exits
      continue;
    }
    set.tiles_m[p] = (op.M + BM - 1) / BM;
    set.tiles_n[p] = (op.N + BN - 1) / BN;
    const long long t = (long long)set.tiles_m[p] * set.tiles_n[p] * op.nbatch;
    total += (t + 7) & ~7LL;
  }
  set.first[set.nprob] = total;
  if (total == 0) return hipSuccess;
  if (total > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((cgemm_set_kernel<Op, BM, BN, BK, WM, WN>), dim3((unsigned)total),
                     dim3(WM * WN * 64), 0, s, set);
  return hipGetLastError();
}

// One problem.
template <int BM, int BN, int BK, int WM, int WN, class Op>
hipError_t launch_cgemm(const Op& op, hipStream_t s) {
  if (op.M <= 0 || op.N <= 0 || op.K <= 0 || op.nbatch <= 0) return hipSuccess;
  const int tm = (op.M + BM - 1) / BM;
  const int tn = (op.N + BN - 1) / BN;
  const long long total = (long long)tm * tn * op.nbatch;
  if (total > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((cgemm_kernel<Op, BM, BN, BK, WM, WN>), dim3((unsigned)total),
                     dim3(WM * WN * 64), 0, s, op, tm, tn);
  return hipGetLastError();
}

// n <= AFQMC_MAXP problems of one stage: the single-problem kernel for one, else one set
// launch.
template <int BM, int BN, int BK, int WM, int WN, class Op>
hipError_t launch_ops(const Op* ops, int n, hipStream_t s) {
  if (n == 1) return launch_cgemm<BM, BN, BK, WM, WN>(ops[0], s);
  if (n < 1 || n > AFQMC_MAXP) return hipErrorInvalidValue;
  OpSet<Op> set;
  set.nprob = n;
  for (int i = 0; i < n; ++i) set.op[i] = ops[i];
  return launch_cgemm_set<BM, BN, BK, WM, WN>(set, s);
}

}  // namespace afqmc
