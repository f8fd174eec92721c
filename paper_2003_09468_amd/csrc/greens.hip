// Overlap, Green's function and walker weights (FP64 on gfx950).
//
// Green's-function equations of the standard representation, blocked by the trial's
// k structure: O = A^H U (nk*nocc square), log det O, Gh = (U O^{-1})^T.
//
// The overlap O is a batched MFMA GEMM over (walker, k); its inverse and log determinant
// come from a Gauss-Jordan elimination with implicit row pivoting, one workgroup per
// walker: register-resident on FP64 MFMA tiles for nk*nocc <= 112, L2-resident in panels
// of 16 up to 256.  The solve Gh = O^{-T} U^T is a batched MFMA GEMM.  The Cholesky factor
// of the re-orthonormalisation's Gram matrix and the inverse of that factor are formed
// in LDS (nk*nocc <= 128) or L2-resident, one workgroup per walker.
#include <math.h>

#include "cgemm.h"
#include "internal.h"

namespace afqmc {

#define AFQMC_PI 3.14159265358979323846

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion of the overlap matrix for n <= 256: one 256-thread
// workgroup per walker, the matrix updated in place in global memory (L2 resident).
//
// Pivoting is implicit: the pivot of column j is the unused physical row q_j of largest
// modulus, and rows are never exchanged.  With T the product of the elimination steps,
// T O = P where P[:, j] = e_{q_j}; the in-place storage keeps T[:, q_k] in column k, so
// O^{-1}[j][q_k] = M[q_j][k] at the end, and det O = sign(j -> q_j) prod_j pivot_j.
//
// Columns go in panels of 16.  Each thread owns one physical row of the panel in
// registers and applies the 16 elimination steps to it (pivot row broadcast through LDS,
// pivot choice by a block-wide max of (|a|^2, row) keys).  The combined effect of the
// steps on every other column is the rank-16 update
//   M[:, rest] += Z M[Q, rest],   Z = panel after the steps - E_Q,  E_Q[q_j][j] = 1,
// computed on FP64 MFMA 16x16x4 tiles with Z and the pivot rows staged in LDS.
struct GjbArgs {
  int n;
  cpx<double>* M;       // [W][n][n] overlap matrix, destroyed
  cpx<double>* out;     // [W][n][n] O^{-T}
  cpx<double>* logdet;  // [W]
  int* status;          // [W]
};

constexpr int GJB_NMAX = 256;

template <int NR>
__device__ __forceinline__ double pick16(const double (&a)[NR], int j) {
  double v = 0.0;
#pragma unroll
  for (int c = 0; c < NR; ++c)
    if (c == j) v = a[c];
  return v;
}

__global__ __launch_bounds__(256) void gj_blocked_kernel(const Batch<GjbArgs> B) {
  long long wloc;
  const int pb = batch_find(B, blockIdx.x, wloc);
  const int n = B.a[pb].n;
  const int w = (int)wloc;
  cpx<double>* __restrict__ M = B.a[pb].M + (int64_t)w * n * n;
  cpx<double>* __restrict__ out = B.a[pb].out + (int64_t)w * n * n;

  __shared__ double Zr[GJB_NMAX][17], Zi[GJB_NMAX][17];
  __shared__ double Rr[16][GJB_NMAX + 1], Ri[16][GJB_NMAX + 1];
  __shared__ double rowr[2][16], rowi[2][16];
  __shared__ unsigned long long red[2][4];
  __shared__ int qs[GJB_NMAX];
  __shared__ double pvr[GJB_NMAX], pvi[GJB_NMAX];
  __shared__ unsigned char vis[GJB_NMAX];
  __shared__ double lsum[2][4];
  __shared__ int flag_s;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = tid;  // physical row owned in the panel steps
  const int np = (n + 15) & ~15, ntile = np >> 4;
  bool used = false;
  int bad = 0;
  if (tid == 0) flag_s = 0;

  for (int j0 = 0; j0 < n; j0 += 16) {
    const int bw = (n - j0 < 16) ? n - j0 : 16;
    double pr[16], pi[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      cpx<double> v{0.0, 0.0};
      if (r < n && c < bw) v = M[(int64_t)r * n + j0 + c];
      pr[c] = v.re;
      pi[c] = v.im;
    }
    int jq = -1;
    for (int jj = 0; jj < bw; ++jj) {
      const int buf = jj & 1;
      unsigned long long key = 0ull;
      if (r < n && !used) {
        const double ar = pick16(pr, jj), ai = pick16(pi, jj);
        const double a2 = ar * ar + ai * ai;
        key = ((unsigned long long)__double_as_longlong(a2) & ~0xffull) |
              (unsigned long long)(255 - r);
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        key = (o > key) ? o : key;
      }
      if (lane == 0) red[buf][wave] = key;
      __syncthreads();
      key = red[buf][0];
#pragma unroll
      for (int v = 1; v < 4; ++v) key = (red[buf][v] > key) ? red[buf][v] : key;
      const int q = 255 - (int)(key & 0xffull);
      if (r == q) {
#pragma unroll
        for (int c = 0; c < 16; ++c) { rowr[buf][c] = pr[c]; rowi[buf][c] = pi[c]; }
        used = true;
        jq = jj;
      }
      __syncthreads();
      double vr = rowr[buf][jj], vi = rowi[buf][jj];
      double den = vr * vr + vi * vi;
      if (tid == 0) { qs[j0 + jj] = q; pvr[j0 + jj] = vr; pvi[j0 + jj] = vi; }
      if (!(den > 0.0) || !isfinite(den)) {
        bad |= isfinite(den) ? 1 : 2;
        vr = 1.0; vi = 0.0; den = 1.0;
      }
      const double inv = 1.0 / den, ir = vr * inv, ii = -vi * inv;  // 1 / pivot
      if (r == q) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const double xr = pr[c], xi = pi[c];
          pr[c] = (c == jj) ? ir : xr * ir - xi * ii;
          pi[c] = (c == jj) ? ii : xr * ii + xi * ir;
        }
      } else if (r < n) {
        const double fr = pick16(pr, jj), fi = pick16(pi, jj);
        const double gr = fr * ir - fi * ii, gi = fr * ii + fi * ir;  // a_rj / pivot
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const double br = rowr[buf][c], bi = rowi[buf][c];
          const double ur = pr[c] - (gr * br - gi * bi), ui = pi[c] - (gr * bi + gi * br);
          pr[c] = (c == jj) ? -gr : ur;
          pi[c] = (c == jj) ? -gi : ui;
        }
      }
    }
    // the panel's columns of T back to memory; Z = panel - E_Q to LDS
    if (r < n) {
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < bw) M[(int64_t)r * n + j0 + c] = cpx<double>{pr[c], pi[c]};
    }
    if (r < np) {
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const bool on = (r < n) && (c < bw);
        Zr[r][c] = on ? pr[c] - ((c == jq) ? 1.0 : 0.0) : 0.0;
        Zi[r][c] = on ? pi[c] : 0.0;
      }
    }
    __syncthreads();
    // pivot rows M[q_k][:] of this panel (values before the update) to LDS
    for (int idx = tid; idx < 16 * np; idx += 256) {
      const int kk = idx / np, c = idx % np;
      cpx<double> v{0.0, 0.0};
      if (kk < bw && c < n && (c < j0 || c >= j0 + 16)) v = M[(int64_t)qs[j0 + kk] * n + c];
      Rr[kk][c] = v.re;
      Ri[kk][c] = v.im;
    }
    __syncthreads();
    // M[:, rest] += Z M[Q, rest] on 16x16 tiles, K = 16
    const int Jp = j0 >> 4;
    for (int t = wave; t < ntile * ntile; t += 4) {
      const int I = t / ntile, J = t % ntile;
      if (J == Jp) continue;
      v4d cr, ci;
      const int col = J * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = I * 16 + mfma16<double>::drow(lane, v);
        cpx<double> x{0.0, 0.0};
        if (row < n && col < n) x = M[(int64_t)row * n + col];
        cr[v] = x.re;
        ci[v] = x.im;
      }
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int k = kb * 4 + (lane >> 4);
        const int arow = I * 16 + (lane & 15);
        cmfma<double>(Zr[arow][k], Zi[arow][k], Rr[k][col], Ri[k][col], cr, ci);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = I * 16 + mfma16<double>::drow(lane, v);
        if (row < n && col < n) M[(int64_t)row * n + col] = cpx<double>{cr[v], ci[v]};
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(&flag_s, bad);

  // log det = sum_j log(pivot_j) + i pi [sign of j -> q_j]
  double lr = 0.0, li = 0.0;
  for (int j = tid; j < n; j += 256) {
    const double pr = pvr[j], pim = pvi[j];
    lr += 0.5 * log(pr * pr + pim * pim);
    li += atan2(pim, pr);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    lr += __shfl_xor(lr, off, 64);
    li += __shfl_xor(li, off, 64);
  }
  if (lane == 0) { lsum[0][wave] = lr; lsum[1][wave] = li; }
  for (int j = tid; j < n; j += 256) vis[j] = 0;
  __syncthreads();
  const int fl = flag_s;
  if (tid == 0) {
    // parity of the permutation: n minus the number of cycles
    int cycles = 0;
    for (int j = 0; j < n; ++j) {
      if (vis[j]) continue;
      ++cycles;
      for (int x = j; !vis[x]; x = qs[x]) vis[x] = 1;
    }
    const double ldr = lsum[0][0] + lsum[0][1] + lsum[0][2] + lsum[0][3];
    double ldi = lsum[1][0] + lsum[1][1] + lsum[1][2] + lsum[1][3];
    if ((n - cycles) & 1) ldi += AFQMC_PI;
    double wi = remainder(ldi, 2.0 * AFQMC_PI);
    if (wi <= -AFQMC_PI) wi += 2.0 * AFQMC_PI;
    B.a[pb].logdet[w] = fl ? cpx<double>{0.0, 0.0} : cpx<double>{ldr, wi};
    if (fl) {
      int bits = 0;
      if (fl & 1) bits |= AFQMC_WALKER_SINGULAR;
      if (fl & 2) bits |= AFQMC_WALKER_NONFINITE;
      B.a[pb].status[w] |= bits;
    }
  }
  // O^{-T}[q_k][j] = O^{-1}[j][q_k] = M[q_j][k]  (0 for a degenerate walker)
  for (int idx = tid; idx < n * n; idx += 256) {
    const int j = idx / n, k = idx % n;
    const cpx<double> v = fl ? cpx<double>{0.0, 0.0} : M[(int64_t)qs[j] * n + k];
    out[(int64_t)qs[k] * n + j] = v;
  }
}

// ---------------------------------------------------------------------------
// The same elimination for n <= 128 with the matrix resident in registers: 512 threads;
// waves 1..7 own the 16x16 tiles of the matrix as FP64 MFMA accumulators for the whole
// elimination, wave 0 eliminates each 16-column panel alone (two rows per lane, no block
// barrier inside a panel): the pivot is a max over (|a|^2, row) keys by DPP lane
// exchanges within rows of 16 lanes and readlane across rows, and the pivot row is
// broadcast by readlane.  Per panel: the owners of the panel's tile column stage it in
// LDS, wave 0 eliminates it, the owners stage the pivot rows M[Q, :] (values before the
// update), and every owner applies M += Z M[Q, :] to its tiles (Z = panel - E_Q, formed
// on the fly from the staged panel).  The inverse is written from the tiles with the
// pivot permutation undone.
template <int CTRL>
__device__ __forceinline__ unsigned long long key_max_dpp(unsigned long long v) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(v >> 32), CTRL, 0xf, 0xf, false);
  const unsigned long long o = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
  return o > v ? o : v;
}

__device__ __forceinline__ unsigned long long key_readlane(unsigned long long v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ double dbl_readlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int TPW>
__global__ __launch_bounds__(512) void gj_reg_kernel(const Batch<GjbArgs> B) {
  constexpr int PW = 8;  // panel width
  long long wloc;
  const int pb = batch_find(B, blockIdx.x, wloc);
  const int n = B.a[pb].n;
  const int w = (int)wloc;
  const cpx<double>* __restrict__ S = B.a[pb].M + (int64_t)w * n * n;
  cpx<double>* __restrict__ out = B.a[pb].out + (int64_t)w * n * n;

  // two panel buffers: the panel being applied (its T columns) and the next one, which
  // wave 0 eliminates while the owners finish applying the current one
  __shared__ double Pr[2][128][PW + 1], Pi[2][128][PW + 1];
  __shared__ double Rr[PW][129], Ri[PW][129];  // pivot rows of the panel being applied
  __shared__ int qs[128], stamp[128], jpos[128];
  __shared__ double pvr[128], pvi[128];
  __shared__ unsigned char vis[128];
  __shared__ int flag_s;
  __shared__ int staged;  // owners that have staged the next panel (monotone count)

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ntile = (n + 15) >> 4;
  const int col16 = lane & 15;
  // tile i of owner wave (1..7): linear index t = (wave - 1) + 7 i over the ntile^2 tiles;
  // row I = t / ntile, column J = t % ntile, skewed by I when ntile = 7 so that the tiles
  // of one column belong to different owners
  auto tile_ij = [&](int i, int& I, int& J) {
    const int t = (wave - 1) + 7 * i;
    I = t / ntile;
    const int jj = t % ntile;
    J = (ntile == 7) ? (jj - I + 7) % 7 : jj;
    return t < ntile * ntile;
  };

  double cr[TPW][4], ci[TPW][4];
  if (wave > 0) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      int I, J;
      const bool ok = tile_ij(i, I, J);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = I * 16 + mfma16<double>::drow(lane, v), col = J * 16 + col16;
        cpx<double> x{0.0, 0.0};
        if (ok && row < n && col < n) x = S[(int64_t)row * n + col];
        cr[i][v] = x.re;
        ci[i][v] = x.im;
      }
    }
  }
  for (int i = tid; i < 128; i += 512) { stamp[i] = -1; jpos[i] = 0; }
  for (int i = tid; i < PW * 129; i += 512) { (&Rr[0][0])[i] = 0.0; (&Ri[0][0])[i] = 0.0; }
  if (tid == 0) { flag_s = 0; staged = 0; }
  bool used0 = false, used1 = false;  // wave 0: rows lane and lane + 64
  int bad = 0;

  // owners: the columns j1 .. j1 + PW - 1 of their tiles to panel buffer pbuf
  auto stage_panel = [&](int j1, int pbuf) {
    const int Jq = j1 >> 4, cq = j1 & 15;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      int I, J;
      if (!tile_ij(i, I, J) || J != Jq) continue;
      const int c = col16 - cq;
      if (c < 0 || c >= PW) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = I * 16 + mfma16<double>::drow(lane, v);
        if (row < n) { Pr[pbuf][row][c] = cr[i][v]; Pi[pbuf][row][c] = ci[i][v]; }
      }
    }
  };

  // wave 0: eliminates the panel at j1 in buffer pbuf (two rows per lane in the registers of
  // its unused tile arrays), writes its T columns back and records the pivots
  auto factor = [&](int j1, int pbuf) {
    const int bw = (n - j1 < PW) ? n - j1 : PW;
    double sar[2][PW], sai[2][PW];
    auto AR = [&](int sl, int c) -> double& {
      if constexpr (TPW >= 4) return cr[(sl * PW + c) >> 2][(sl * PW + c) & 3];
      else return sar[sl][c];
    };
    auto AI = [&](int sl, int c) -> double& {
      if constexpr (TPW >= 4) return ci[(sl * PW + c) >> 2][(sl * PW + c) & 3];
      else return sai[sl][c];
    };
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int r = lane + 64 * sl;
#pragma unroll
      for (int c = 0; c < PW; ++c) {
        AR(sl, c) = (r < n) ? Pr[pbuf][r][c] : 0.0;
        AI(sl, c) = (r < n) ? Pi[pbuf][r][c] : 0.0;
      }
    }
#pragma unroll
    for (int jj = 0; jj < PW; ++jj) {
      if (jj < bw) {
        unsigned long long key = 0ull;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int r = lane + 64 * sl;
          const bool u = sl ? used1 : used0;
          if (r < n && !u) {
            const double a2 = AR(sl, jj) * AR(sl, jj) + AI(sl, jj) * AI(sl, jj);
            const unsigned long long k2 =
                ((unsigned long long)__double_as_longlong(a2) & ~0xffull) |
                (unsigned long long)(255 - r);
            key = (k2 > key) ? k2 : key;
          }
        }
        key = key_max_dpp<0xB1>(key);   // quad_perm [1,0,3,2]
        key = key_max_dpp<0x4E>(key);   // quad_perm [2,3,0,1]
        key = key_max_dpp<0x141>(key);  // row_half_mirror
        key = key_max_dpp<0x140>(key);  // row_mirror
        unsigned long long kmax = key_readlane(key, 0);
#pragma unroll
        for (int rr = 1; rr < 4; ++rr) {
          const unsigned long long o = key_readlane(key, 16 * rr);
          kmax = (o > kmax) ? o : kmax;
        }
        const int q = 255 - (int)(kmax & 0xffull);
        const int ql = q & 63, qsl = q >> 6;
        // the pivot row by readlane from the lane that holds it (qsl is wave-uniform: a
        // branch, not a select per value)
        double br[PW], bi[PW];
        if (qsl) {
#pragma unroll
          for (int c = 0; c < PW; ++c) {
            br[c] = dbl_readlane(AR(1, c), ql);
            bi[c] = dbl_readlane(AI(1, c), ql);
          }
        } else {
#pragma unroll
          for (int c = 0; c < PW; ++c) {
            br[c] = dbl_readlane(AR(0, c), ql);
            bi[c] = dbl_readlane(AI(0, c), ql);
          }
        }
        double vr = br[jj], vi = bi[jj];
        double den = vr * vr + vi * vi;
        if (lane == 0) {
          qs[j1 + jj] = q; pvr[j1 + jj] = vr; pvi[j1 + jj] = vi; stamp[q] = j1; jpos[q] = jj;
        }
        if (!(den > 0.0) || !isfinite(den)) {
          bad |= isfinite(den) ? 1 : 2;
          vr = 1.0; vi = 0.0; den = 1.0;
        }
        const double inv = 1.0 / den, ir = vr * inv, ii = -vi * inv;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int r = lane + 64 * sl;
          if (r >= n) continue;
          if (r == q) {
            if (sl) used1 = true; else used0 = true;
#pragma unroll
            for (int c = 0; c < PW; ++c) {
              const double xr = AR(sl, c), xi = AI(sl, c);
              AR(sl, c) = (c == jj) ? ir : xr * ir - xi * ii;
              AI(sl, c) = (c == jj) ? ii : xr * ii + xi * ir;
            }
          } else {
            const double fr = AR(sl, jj), fi = AI(sl, jj);
            const double gr = fr * ir - fi * ii, gi = fr * ii + fi * ir;
#pragma unroll
            for (int c = 0; c < PW; ++c) {
              // a - g b as two fused steps per component
              const double ur = fma(-gr, br[c], fma(gi, bi[c], AR(sl, c)));
              const double ui = fma(-gr, bi[c], fma(-gi, br[c], AI(sl, c)));
              AR(sl, c) = (c == jj) ? -gr : ur;
              AI(sl, c) = (c == jj) ? -gi : ui;
            }
          }
        }
      }
    }
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int r = lane + 64 * sl;
      if (r < n) {
#pragma unroll
        for (int c = 0; c < PW; ++c) { Pr[pbuf][r][c] = AR(sl, c); Pi[pbuf][r][c] = AI(sl, c); }
      }
    }
  };

  // owners: M += Z M[Q, :] on tile i (K = PW) for the panel at j0 (buffer pbuf); the
  // panel's own columns take T
  auto update = [&](int i, int j0, int pbuf) {
    const int bw = (n - j0 < PW) ? n - j0 : PW;
    const int Jp = j0 >> 4, c0 = j0 & 15;
    int I, J;
    if (!tile_ij(i, I, J)) return;
    v4d ur, ui;
#pragma unroll
    for (int v = 0; v < 4; ++v) { ur[v] = cr[i][v]; ui[v] = ci[i][v]; }
    const int arow = I * 16 + col16;
#pragma unroll
    for (int kb = 0; kb < PW / 4; ++kb) {
      const int k = kb * 4 + (lane >> 4);
      double zr = 0.0, zi = 0.0;
      if (arow < n && k < bw) {
        zr = Pr[pbuf][arow][k] - ((qs[j0 + k] == arow) ? 1.0 : 0.0);
        zi = Pi[pbuf][arow][k];
      }
      cmfma<double>(zr, zi, Rr[k][J * 16 + col16], Ri[k][J * 16 + col16], ur, ui);
    }
    const int c = col16 - c0;
    const bool inpanel = (J == Jp) && c >= 0 && c < PW;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = I * 16 + mfma16<double>::drow(lane, v);
      const bool ok = inpanel && row < n && c < bw;
      cr[i][v] = inpanel ? (ok ? Pr[pbuf][row][c] : 0.0) : ur[v];
      ci[i][v] = inpanel ? (ok ? Pi[pbuf][row][c] : 0.0) : ui[v];
    }
  };

  __syncthreads();
  // the first panel: staged by its owners, eliminated by wave 0
  if (wave > 0) stage_panel(0, 0);
  __syncthreads();
  if (wave == 0) factor(0, 0);
  __syncthreads();

  int np = 0;
  for (int j0 = 0; j0 < n; j0 += PW, ++np) {
    const int pbuf = np & 1;
    const bool next = j0 + PW < n;
    const int Jn = (j0 + PW) >> 4;
    // (1) pivot rows M[Q, :] of this panel, before its update
    if (wave > 0) {
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        int I, J;
        if (!tile_ij(i, I, J)) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = I * 16 + mfma16<double>::drow(lane, v);
          if (row < n && stamp[row] == j0) {
            Rr[jpos[row]][J * 16 + col16] = cr[i][v];
            Ri[jpos[row]][J * 16 + col16] = ci[i][v];
          }
        }
      }
    }
    __syncthreads();
    if (wave > 0) {
      // (2) the tiles that hold the next panel first, then that panel to the other buffer
      if (next) {
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          int I, J;
          if (tile_ij(i, I, J) && J == Jn) update(i, j0, pbuf);
        }
        stage_panel(j0 + PW, pbuf ^ 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) __hip_atomic_fetch_add(&staged, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      // (3) every other tile, while wave 0 eliminates the next panel
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        int I, J;
        if (tile_ij(i, I, J) && (!next || J != Jn)) update(i, j0, pbuf);
      }
    } else if (next) {
      // wait for the seven owners (a bounded wait: past the bound the walker is flagged and
      // the elimination goes on, so the workgroup always finishes)
      const int target = 7 * (np + 1);
      int it = 0;
      while (__hip_atomic_load(&staged, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
        if (++it > (1 << 22)) { bad |= 2; break; }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      factor(j0 + PW, pbuf ^ 1);
    }
    __syncthreads();
  }
  if (wave == 0 && bad) atomicOr(&flag_s, bad);
  __syncthreads();
  const int fl = flag_s;
  // O^{-T}[q_k][j] = M[q_j][k], with j = stamp[q_j] + jpos[q_j]
  if (wave > 0) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      int I, J;
      if (!tile_ij(i, I, J)) continue;
      const int col = J * 16 + col16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = I * 16 + mfma16<double>::drow(lane, v);
        if (row < n && col < n) {
          const int j = stamp[row] + jpos[row];
          out[(int64_t)qs[col] * n + j] = fl ? cpx<double>{0.0, 0.0} : cpx<double>{cr[i][v], ci[i][v]};
        }
      }
    }
  } else {
    // log det = sum_j log(pivot_j) + i pi [sign of j -> q_j]: the logarithms by the lanes
    // of wave 0, the permutation's cycles by lane 0
    double lr = 0.0, li = 0.0;
    for (int j = lane; j < n; j += 64) {
      lr += 0.5 * log(pvr[j] * pvr[j] + pvi[j] * pvi[j]);
      li += atan2(pvi[j], pvr[j]);
      vis[j] = 0;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      lr += __shfl_xor(lr, off, 64);
      li += __shfl_xor(li, off, 64);
    }
    if (lane == 0) {
      int cycles = 0;
      for (int j = 0; j < n; ++j) {
        if (vis[j]) continue;
        ++cycles;
        for (int x = j; !vis[x]; x = qs[x]) vis[x] = 1;
      }
      if ((n - cycles) & 1) li += AFQMC_PI;
      double wi = remainder(li, 2.0 * AFQMC_PI);
      if (wi <= -AFQMC_PI) wi += 2.0 * AFQMC_PI;
      B.a[pb].logdet[w] = fl ? cpx<double>{0.0, 0.0} : cpx<double>{lr, wi};
      if (fl) {
        int bits = 0;
        if (fl & 1) bits |= AFQMC_WALKER_SINGULAR;
        if (fl & 2) bits |= AFQMC_WALKER_NONFINITE;
        B.a[pb].status[w] |= bits;
      }
    }
  }
}

hipError_t launch_gj_blocked(const Job* jobs, int n, void* const* S, void* const* out,
                             void* const* logdet_out, hipStream_t s) {
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    Batch<GjbArgs> B;
    B.nprob = c;
    long long cnt[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const afqmc_kpt_problem& p = jobs[c0 + q].p;
      B.a[q].n = p.nk * p.nocc;
      if (B.a[q].n > GJB_NMAX) return hipErrorInvalidValue;
      B.a[q].M = (cpx<double>*)S[c0 + q];
      B.a[q].out = (cpx<double>*)out[c0 + q];
      B.a[q].logdet = (cpx<double>*)logdet_out[c0 + q];
      B.a[q].status = p.status;
      cnt[q] = p.nwalk;
    }
    const long long g = batch_close(B, cnt);
    if (g < 0) return hipErrorInvalidValue;
    if (g == 0) continue;
    int nmax = 0;
    for (int q = 0; q < c; ++q) nmax = B.a[q].n > nmax ? B.a[q].n : nmax;
    // tiles per owner wave: ceil(ntile^2 / 7)
    const int nt = (nmax + 15) / 16, tpw = (nt * nt + 6) / 7;
    if (tpw <= 1)
      hipLaunchKernelGGL((gj_reg_kernel<1>), dim3((unsigned)g), dim3(512), 0, s, B);
    else if (tpw <= 3)
      hipLaunchKernelGGL((gj_reg_kernel<3>), dim3((unsigned)g), dim3(512), 0, s, B);
    else if (tpw <= 7)
      hipLaunchKernelGGL((gj_reg_kernel<7>), dim3((unsigned)g), dim3(512), 0, s, B);
    else
      hipLaunchKernelGGL(gj_blocked_kernel, dim3((unsigned)g), dim3(256), 0, s, B);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// O[w][(k a)][j] = sum_p conj(A[k][p][a]) U[w][(k p)][j], batched over (w, k)
struct OpOverlap {
  typedef double T;
  static constexpr bool A_KCONTIG = false;
  static constexpr bool B_NCONTIG = true;
  int M, N, K, nbatch;  // M = nocc, K = m, N = nk*nocc, nbatch = W*nk
  int nk;
  const cpx<double>* A;  // [nk][m][nocc]
  const cpx<double>* U;  // [W][nk*m][n]
  cpx<double>* O;        // [W][nk*nocc][n]
  __device__ void load_a(int b, int row, int k, double& re, double& im) const {
    const cpx<double> v = A[((int64_t)(b % nk) * K + k) * M + row];
    re = v.re; im = -v.im;
  }
  __device__ void load_b(int b, int k, int col, double& re, double& im) const {
    const cpx<double> v = U[((int64_t)b * K + k) * N + col];
    re = v.re; im = v.im;
  }
  __device__ void store(int b, int row, int col, double re, double im) const {
    O[((int64_t)b * M + row) * N + col] = cpx<double>{re, im};
  }
};

// ---------------------------------------------------------------------------
// Cholesky factor and its inverse for 128 < n <= 256 (re-orthonormalisation of large
// walkers), one 256-thread workgroup per walker, in global memory (L2 resident).
// Column j of the factor S = L L^H (left-looking): row j of L (final for k < j) is staged
// in LDS, and thread r >= j forms t_r = S[r][j] - sum_{k<j} L[r][k] conj(L[j][k]);
// L[j][j] = sqrt(t_j), L[r][j] = t_r / L[j][j].  Then thread c solves L x = e_c by forward
// substitution (x = column c of L^{-1}) and writes out[c][i] = conj(x_i), the row c of
// R^{-1} = (L^{-1})^H.  A non-positive or non-finite pivot marks the walker and leaves
// R^{-1} = identity.
struct CholArgs {
  int n;
  cpx<double>* S;    // [W][n][n], lower triangle overwritten by L
  cpx<double>* out;  // [W][n][n] R^{-1}
  int* status;       // [W]
};

__global__ __launch_bounds__(256) void chol_inv_kernel(const Batch<CholArgs> B) {
  long long wloc;
  const int pb = batch_find(B, blockIdx.x, wloc);
  const int n = B.a[pb].n;
  const int w = (int)wloc;
  cpx<double>* __restrict__ L = B.a[pb].S + (int64_t)w * n * n;
  cpx<double>* __restrict__ out = B.a[pb].out + (int64_t)w * n * n;
  const int r = threadIdx.x;
  __shared__ double rjr[256], rji[256];
  __shared__ double diag[256];
  __shared__ int flag_s;
  if (r == 0) flag_s = 0;
  int bad = 0;  // 1: non-positive pivot, 2: non-finite
  for (int j = 0; j < n; ++j) {
    if (r < j) {
      const cpx<double> v = L[(int64_t)j * n + r];
      rjr[r] = v.re;
      rji[r] = v.im;
    }
    __syncthreads();
    double tr = 0.0, ti = 0.0;
    if (r >= j && r < n) {
      const cpx<double>* __restrict__ Lr = L + (int64_t)r * n;
      tr = Lr[j].re;
      ti = Lr[j].im;
#pragma unroll 4
      for (int k = 0; k < j; ++k) {
        const cpx<double> a = Lr[k];
        // a conj(b), b = L[j][k]
        tr -= a.re * rjr[k] + a.im * rji[k];
        ti -= a.im * rjr[k] - a.re * rji[k];
      }
    }
    if (r == j) {
      double d = tr;
      if (!(d > 0.0) || !isfinite(d)) {
        bad |= isfinite(d) ? 1 : 2;
        d = 1.0;
      }
      diag[j] = sqrt(d);
    }
    __syncthreads();
    if (r >= j && r < n) {
      const double sd = diag[j];
      L[(int64_t)r * n + j] = (r == j) ? cpx<double>{sd, 0.0} : cpx<double>{tr / sd, ti / sd};
    }
    __syncthreads();
  }
  if (bad) atomicOr(&flag_s, bad);
  __syncthreads();
  const int fl = flag_s;
  if (r < n) {
    cpx<double>* __restrict__ Or = out + (int64_t)r * n;
    for (int i = 0; i < r; ++i) Or[i] = cpx<double>{0.0, 0.0};
    if (fl) {
      for (int i = r; i < n; ++i) Or[i] = cpx<double>{i == r ? 1.0 : 0.0, 0.0};
    } else {
      Or[r] = cpx<double>{1.0 / diag[r], 0.0};
      for (int i = r + 1; i < n; ++i) {
        const cpx<double>* __restrict__ Li = L + (int64_t)i * n;
        double sr = 0.0, si = 0.0;
#pragma unroll 4
        for (int k = r; k < i; ++k) {
          // L[i][k] x_k with x_k = conj(Or[k])
          const cpx<double> a = Li[k], x = Or[k];
          sr += a.re * x.re + a.im * x.im;
          si += a.im * x.re - a.re * x.im;
        }
        const double id = 1.0 / diag[i];
        Or[i] = cpx<double>{-sr * id, si * id};  // conj(x_i), x_i = -s / L[i][i]
      }
    }
  }
  if (r == 0 && fl) {
    int bits = 0;
    if (fl & 1) bits |= AFQMC_WALKER_SINGULAR;
    if (fl & 2) bits |= AFQMC_WALKER_NONFINITE;
    B.a[pb].status[w] |= bits;
  }
}

// ---------------------------------------------------------------------------
// The same for n <= 128 with the lower triangle in LDS (n (n + 1) / 2 complex entries,
// 132 KB at n = 128), one 512-thread workgroup per walker, four threads per row (each
// takes every fourth term of a row's sum, combined by lane exchanges).  Cholesky column j
// (left-looking): row r >= j forms t_r = S[r][j] - sum_{k<j} L[r][k] conj(L[j][k]) from
// LDS.  Then the factor is inverted in place, column by column from the last: with
// X = L^{-1}, X L = I gives X[i][j] = -(sum_{k=j+1}^{i} X[i][k] L[k][j]) / L[j][j] (i > j),
// which needs only the columns of X to the right of j and column j of L.  Output as the
// L2 version: out[c][i] = conj(X[i][c]), the rows of R^{-1} = X^H.
__device__ __forceinline__ int tri(int r, int k) { return r * (r + 1) / 2 + k; }

__device__ __forceinline__ double quad_sum(double v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  return v;
}

__global__ __launch_bounds__(512) void chol_inv_lds_kernel(const Batch<CholArgs> B) {
  constexpr int NMAX = 128;
  __shared__ cpx<double> T[NMAX * (NMAX + 1) / 2];
  __shared__ double diag[NMAX];
  __shared__ int flag_s;
  long long wloc;
  const int pb = batch_find(B, blockIdx.x, wloc);
  const int n = B.a[pb].n;
  const int w = (int)wloc;
  const cpx<double>* __restrict__ S = B.a[pb].S + (int64_t)w * n * n;
  cpx<double>* __restrict__ out = B.a[pb].out + (int64_t)w * n * n;
  const int tid = threadIdx.x;
  const int r = tid >> 2, sub = tid & 3;  // row, and the residue of its terms mod 4
  if (tid == 0) flag_s = 0;
  for (int e = tid; e < n * n; e += 512) {
    const int rr = e / n, k = e % n;
    if (k <= rr) T[tri(rr, k)] = S[e];
  }
  __syncthreads();
  int bad = 0;  // 1: non-positive pivot, 2: non-finite
  for (int j = 0; j < n; ++j) {
    double tr = 0.0, ti = 0.0;
    const bool act = r >= j && r < n;
    if (act) {
      const cpx<double>* Lr = T + tri(r, 0);
      const cpx<double>* Lj = T + tri(j, 0);
#pragma unroll 4
      for (int k = sub; k < j; k += 4) {
        const cpx<double> a = Lr[k], b = Lj[k];
        tr += a.re * b.re + a.im * b.im;
        ti += a.im * b.re - a.re * b.im;
      }
    }
    tr = quad_sum(tr);
    ti = quad_sum(ti);
    if (act) {
      const cpx<double> sv = T[tri(r, j)];
      tr = sv.re - tr;
      ti = sv.im - ti;
    }
    if (act && r == j && sub == 0) {
      double d = tr;
      if (!(d > 0.0) || !isfinite(d)) {
        bad |= isfinite(d) ? 1 : 2;
        d = 1.0;
      }
      diag[j] = sqrt(d);
    }
    __syncthreads();
    if (act && sub == 0) {
      const double sd = diag[j];
      T[tri(r, j)] = (r == j) ? cpx<double>{sd, 0.0} : cpx<double>{tr / sd, ti / sd};
    }
    __syncthreads();
  }
  if (bad) atomicOr(&flag_s, bad);
  __syncthreads();
  const int fl = flag_s;
  if (!fl) {
    for (int j = n - 1; j >= 0; --j) {
      const int i = r;
      const bool act = i > j && i < n;
      double xr = 0.0, xi = 0.0;
      if (act) {
        const cpx<double>* Xi = T + tri(i, 0);
#pragma unroll 4
        for (int k = j + 1 + sub; k <= i; k += 4) {
          const cpx<double> x = Xi[k], l = T[tri(k, j)];  // X[i][k] L[k][j]
          xr += x.re * l.re - x.im * l.im;
          xi += x.re * l.im + x.im * l.re;
        }
      }
      xr = quad_sum(xr);
      xi = quad_sum(xi);
      const double id = 1.0 / diag[j];
      __syncthreads();
      if (act && sub == 0) T[tri(i, j)] = cpx<double>{-xr * id, -xi * id};
      if (tid == 0) T[tri(j, j)] = cpx<double>{id, 0.0};
      __syncthreads();
    }
  }
  // out[c][i] = conj(X[i][c]) for i >= c, 0 below; identity for a flagged walker
  for (int e = tid; e < n * n; e += 512) {
    const int c = e / n, i = e % n;
    cpx<double> v{0.0, 0.0};
    if (fl) {
      v.re = (i == c) ? 1.0 : 0.0;
    } else if (i >= c) {
      const cpx<double> x = T[tri(i, c)];
      v = cpx<double>{x.re, -x.im};
    }
    out[e] = v;
  }
  if (tid == 0 && fl) {
    int bits = 0;
    if (fl & 1) bits |= AFQMC_WALKER_SINGULAR;
    if (fl & 2) bits |= AFQMC_WALKER_NONFINITE;
    B.a[pb].status[w] |= bits;
  }
}

static hipError_t launch_chol_inv(const Job* jobs, const int* ids, int c, void* const* S,
                                  void* const* out, hipStream_t s) {
  Batch<CholArgs> B;
  B.nprob = c;
  long long cnt[AFQMC_MAXP];
  for (int q = 0; q < c; ++q) {
    const afqmc_kpt_problem& p = jobs[ids[q]].p;
    B.a[q].n = p.nk * p.nocc;
    if (B.a[q].n > 256) return hipErrorInvalidValue;
    B.a[q].S = (cpx<double>*)S[ids[q]];
    B.a[q].out = (cpx<double>*)out[ids[q]];
    B.a[q].status = p.status;
    cnt[q] = p.nwalk;
  }
  const long long g = batch_close(B, cnt);
  if (g < 0) return hipErrorInvalidValue;
  if (g == 0) return hipSuccess;
  if (B.a[0].n <= 128)
    hipLaunchKernelGGL(chol_inv_lds_kernel, dim3((unsigned)g), dim3(512), 0, s, B);
  else
    hipLaunchKernelGGL(chol_inv_kernel, dim3((unsigned)g), dim3(256), 0, s, B);
  return hipGetLastError();
}

// Cholesky factor and R^{-1} of the Gram matrices S[j] of every job (out[j]), the
// LDS-resident kernel for nk*nocc <= 128, the L2-resident one above.
hipError_t launch_ortho_factor(const Job* jobs, int n, void* const* S, void* const* out,
                               hipStream_t s) {
  return for_groups(
      n, [&](int i) { return jobs[i].p.nk * jobs[i].p.nocc <= 128 ? 0 : 1; },
      [&](const int* ids, int c) { return launch_chol_inv(jobs, ids, c, S, out, s); });
}

// Gh[w][i][R] = sum_j OinvT[w][i][j] U[w][R][j]; FP64, or (T = float) with the operands
// rounded to FP32 and FP32 accumulation
template <typename TT>
struct OpGreensSolve {
  typedef TT T;
  static constexpr bool A_KCONTIG = true;
  static constexpr bool B_NCONTIG = false;
  int M, N, K, nbatch;
  const cpx<double>* oinvT;
  const cpx<double>* U;
  cpx<double>* Gh;
  __device__ void load_a(int b, int row, int k, T& re, T& im) const {
    const cpx<double> v = oinvT[((int64_t)b * M + row) * K + k];
    re = (T)v.re; im = (T)v.im;
  }
  __device__ void load_b(int b, int k, int col, T& re, T& im) const {
    const cpx<double> v = U[((int64_t)b * N + col) * K + k];
    re = (T)v.re; im = (T)v.im;
  }
  __device__ void store(int b, int row, int col, T re, T im) const {
    Gh[((int64_t)b * M + row) * N + col] = cpx<double>{(double)re, (double)im};
  }
};

size_t carve_greens(Carve& c, const Dims& d, GreensWs& g) {
  g.omat = c.take(sizeof(double) * 2 * d.W * d.n() * d.n());
  g.oinvT = c.take(sizeof(double) * 2 * d.W * d.n() * d.n());
  g.logdet_new = c.take(sizeof(double) * 2 * d.W);
  return c.off;
}

// Greens for the current U of every job.  With write_logdet_new_only the log determinant
// goes to the workspace slot (the weight update then moves it into p.logdet), else into
// p.logdet.  With reduced_gh, jobs whose contraction precision is FP32 or BF16X3 form Gh by
// the FP32 product (the overlap, its inverse and log det stay FP64).
hipError_t run_greens(const Job* jobs, int n, bool write_logdet_new_only, hipStream_t s,
                      bool reduced_gh) {
  TimedScope ts(KC_GREENS, s);
  void* omat[AFQMC_MAXP];
  void* oinvT[AFQMC_MAXP];
  void* ldo[AFQMC_MAXP];
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    const Job* J = jobs + c0;
    OpOverlap ov[AFQMC_MAXP];
    OpGreensSolve<double> sv[AFQMC_MAXP];
    OpGreensSolve<float> sf[AFQMC_MAXP];
    int nd = 0, nf = 0;
    for (int q = 0; q < c; ++q) {
      const afqmc_kpt_problem& p = J[q].p;
      Carve cv(J[q].ws);
      GreensWs g;
      carve_greens(cv, dims_of(p), g);
      omat[q] = g.omat;
      oinvT[q] = g.oinvT;
      ldo[q] = write_logdet_new_only ? g.logdet_new : p.logdet;
      OpOverlap& op = ov[q];
      op.M = p.nocc; op.K = p.m; op.N = p.nk * p.nocc;
      op.nbatch = p.nwalk * p.nk;
      op.nk = p.nk;
      op.A = (const cpx<double>*)p.A;
      op.U = (const cpx<double>*)p.U;
      op.O = (cpx<double>*)g.omat;
      const bool f32 = reduced_gh && low_prec(p.prec);
      auto fill = [&](auto& sl) {
        sl.M = p.nk * p.nocc;
        sl.N = p.nk * p.m;
        sl.K = p.nk * p.nocc;
        sl.nbatch = p.nwalk;
        sl.oinvT = (const cpx<double>*)g.oinvT;
        sl.U = (const cpx<double>*)p.U;
        sl.Gh = (cpx<double>*)p.Gh;
      };
      if (f32) fill(sf[nf++]);
      else fill(sv[nd++]);
    }
    hipError_t e = launch_ops<16, 64, 16, 1, 4>(ov, c, s);
    if (e != hipSuccess) return e;
    e = launch_gj_blocked(J, c, omat, oinvT, ldo, s);
    if (e != hipSuccess) return e;
    // up to 112 rows (nk nocc) in one row tile, so that every U column is read once
    int md = 0, mf = 0;
    for (int q = 0; q < nd; ++q) md = sv[q].M > md ? sv[q].M : md;
    for (int q = 0; q < nf; ++q) mf = sf[q].M > mf ? sf[q].M : mf;
    if (nd) e = (md <= 112) ? launch_ops<112, 64, 16, 1, 4>(sv, nd, s)
                            : launch_ops<64, 64, 16, 2, 2>(sv, nd, s);
    if (e != hipSuccess) return e;
    if (nf) e = (mf <= 112) ? launch_ops<112, 64, 16, 1, 4>(sf, nf, s)
                            : launch_ops<64, 64, 16, 2, 2>(sf, nf, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Hybrid phaseless weight update, one workgroup per walker:
//   log I = 2 (logdet' - logdet) + sum_{Q,g,+/-} (x xbar - xbar^2/2),
//   dtheta = arg exp(2 (logdet' - logdet)), w <- |I| max(0, cos dtheta) w.
// A two-determinant walker (one per spin) takes the sum of the two spins' log-overlap
// changes in place of twice one, and writes the same weight and status to both halves.
struct WeightArgs {
  int64_t nf;                    // nk * nchol * 2 field components per walker
  const double* x;               // [W][nf]
  const cpx<double>* xbar;       // [W][nf]
  cpx<double>* logdet;           // [W]
  const cpx<double>* logdet_new; // [W]
  double* weight;                // [W]
  int* status;                   // [W]
  const double* etrial;          // [1] E_T per supercell, or null (no shift)
  double dt;
  // the down half of a two-determinant walker set (null for one determinant)
  cpx<double>* logdet2;
  const cpx<double>* logdet2_new;
  double* weight2;
  int* status2;
};

__global__ __launch_bounds__(1024) void weight_kernel(const Batch<WeightArgs> B) {
  long long wloc;
  const int pb = batch_find(B, blockIdx.x, wloc);
  const int64_t nf = B.a[pb].nf;
  const double* __restrict__ x = B.a[pb].x;
  const cpx<double>* __restrict__ xbar = B.a[pb].xbar;
  cpx<double>* __restrict__ logdet = B.a[pb].logdet;
  const cpx<double>* __restrict__ logdet_new = B.a[pb].logdet_new;
  double* __restrict__ weight = B.a[pb].weight;
  int* __restrict__ status = B.a[pb].status;
  const int w = (int)wloc;
  const int tid = threadIdx.x;
  constexpr int NT = 1024;
  __shared__ double sr[NT], si[NT];
  double ar = 0.0, ai = 0.0;
  const double* xw = x + (int64_t)w * nf;
  const cpx<double>* bw = xbar + (int64_t)w * nf;
  // eight elements per thread and pass, all loads issued before the sums (one workgroup per
  // walker: the latency of the loads, not their bytes, bounds this loop, so the workgroup
  // is as wide as allowed and a c1 walker takes two passes)
  constexpr int U = 8;
  for (int64_t i0 = tid; i0 < nf; i0 += NT * U) {
    double xv[U];
    cpx<double> b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + NT * u;
      xv[u] = i < nf ? xw[i] : 0.0;
      b[u] = i < nf ? bw[i] : cpx<double>{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // x b - b^2 / 2
      ar += xv[u] * b[u].re - 0.5 * (b[u].re * b[u].re - b[u].im * b[u].im);
      ai += xv[u] * b[u].im - b[u].re * b[u].im;
    }
  }
  sr[tid] = ar;
  si[tid] = ai;
  __syncthreads();
  for (int o = NT / 2; o >= 1; o >>= 1) {
    if (tid < o) { sr[tid] += sr[tid + o]; si[tid] += si[tid + o]; }
    __syncthreads();
  }
  if (tid == 0) {
    const cpx<double> l0 = logdet[w], l1 = logdet_new[w];
    cpx<double>* const ld2 = B.a[pb].logdet2;
    cpx<double> m1{0.0, 0.0};
    double lrr, lri;
    if (ld2) {
      const cpx<double> m0 = ld2[w];
      m1 = B.a[pb].logdet2_new[w];
      lrr = (l1.re - l0.re) + (m1.re - m0.re);
      lri = (l1.im - l0.im) + (m1.im - m0.im);
    } else {
      lrr = 2.0 * (l1.re - l0.re);
      lri = 2.0 * (l1.im - l0.im);
    }
    // the projector's energy shift exp(dt E_T) joins the modulus of I
    const double* et = B.a[pb].etrial;
    const double lIr = lrr + sr[0] + (et ? B.a[pb].dt * et[0] : 0.0);
    const double dth = atan2(sin(lri), cos(lri));
    const double c = cos(dth);
    int st = status[w] | (ld2 ? B.a[pb].status2[w] : 0);
    double wn = weight[w];
    if (st & (AFQMC_WALKER_SINGULAR | AFQMC_WALKER_NONFINITE)) {
      wn = 0.0;
    } else {
      if (!(c > 0.0)) st |= AFQMC_WALKER_KILLED;
      wn = exp(lIr) * fmax(0.0, c) * wn;
      if (!isfinite(wn)) { st |= AFQMC_WALKER_NONFINITE; wn = 0.0; }
    }
    weight[w] = wn;
    status[w] = st;
    logdet[w] = l1;
    if (ld2) {
      B.a[pb].weight2[w] = wn;
      B.a[pb].status2[w] = st;
      ld2[w] = m1;
    }
  }
}

hipError_t launch_weights(const Job* jobs, int n, hipStream_t s) {
  TimedScope ts(KC_WEIGHTS, s);
  // one entry per closed-shell problem and per two-determinant pair (its up half)
  std::vector<int> ids;
  for (int i = 0; i < n; ++i)
    if (jobs[i].p.spin != AFQMC_SPIN_DOWN) ids.push_back(i);
  const int ne = (int)ids.size();
  for (int c0 = 0; c0 < ne; c0 += AFQMC_MAXP) {
    const int c = (ne - c0 < AFQMC_MAXP) ? ne - c0 : AFQMC_MAXP;
    Batch<WeightArgs> B;
    B.nprob = c;
    long long cnt[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const int i = ids[c0 + q];
      const Job& j = jobs[i];
      const afqmc_kpt_problem& p = j.p;
      Carve cv(j.ws);
      GreensWs g;
      carve_greens(cv, dims_of(p), g);
      WeightArgs& a = B.a[q];
      a.logdet2 = nullptr;
      a.logdet2_new = nullptr;
      a.weight2 = nullptr;
      a.status2 = nullptr;
      if (p.spin == AFQMC_SPIN_UP) {
        const Job& d = jobs[i + 1];
        Carve cd(d.ws);
        GreensWs gd;
        carve_greens(cd, dims_of(d.p), gd);
        a.logdet2 = (cpx<double>*)d.p.logdet;
        a.logdet2_new = (const cpx<double>*)gd.logdet_new;
        a.weight2 = d.p.weight;
        a.status2 = d.p.status;
      }
      a.nf = (int64_t)p.nk * p.nchol * 2;
      a.x = j.x;
      a.xbar = (const cpx<double>*)j.xbar;
      a.logdet = (cpx<double>*)p.logdet;
      a.logdet_new = (const cpx<double>*)g.logdet_new;
      a.weight = p.weight;
      a.status = p.status;
      a.etrial = p.etrial;
      a.dt = p.dt;
      cnt[q] = p.nwalk;
    }
    const long long g = batch_close(B, cnt);
    if (g < 0) return hipErrorInvalidValue;
    if (g == 0) continue;
    hipLaunchKernelGGL(weight_kernel, dim3((unsigned)g), dim3(1024), 0, s, B);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace afqmc
