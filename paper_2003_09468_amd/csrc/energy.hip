// Local energy and its adjoint (k-point local-energy equation; energy-evaluation
// algorithm of the GPU-implementation section, steps 1-3).
//
// Exchange.  For t = (Q, k, k') the algorithm forms
//   T1_t[w][b][a][g] = sum_r Lh[Q][k][a][r][g]      Gh[w][((k'-Q) b), ((k-Q) r)]
//   T2_t[w][a][b][g] = sum_s Lh[-Q][k'-Q][b][s][g]  Gh[w][(k a), (k' s)]
// and accumulates -sum T1_t[b,a,g] T2_t[a,b,g].  With pi(t) = (-Q, k'-Q, k-Q), the time-
// reversal partner, T2_t[a][b] = T1_{pi(t)}[a][b] and the summand of pi(t) equals that of t,
// so one workgroup per unordered pair {t, pi(t)} computes the two T1 tiles on MFMA (K = m),
// pairs element (b, a) of one with (a, b) of the other through a wave-private LDS tile, and
// accumulates in FP64.  T1 never reaches memory.  Work per pair: one GEMM per triple
// instead of two.
//
// Layout of one 16 x 16 MFMA tile: rows (g, a) with 16/nocc values of g, columns (w, b)
// with 16/nocc walkers; each of the 4 waves of a workgroup owns its walkers (their Gh
// blocks stay in registers for the whole g loop) and all waves share LDS-staged slabs of
// the half-rotated Cholesky vectors, double buffered over g.
#include <math.h>

#include "cgemm.h"
#include "internal.h"

namespace afqmc {


struct ExchArgs {
  int nk, m, nocc, C, W, nchunk_w;
  KMesh mesh;
  const void* Lh;           // [nk][nk][nocc][m][C] in the contraction precision, or for
                            // BF16X3 the split planes [nk][nk][C][nocc][4][KP] (bf16)
  const cpx<double>* Gh;    // [W][nk*nocc][nk*m]
  cpx<double>* part;        // [nk^3][W]
};

template <typename T, int KSMAX>
__global__ __launch_bounds__(256) void exchange_kernel(const Batch<ExchArgs> B) {
  typedef typename mfma16<T>::acc_t acc_t;
  constexpr int RP = 4 * KSMAX;
  constexpr int NLD = (2 * 16 * RP) / 256;  // slab elements per thread (both slabs)

  __shared__ T LA[2][2][2][RP][16];  // [buf][slab][re/im][r][(g, a)]
  __shared__ T XB[4][2][16][17];     // per-wave exchange tile
  __shared__ double red[2][256];

  long long bid;
  // launch order (consecutive workgroups on different XCDs): neighbouring triples, which
  // share a slab of Lh, run at the same time on all XCDs
  const int pb = batch_find(B, blockIdx.x, bid);
  const int nk = B.a[pb].nk, m = B.a[pb].m, nocc = B.a[pb].nocc, C = B.a[pb].C, W = B.a[pb].W;
  const int nchunk_w = B.a[pb].nchunk_w;
  const KMesh mesh = B.a[pb].mesh;
  const cpx<T>* __restrict__ Lh = (const cpx<T>*)B.a[pb].Lh;
  const cpx<double>* __restrict__ Gh = B.a[pb].Gh;
  cpx<double>* __restrict__ part = B.a[pb].part;
  const int chunk = (int)(bid % nchunk_w);
  const int t = (int)(bid / nchunk_w);
  const int kp = t % nk, k = (t / nk) % nk, Q = t / (nk * nk);
  const int mQ = mesh.neg(Q), kpq = mesh.kmq(kp, Q), kq = mesh.kmq(k, Q);
  const int tp = (mQ * nk + kpq) * nk + kq;  // partner triple (-Q, k'-Q, k-Q)
  if (t > tp) return;
  const double mult = (t == tp) ? 1.0 : 2.0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Gs = 16 / nocc, Ws = 16 / nocc;
  const int KS = (m + 3) >> 2;
  const int col = lane & 15;
  const int ws_l = col / nocc, b_l = col % nocc;
  const int wl = chunk * 4 * Ws + wave * Ws + ws_l;
  const bool colok = (ws_l < Ws) && (wl < W);
  const int64_t Nn = (int64_t)nk * m, nn = (int64_t)nk * nocc;

  // Gh fragments of this lane's column, for both GEMMs (B operand: B[r][(w, b)])
  T b1r[KSMAX], b1i[KSMAX], b2r[KSMAX], b2i[KSMAX];
#pragma unroll
  for (int s = 0; s < KSMAX; ++s) {
    const int r = 4 * s + (lane >> 4);
    T x1r = 0, x1i = 0, x2r = 0, x2i = 0;
    if (s < KS && r < m && colok) {
      const cpx<double> g1 = Gh[((int64_t)wl * nn + (int64_t)kpq * nocc + b_l) * Nn + (int64_t)kq * m + r];
      const cpx<double> g2 = Gh[((int64_t)wl * nn + (int64_t)k * nocc + b_l) * Nn + (int64_t)kp * m + r];
      x1r = (T)g1.re; x1i = (T)g1.im; x2r = (T)g2.re; x2i = (T)g2.im;
    }
    b1r[s] = x1r; b1i[s] = x1i; b2r[s] = x2r; b2i[s] = x2i;
  }

  const cpx<T>* slab0 = Lh + ((int64_t)Q * nk + k) * nocc * m * C;
  const cpx<T>* slab1 = Lh + ((int64_t)mQ * nk + kpq) * nocc * m * C;
  const int nch = (C + Gs - 1) / Gs;

  // slab element e of this thread: idx = (sl, r, q), q = a * Gs + g_s (g fastest in memory)
  T pr[NLD], pi[NLD];
  auto fetch = [&](int c) {
    const int g0 = c * Gs;
#pragma unroll
    for (int e = 0; e < NLD; ++e) {
      const int idx = tid + 256 * e;
      const int sl = idx / (16 * RP), rem = idx % (16 * RP);
      const int r = rem / 16, q = rem % 16;
      const int a = q / Gs, g_s = q % Gs;
      T vr = 0, vi = 0;
      if (a < nocc && r < m && g0 + g_s < C) {
        const cpx<T>* sb = sl ? slab1 : slab0;
        const cpx<T> v = sb[((int64_t)a * m + r) * C + g0 + g_s];
        vr = v.re; vi = v.im;
      }
      pr[e] = vr; pi[e] = vi;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NLD; ++e) {
      const int idx = tid + 256 * e;
      const int sl = idx / (16 * RP), rem = idx % (16 * RP);
      const int r = rem / 16, q = rem % 16;
      const int a = q / Gs, g_s = q % Gs;
      if (a < nocc) {
        LA[buf][sl][0][r][g_s * nocc + a] = pr[e];
        LA[buf][sl][1][r][g_s * nocc + a] = pi[e];
      }
    }
  };
  // rows (g, a) beyond Gs * nocc stay zero
  for (int i = tid; i < 2 * 2 * 2 * RP * 16; i += 256) (&LA[0][0][0][0][0])[i] = (T)0;
  __syncthreads();

  double sr = 0.0, si = 0.0;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) fetch(c + 1);
    acc_t a1r = mfma16<T>::zero(), a1i = mfma16<T>::zero();
    acc_t a2r = mfma16<T>::zero(), a2i = mfma16<T>::zero();
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) {
      if (s < KS) {
        const int r = 4 * s + (lane >> 4);
        const T x1r = LA[buf][0][0][r][col], x1i = LA[buf][0][1][r][col];
        const T x2r = LA[buf][1][0][r][col], x2i = LA[buf][1][1][r][col];
        cmfma<T>(x1r, x1i, b1r[s], b1i[s], a1r, a1i);
        cmfma<T>(x2r, x2i, b2r[s], b2i[s], a2r, a2i);
      }
    }
    // T1 of the partner triple to the wave-private tile
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = mfma16<T>::drow(lane, v);
      XB[wave][0][row][col] = a2r[v];
      XB[wave][1][row][col] = a2i[v];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int g0 = c * Gs;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = mfma16<T>::drow(lane, v);
      const int g_s = row / nocc, a = row % nocc;
      if (colok && g_s < Gs && g0 + g_s < C) {
        const int rp = g_s * nocc + b_l, cp = ws_l * nocc + a;
        const double pr2 = (double)XB[wave][0][rp][cp], pi2 = (double)XB[wave][1][rp][cp];
        const double p1r = (double)a1r[v], p1i = (double)a1i[v];
        sr += p1r * pr2 - p1i * pi2;
        si += p1r * pi2 + p1i * pr2;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (c + 1 < nch) stash(buf ^ 1);
    __syncthreads();
  }

  // per-walker reduction: lanes of a wave with the same column walker
  red[0][tid] = sr;
  red[1][tid] = si;
  __syncthreads();
  if (tid < 4 * Ws) {
    const int wv = tid / Ws, wsi = tid % Ws;
    const int w = chunk * 4 * Ws + wv * Ws + wsi;
    if (w < W) {
      double ar = 0.0, ai = 0.0;
      for (int grp = 0; grp < 4; ++grp)
        for (int b = 0; b < nocc; ++b) {
          const int l = wv * 64 + grp * 16 + wsi * nocc + b;
          ar += red[0][l];
          ai += red[1][l];
        }
      part[(int64_t)t * W + w] = cpx<double>{-mult * ar, -mult * ai};
    }
  }
}

// ---------------------------------------------------------------------------
// The exchange with BF16-split operands (three BF16 MFMA passes, FP32 accumulation).
//
// Every FP32 operand x is split as x = hi + lo with hi = bf16(x) and lo = bf16(x - hi)
// (round to nearest even), so x - hi - lo = O(2^-16 |x|); a real product is taken as
// hi hi' + hi lo' + lo hi' (the lo lo' term, O(2^-16 |x x'|), is dropped) on the
// 16x16x32 BF16 MFMA.  Same work decomposition as exchange_kernel: rows (g, a), columns
// (w, b), K = r padded to 32 * KB; the Gh fragments are split once into registers, and the
// Lh slabs come pre-split from prepare (four bf16 planes: re hi, re lo, im hi, im lo, r
// contiguous) and are staged into LDS with 16-byte copies.
template <int KB, int WT>
__global__ __launch_bounds__(256) void exchange_bf16x3_kernel(const Batch<ExchArgs> B) {
  constexpr int KP = 32 * KB;  // r padded to the MFMA K
  constexpr int RS = KP + 8;   // LDS row stride (bf16): rows start 16-byte aligned

  __shared__ __attribute__((aligned(16))) unsigned short LA[2][2][4][16][RS];  // [buf][slab][plane][(g, a)][r]
  __shared__ float XB[4][2][16][17];
  __shared__ double red[2][256];

  long long bid;
  const int pb = batch_find(B, blockIdx.x, bid);
  const int nk = B.a[pb].nk, m = B.a[pb].m, nocc = B.a[pb].nocc, C = B.a[pb].C, W = B.a[pb].W;
  const int nchunk_w = B.a[pb].nchunk_w;
  const KMesh mesh = B.a[pb].mesh;
  const unsigned short* __restrict__ Lhs = (const unsigned short*)B.a[pb].Lh;
  const cpx<double>* __restrict__ Gh = B.a[pb].Gh;
  cpx<double>* __restrict__ part = B.a[pb].part;
  const int chunk = (int)(bid % nchunk_w);
  const int t = (int)(bid / nchunk_w);
  const int kp = t % nk, k = (t / nk) % nk, Q = t / (nk * nk);
  const int mQ = mesh.neg(Q), kpq = mesh.kmq(kp, Q), kq = mesh.kmq(k, Q);
  const int tp = (mQ * nk + kpq) * nk + kq;
  if (t > tp) return;
  const double mult = (t == tp) ? 1.0 : 2.0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Gs = 16 / nocc, Ws = 16 / nocc;
  const int col = lane & 15;
  const int ws_l = col / nocc, b_l = col % nocc;
  const int64_t Nn = (int64_t)nk * m, nn = (int64_t)nk * nocc;
  // column tile ct of this wave: walkers chunk 4 WT Ws + (wave WT + ct) Ws + (0 .. Ws-1)
  auto walker = [&](int ct) { return chunk * 4 * WT * Ws + (wave * WT + ct) * Ws + ws_l; };

  // Gh fragments (B operand, B[r][(w, b)], r = 32 kb + 8 (lane / 16) + i), split; the
  // Lh fragments of a g chunk serve all WT column tiles
  u16x8 g1[WT][KB][4], g2[WT][KB][4];
#pragma unroll
  for (int ct = 0; ct < WT; ++ct) {
    const int wl = walker(ct);
    const bool colok = (ws_l < Ws) && (wl < W);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = 32 * kb + 8 * (lane >> 4) + i;
        float x1r = 0.f, x1i = 0.f, x2r = 0.f, x2i = 0.f;
        if (r < m && colok) {
          const cpx<double> v1 = Gh[((int64_t)wl * nn + (int64_t)kpq * nocc + b_l) * Nn + (int64_t)kq * m + r];
          const cpx<double> v2 = Gh[((int64_t)wl * nn + (int64_t)k * nocc + b_l) * Nn + (int64_t)kp * m + r];
          x1r = (float)v1.re; x1i = (float)v1.im; x2r = (float)v2.re; x2i = (float)v2.im;
        }
        unsigned short h, l;
        bf16_split(x1r, h, l); g1[ct][kb][0][i] = h; g1[ct][kb][1][i] = l;
        bf16_split(x1i, h, l); g1[ct][kb][2][i] = h; g1[ct][kb][3][i] = l;
        bf16_split(x2r, h, l); g2[ct][kb][0][i] = h; g2[ct][kb][1][i] = l;
        bf16_split(x2i, h, l); g2[ct][kb][2][i] = h; g2[ct][kb][3][i] = l;
      }
  }

  // the pre-split planes: slab (Q, k) is [C][nocc][4][KP] bf16, contiguous per g chunk
  const unsigned short* slab0 = Lhs + ((int64_t)Q * nk + k) * C * nocc * 4 * KP;
  const unsigned short* slab1 = Lhs + ((int64_t)mQ * nk + kpq) * C * nocc * 4 * KP;
  const int nch = (C + Gs - 1) / Gs;

  // 16-byte units of a chunk: u = ((g_s nocc + a) 4 + plane) (KP / 8) + r8, per slab.
  // DEPTH chunks are in flight in registers (the slabs mostly come from beyond L2); the
  // loads are unconditional (clamped addresses, zeros selected when staged) so that each
  // wait covers only the oldest chunk.
  constexpr int UPR = KP / 8;                 // units per (row, plane)
  constexpr int NU = (2 * 16 * 4 * UPR) / 256;  // units per thread (both slabs)
  constexpr int DEPTH = KB == 1 ? 4 : 3;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 pu[DEPTH][NU];
  auto fetch = [&](int c, u4 (&xu)[NU]) {
    const int g0 = (c < nch ? c : nch - 1) * Gs;
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int idx = tid + 256 * e;
      const int sl = idx / (16 * 4 * UPR), u = idx % (16 * 4 * UPR);
      const int row = min(u / (4 * UPR), Gs * nocc - 1);  // g_s * nocc + a
      const int gg = min(g0 + row / nocc, C - 1);
      const unsigned short* sb = sl ? slab1 : slab0;
      xu[e] = *reinterpret_cast<const u4*>(
          sb + (((int64_t)gg * nocc + row % nocc) * 4 * UPR + u % (4 * UPR)) * 8);
    }
  };
  auto stash = [&](int c, int buf, const u4 (&xu)[NU]) {
    const int g0 = c * Gs;
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int idx = tid + 256 * e;
      const int sl = idx / (16 * 4 * UPR), u = idx % (16 * 4 * UPR);
      const int row = u / (4 * UPR), pl = (u / UPR) % 4, r8 = u % UPR;
      const u4 z = {0u, 0u, 0u, 0u};
      if (row < Gs * nocc)
        *reinterpret_cast<u4*>(&LA[buf][sl][pl][row][r8 * 8]) =
            g0 + row / nocc < C ? xu[e] : z;
    }
  };
  // rows (g, a) beyond Gs * nocc stay zero
  for (int i = tid; i < 2 * 2 * 4 * 16 * RS; i += 256) (&LA[0][0][0][0][0])[i] = 0;
  __syncthreads();

  double sr[WT], si[WT];
#pragma unroll
  for (int ct = 0; ct < WT; ++ct) sr[ct] = si[ct] = 0.0;
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) fetch(d, pu[d]);
  stash(0, 0, pu[0]);
  fetch(DEPTH, pu[0]);
  __syncthreads();
  // iteration c: chunk c from LDS buffer c & 1; chunk c + 1 (slot (c + 1) % DEPTH) to the
  // other buffer; chunk c + 1 + DEPTH requested into the freed slot
  for (int c0 = 0; c0 < nch; c0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const int c = c0 + d;
      const int buf = c & 1;
      if (c < nch) {
        v4f a1r[WT], a1i[WT], a2r[WT], a2i[WT];
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
          a1r[ct] = v4f{0.f, 0.f, 0.f, 0.f};
          a1i[ct] = a1r[ct]; a2r[ct] = a1r[ct]; a2i[ct] = a1r[ct];
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const int r0 = 32 * kb + 8 * (lane >> 4);
          u16x8 x[2][4];
#pragma unroll
          for (int sl = 0; sl < 2; ++sl)
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
              x[sl][pl] = *reinterpret_cast<const u16x8*>(&LA[buf][sl][pl][col][r0]);
          const u16x8 n02 = bf16_neg(x[0][2]), n03 = bf16_neg(x[0][3]), n12 = bf16_neg(x[1][2]),
                      n13 = bf16_neg(x[1][3]);
#pragma unroll
          for (int ct = 0; ct < WT; ++ct) {
            // re += Lr Gr - Li Gi,  im += Lr Gi + Li Gr  (-Li: flipped sign bits)
            a1r[ct] = mul3(x[0][0], x[0][1], g1[ct][kb][0], g1[ct][kb][1], a1r[ct]);
            a1r[ct] = mul3(n02, n03, g1[ct][kb][2], g1[ct][kb][3], a1r[ct]);
            a1i[ct] = mul3(x[0][0], x[0][1], g1[ct][kb][2], g1[ct][kb][3], a1i[ct]);
            a1i[ct] = mul3(x[0][2], x[0][3], g1[ct][kb][0], g1[ct][kb][1], a1i[ct]);
            a2r[ct] = mul3(x[1][0], x[1][1], g2[ct][kb][0], g2[ct][kb][1], a2r[ct]);
            a2r[ct] = mul3(n12, n13, g2[ct][kb][2], g2[ct][kb][3], a2r[ct]);
            a2i[ct] = mul3(x[1][0], x[1][1], g2[ct][kb][2], g2[ct][kb][3], a2i[ct]);
            a2i[ct] = mul3(x[1][2], x[1][3], g2[ct][kb][0], g2[ct][kb][1], a2i[ct]);
          }
        }
        const int g0 = c * Gs;
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
          const bool colok = (ws_l < Ws) && (walker(ct) < W);
          // T1 of the partner triple to the wave-private tile (FP32 MFMA output layout)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = mfma16<float>::drow(lane, v);
            XB[wave][0][row][col] = a2r[ct][v];
            XB[wave][1][row][col] = a2i[ct][v];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = mfma16<float>::drow(lane, v);
            const int g_s = row / nocc, a = row % nocc;
            if (colok && g_s < Gs && g0 + g_s < C) {
              const int rp = g_s * nocc + b_l, cp = ws_l * nocc + a;
              const double pr2 = (double)XB[wave][0][rp][cp], pi2 = (double)XB[wave][1][rp][cp];
              const double p1r = (double)a1r[ct][v], p1i = (double)a1i[ct][v];
              sr[ct] += p1r * pr2 - p1i * pi2;
              si[ct] += p1r * pi2 + p1i * pr2;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      // past the last chunk the stores go to the buffer nobody reads
      stash(c + 1, buf ^ 1, pu[(d + 1) % DEPTH]);
      fetch(c + 1 + DEPTH, pu[(d + 1) % DEPTH]);
      __syncthreads();
    }
  }

  // per-walker reduction over the lanes of a wave with the same column walker
#pragma unroll
  for (int ct = 0; ct < WT; ++ct) {
    red[0][tid] = sr[ct];
    red[1][tid] = si[ct];
    __syncthreads();
    if (tid < 4 * Ws) {
      const int wv = tid / Ws, wsi = tid % Ws;
      const int w = chunk * 4 * WT * Ws + (wv * WT + ct) * Ws + wsi;
      if (w < W) {
        double ar = 0.0, ai = 0.0;
        for (int grp = 0; grp < 4; ++grp)
          for (int b = 0; b < nocc; ++b) {
            const int l = wv * 64 + grp * 16 + wsi * nocc + b;
            ar += red[0][l];
            ai += red[1][l];
          }
        part[(int64_t)t * W + w] = cpx<double>{-mult * ar, -mult * ai};
      }
    }
    __syncthreads();
  }
}

// The same for nocc = 4 (four occupied bands per k-point, as in the diamond workloads),
// with the occupied dimension fixed: a 16-row tile holds 4 values of g and a 16-column
// tile 4 walkers.  Lane (g_s, w_s, b) of a wave holds T1_t[b][a] of its (g, w) in
// register a, and the partner's T1_pi(t)[a][b] sits in lane (g_s, w_s, a), register b:
// the partner tile is transposed inside each lane quad through a wave-private LDS tile
// (row stride 20 words, so the 32-bit scatter of 64 lanes hits 64 distinct banks), and
// the four products of one (g, w, b) are summed in FP32 before the FP64 sum over g.
// Rows of g >= C and columns of walkers >= W hold zeros, so their products vanish.
template <int KB, int WT>
__global__ __launch_bounds__(256) void exchange_bf16x3_q4_kernel(const Batch<ExchArgs> B) {
  constexpr int KP = 32 * KB;        // r padded to the MFMA K
  constexpr int RS = KP + 8;         // LDS row stride (bf16): rows start 16-byte aligned
  constexpr int UPR = KP / 8;        // 16-byte units per (row, plane)
  constexpr int CU = 16 * 4 * UPR;   // units of one slab chunk: rows (g, a) x planes x r
  constexpr int NU = 2 * CU / 256;   // units per thread (both slabs)
  constexpr int DEPTH = 2;           // chunks in flight (3 waves per SIMD at K = 32)
  constexpr int TS = 20;             // transpose tile row stride (words)

  // [buf][slab][plane][(g, a) r]: rows of RS (80 bytes: the 16 rows of one fragment read hit
  // distinct banks), planes padded by 64 bytes (the staging stores of 4 planes x 4 units
  // hit distinct banks)
  constexpr int PS = 16 * RS + 32;
  __shared__ __attribute__((aligned(16))) unsigned short LA[2][2][4][PS];
  __shared__ __attribute__((aligned(16))) float XT[4][WT][2][16 * TS];         // [wave][ct][re/im][quad][.]
  __shared__ double red[2][256];

  long long bid;
  const int pb = batch_find(B, blockIdx.x, bid);
  const int nk = B.a[pb].nk, m = B.a[pb].m, C = B.a[pb].C, W = B.a[pb].W;
  const int nchunk_w = B.a[pb].nchunk_w;
  const KMesh mesh = B.a[pb].mesh;
  const unsigned short* __restrict__ Lhs = (const unsigned short*)B.a[pb].Lh;
  const cpx<double>* __restrict__ Gh = B.a[pb].Gh;
  cpx<double>* __restrict__ part = B.a[pb].part;
  const int chunk = (int)(bid % nchunk_w);
  const int t = (int)(bid / nchunk_w);
  const int kp = t % nk, k = (t / nk) % nk, Q = t / (nk * nk);
  const int mQ = mesh.neg(Q), kpq = mesh.kmq(kp, Q), kq = mesh.kmq(k, Q);
  const int tp = (mQ * nk + kpq) * nk + kq;
  if (t > tp) return;
  const double mult = (t == tp) ? 1.0 : 2.0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, ws_l = col >> 2, b_l = col & 3;
  const int64_t Nn = (int64_t)nk * m, nn = (int64_t)nk * 4;
  // column tile ct of this wave: walkers 16 WT chunk + 4 (wave WT + ct) + (0 .. 3)
  auto walker = [&](int ct) { return chunk * 16 * WT + (wave * WT + ct) * 4 + ws_l; };

  // Gh fragments (B operand, B[r][(w, b)], r = 32 kb + 8 (lane / 16) + i), split
  u16x8 g1[WT][KB][4], g2[WT][KB][4];
#pragma unroll
  for (int ct = 0; ct < WT; ++ct) {
    const int wl = walker(ct);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = 32 * kb + 8 * (lane >> 4) + i;
        float x1r = 0.f, x1i = 0.f, x2r = 0.f, x2i = 0.f;
        if (r < m && wl < W) {
          const cpx<double> v1 = Gh[((int64_t)wl * nn + (int64_t)kpq * 4 + b_l) * Nn + (int64_t)kq * m + r];
          const cpx<double> v2 = Gh[((int64_t)wl * nn + (int64_t)k * 4 + b_l) * Nn + (int64_t)kp * m + r];
          x1r = (float)v1.re; x1i = (float)v1.im; x2r = (float)v2.re; x2i = (float)v2.im;
        }
        unsigned short h, l;
        bf16_split(x1r, h, l); g1[ct][kb][0][i] = h; g1[ct][kb][1][i] = l;
        bf16_split(x1i, h, l); g1[ct][kb][2][i] = h; g1[ct][kb][3][i] = l;
        bf16_split(x2r, h, l); g2[ct][kb][0][i] = h; g2[ct][kb][1][i] = l;
        bf16_split(x2i, h, l); g2[ct][kb][2][i] = h; g2[ct][kb][3][i] = l;
      }
  }

  // slab (Q, k) is [C][4][4][KP] bf16: chunk c (g = 4c .. 4c + 3) is units [c CU, (c + 1) CU)
  const unsigned short* slab0 = Lhs + ((int64_t)Q * nk + k) * C * 16 * KP;
  const unsigned short* slab1 = Lhs + ((int64_t)mQ * nk + kpq) * C * 16 * KP;
  const int nch = (C + 3) / 4;
  const int64_t ulast = (int64_t)C * 16 * UPR - 1;  // last unit of a slab

  // DEPTH chunks in flight in registers; the loads are unconditional (clamped into the
  // slab; rows of g >= C are zeroed when staged) so that each wait covers only the oldest
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 pu[DEPTH][NU];
  auto fetch = [&](int c, u4 (&xu)[NU]) {
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int idx = tid + 256 * e;
      const int sl = idx / CU, u = idx % CU;
      const int64_t un = min((int64_t)c * CU + u, ulast);
      xu[e] = *reinterpret_cast<const u4*>((sl ? slab1 : slab0) + un * 8);
    }
  };
  auto stash = [&](int c, int buf, const u4 (&xu)[NU]) {
    const bool full = 4 * c + 4 <= C;  // uniform: every row of the chunk is a valid g
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int idx = tid + 256 * e;
      const int sl = idx / CU, u = idx % CU;
      const int row = u / (4 * UPR), pl = (u / UPR) % 4, r8 = u % UPR;
      u4 v = xu[e];
      if (!full && 4 * c + row / 4 >= C) v = u4{0u, 0u, 0u, 0u};
      *reinterpret_cast<u4*>(&LA[buf][sl][pl][row * RS + r8 * 8]) = v;
    }
  };

  double sr[WT], si[WT];
#pragma unroll
  for (int ct = 0; ct < WT; ++ct) sr[ct] = si[ct] = 0.0;
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) fetch(d, pu[d]);
  stash(0, 0, pu[0]);
  fetch(DEPTH, pu[0]);
  __syncthreads();
  const int quad = lane >> 2, bq = lane & 3;
  // iteration c: chunk c from LDS buffer c & 1; chunk c + 1 (slot (c + 1) % DEPTH) to the
  // other buffer; chunk c + 1 + DEPTH requested into the freed slot
  for (int c0 = 0; c0 < nch; c0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const int c = c0 + d;
      const int buf = c & 1;
      if (c < nch) {
        v4f a1r[WT], a1i[WT], a2r[WT], a2i[WT];
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
          a1r[ct] = v4f{0.f, 0.f, 0.f, 0.f};
          a1i[ct] = a1r[ct]; a2r[ct] = a1r[ct]; a2i[ct] = a1r[ct];
        }
        // one slab at a time (register budget): re += Lr Gr - Li Gi, im += Lr Gi + Li Gr
        // (-Li: flipped sign bits)
        auto slab_mfma = [&](int sl, const u16x8 (&g)[WT][KB][4], v4f (&ar)[WT], v4f (&ai)[WT]) {
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
            const int r0 = 32 * kb + 8 * (lane >> 4);
            u16x8 x[4];
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
              x[pl] = *reinterpret_cast<const u16x8*>(&LA[buf][sl][pl][col * RS + r0]);
            const u16x8 n2 = bf16_neg(x[2]), n3 = bf16_neg(x[3]);
#pragma unroll
            for (int ct = 0; ct < WT; ++ct) {
              ar[ct] = mul3(x[0], x[1], g[ct][kb][0], g[ct][kb][1], ar[ct]);
              ar[ct] = mul3(n2, n3, g[ct][kb][2], g[ct][kb][3], ar[ct]);
              ai[ct] = mul3(x[0], x[1], g[ct][kb][2], g[ct][kb][3], ai[ct]);
              ai[ct] = mul3(x[2], x[3], g[ct][kb][0], g[ct][kb][1], ai[ct]);
            }
          }
        };
        slab_mfma(1, g2, a2r, a2i);  // the partner tile first: its transpose overlaps slab 0
        slab_mfma(0, g1, a1r, a1i);
        // register v of lane (quad, bq) to word v TS-row quad, column 4 v + bq; read back
        // as the 4 words 4 bq .. 4 bq + 3: register v of lane bq then holds register bq of
        // lane v
#pragma unroll
        for (int ct = 0; ct < WT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            XT[wave][ct][0][quad * TS + 4 * v + bq] = a2r[ct][v];
            XT[wave][ct][1][quad * TS + 4 * v + bq] = a2i[ct][v];
          }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
          const v4f tr = *reinterpret_cast<const v4f*>(&XT[wave][ct][0][quad * TS + 4 * bq]);
          const v4f ti = *reinterpret_cast<const v4f*>(&XT[wave][ct][1][quad * TS + 4 * bq]);
          float qr = 0.f, qi = 0.f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            qr = fmaf(a1r[ct][v], tr[v], qr);
            qr = fmaf(-a1i[ct][v], ti[v], qr);
            qi = fmaf(a1r[ct][v], ti[v], qi);
            qi = fmaf(a1i[ct][v], tr[v], qi);
          }
          sr[ct] += (double)qr;
          si[ct] += (double)qi;
        }
      }
      // past the last chunk the stores go to the buffer nobody reads (the barrier below
      // also orders this chunk's transpose reads before the next chunk's writes)
      stash(c + 1, buf ^ 1, pu[(d + 1) % DEPTH]);
      fetch(c + 1 + DEPTH, pu[(d + 1) % DEPTH]);
      __syncthreads();
    }
  }

  // per-walker reduction over the 16 lanes (g_s, b) of a wave with the same walker
#pragma unroll
  for (int ct = 0; ct < WT; ++ct) {
    red[0][tid] = sr[ct];
    red[1][tid] = si[ct];
    __syncthreads();
    if (tid < 16) {
      const int wv = tid >> 2, wsi = tid & 3;
      const int w = chunk * 16 * WT + (wv * WT + ct) * 4 + wsi;
      if (w < W) {
        double ar = 0.0, ai = 0.0;
        for (int gs = 0; gs < 4; ++gs)
          for (int b = 0; b < 4; ++b) {
            const int l = wv * 64 + gs * 16 + wsi * 4 + b;
            ar += red[0][l];
            ai += red[1][l];
          }
        part[(int64_t)t * W + w] = cpx<double>{-mult * ar, -mult * ai};
      }
    }
    __syncthreads();
  }
}

// E1B[w] = 2 sum_k sum_{a,r} h1h[k][a][r] Gh[w][(k a),(k r)];  EC[w] = 1/2 sum X_Q X_-Q;
// EX[w] = sum over canonical triples of the exchange partials.  One workgroup per walker.
struct EfinArgs {
  int nk, m, nocc, C, W;
  KMesh mesh;
  const cpx<double>* h1h;   // [nk][nocc][m]
  const cpx<double>* Gh;    // [W][nk*nocc][nk*m]
  const cpx<double>* X;     // [W][nk][C]
  const cpx<double>* part;  // [nk^3][W]
  cpx<double>* E;           // [W][3]
};

__global__ __launch_bounds__(256) void energy_final_kernel(const Batch<EfinArgs> B) {
  long long wloc;
  const int pb = batch_find(B, blockIdx.x, wloc);
  const int nk = B.a[pb].nk, m = B.a[pb].m, nocc = B.a[pb].nocc, C = B.a[pb].C, W = B.a[pb].W;
  const KMesh mesh = B.a[pb].mesh;
  const cpx<double>* __restrict__ h1h = B.a[pb].h1h;
  const cpx<double>* __restrict__ Gh = B.a[pb].Gh;
  const cpx<double>* __restrict__ X = B.a[pb].X;
  const cpx<double>* __restrict__ part = B.a[pb].part;
  cpx<double>* __restrict__ E = B.a[pb].E;
  const int w = (int)wloc, tid = threadIdx.x;
  __shared__ double red[6][256];
  const int64_t Nn = (int64_t)nk * m, nn = (int64_t)nk * nocc;
  double e1r = 0, e1i = 0, ecr = 0, eci = 0, exr = 0, exi = 0;
  for (int64_t i = tid; i < (int64_t)nk * nocc * m; i += 256) {
    const int kk = (int)(i / (nocc * m)), ar = (int)(i % (nocc * m));
    const int a = ar / m, r = ar % m;
    const cpx<double> h = h1h[i];
    const cpx<double> g = Gh[((int64_t)w * nn + (int64_t)kk * nocc + a) * Nn + (int64_t)kk * m + r];
    e1r += h.re * g.re - h.im * g.im;
    e1i += h.re * g.im + h.im * g.re;
  }
  for (int64_t i = tid; i < (int64_t)nk * C; i += 256) {
    const int Q = (int)(i / C), g = (int)(i % C);
    const cpx<double> x1 = X[((int64_t)w * nk + Q) * C + g];
    const cpx<double> x2 = X[((int64_t)w * nk + mesh.neg(Q)) * C + g];
    ecr += x1.re * x2.re - x1.im * x2.im;
    eci += x1.re * x2.im + x1.im * x2.re;
  }
  const int64_t nt = (int64_t)nk * nk * nk;
  for (int64_t t = tid; t < nt; t += 256) {
    const int kp = (int)(t % nk), k = (int)((t / nk) % nk), Q = (int)(t / ((int64_t)nk * nk));
    const int64_t tp = ((int64_t)mesh.neg(Q) * nk + mesh.kmq(kp, Q)) * nk + mesh.kmq(k, Q);
    if (t > tp) continue;
    const cpx<double> v = part[t * W + w];
    exr += v.re;
    exi += v.im;
  }
  red[0][tid] = e1r; red[1][tid] = e1i; red[2][tid] = ecr;
  red[3][tid] = eci; red[4][tid] = exr; red[5][tid] = exi;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o)
      for (int j = 0; j < 6; ++j) red[j][tid] += red[j][tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    E[3 * (int64_t)w + 0] = cpx<double>{2.0 * red[0][0], 2.0 * red[1][0]};
    E[3 * (int64_t)w + 1] = cpx<double>{0.5 * red[2][0], 0.5 * red[3][0]};
    E[3 * (int64_t)w + 2] = cpx<double>{red[4][0], red[5][0]};
  }
}

// ---------------------------------------------------------------------------
// The exchange on int8 MFMA with exact integer accumulation (energy precisions INT8X5 and
// INT8X4: five or four digits per operand).
//
// The complex contraction T1 = sum_r Lh[a][r][g] G[b][r] is taken as two real products
// over kk < 2m: Re T1 = [Re Lh | Im Lh] . [Re G ; -Im G], Im T1 = [Re Lh | Im Lh] .
// [Im G ; Re G].  Every real row is scaled by a power of two s (|x| < s / 2) and written as
// five signed 7-bit digits, x / s = d1 / 128 + ... + d5 / 128^5 + rest (|d| <= 64, |rest|
// <= 128^-5 / 2): the rows of Lh by prepare, the Gh rows of a workgroup's columns here, in
// registers (INT8X4 keeps four).  The digit products d_i d'_j with i + j <= 6 (5) run on
// the 16x16x64 int8 MFMA and
// are summed exactly in int32 per level i + j (at most five pairs of at most 2 x 64 products
// of |d d'| <= 4096 each: |sum| < 2^22); the levels are combined exactly in FP64 (Horner
// in 128: |D| < 2^49) and scaled by the two powers of two and 128^-6.  What is lost per
// real product is the truncation of both operands and the levels 7 .. 10, at most
// 1.5 * 2^-35 s s' (INT8X4: levels 6 .. 8, 1.25 * 2^-28 s s').  Work decomposition,
// pairing and FP64 sums as in exchange_kernel.
typedef int v4i __attribute__((ext_vector_type(4)));
constexpr int I8_STORE = 5;  // digits per value of the Lh digit rows written by prepare

__device__ __forceinline__ v4i mfma_i8(const v4i& a, const v4i& b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// Digits of x (|x| < 2^(e-1)): x 2^-e = sum_i d_i 128^-(i+1) + rest; each step is exact.
template <int ND>
__device__ __forceinline__ void i8_digits(double x, int e, int (&d)[ND]) {
  double r = ldexp(x, -e);
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    r *= 128.0;
    const double q = rint(r);
    r -= q;
    d[i] = (int)q;
  }
}

// Exponent e of a row whose largest magnitude is amax: 2^(e-2) <= amax < 2^(e-1), or 0 for
// a zero row.
__device__ __forceinline__ int i8_exponent(double amax) {
  return amax > 0.0 ? ilogb(amax) + 2 : 0;
}

// ND digits per operand (5: INT8X5, 4: INT8X4, which reads the first four of the five
// stored Lh digits); the digit products of levels i + j <= ND + 1 are formed.
template <int KB, int ND>
__global__ __launch_bounds__(256) void exchange_int8_kernel(const Batch<ExchArgs> B) {
  constexpr int I8_ND = ND;
  constexpr int KP8 = 64 * KB;           // kk padded to the MFMA K
  constexpr int ROWG = I8_STORE * KP8;   // bytes of one stored (g, a) row
  constexpr int ROWB = I8_ND * KP8;      // digit bytes of one row that the kernel reads
  constexpr int RSB = ROWB + 16;         // LDS row stride (bytes)
  constexpr int UNITS = 2 * 16 * ROWB / 16;         // 16-byte units of one chunk, both slabs
  constexpr int NU = (UNITS + 255) / 256;

  __shared__ __attribute__((aligned(16))) signed char LA[2][2][16][RSB];  // [buf][slab][(g, a)][digit][kk]
  __shared__ int LE[2][2][16];                                        // row exponents
  __shared__ double XB[4][2][16][17];                                 // per-wave exchange tile
  __shared__ double red[2][256];

  long long bid;
  const int pb = batch_find(B, blockIdx.x, bid);
  const int nk = B.a[pb].nk, m = B.a[pb].m, nocc = B.a[pb].nocc, C = B.a[pb].C, W = B.a[pb].W;
  const int nchunk_w = B.a[pb].nchunk_w;
  const KMesh mesh = B.a[pb].mesh;
  const signed char* __restrict__ L8 = (const signed char*)B.a[pb].Lh;
  const int64_t nrows = (int64_t)nk * nk * C * nocc;
  const int* __restrict__ L8e = (const int*)(L8 + nrows * ROWG);
  const cpx<double>* __restrict__ Gh = B.a[pb].Gh;
  cpx<double>* __restrict__ part = B.a[pb].part;
  const int chunk = (int)(bid % nchunk_w);
  const int t = (int)(bid / nchunk_w);
  const int kp = t % nk, k = (t / nk) % nk, Q = t / (nk * nk);
  const int mQ = mesh.neg(Q), kpq = mesh.kmq(kp, Q), kq = mesh.kmq(k, Q);
  const int tp = (mQ * nk + kpq) * nk + kq;  // partner triple (-Q, k'-Q, k-Q)
  if (t > tp) return;
  const double mult = (t == tp) ? 1.0 : 2.0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Gs = 16 / nocc, Ws = 16 / nocc;
  const int col = lane & 15;
  const int ws_l = col / nocc, b_l = col % nocc;
  const int wl = chunk * 4 * Ws + wave * Ws + ws_l;
  const bool colok = (ws_l < Ws) && (wl < W);
  const int64_t Nn = (int64_t)nk * m, nn = (int64_t)nk * nocc;

  // B operands of both GEMMs for this lane's column: positions kk = 64 kb + 16 (lane / 16)
  // + i; the value there is Re/-Im G (first real product) and Im/Re G (second)
  v4i b1r[KB][I8_ND], b1i[KB][I8_ND], b2r[KB][I8_ND], b2i[KB][I8_ND];
  int e1 = 0, e2 = 0;
  bool bad = false;
  {
    // INT8X4: two passes over the column's Gh entries (the second hits the cache), the row
    // maxima first, then the digits, so that no more than one entry is held at a time; the
    // register peak then is the chunk loop's and three waves fit a SIMD.  INT8X5's chunk
    // loop needs more registers than the held entries, so it keeps them from the first pass.
    constexpr bool RELOAD = (I8_ND == 4);
    double hv[RELOAD ? 1 : KB][RELOAD ? 1 : 16][4];
    auto load = [&](int kb, int i, double& x1r, double& x1i, double& x2r, double& x2i) {
      const int pos = 64 * kb + 16 * (lane >> 4) + i;
      const bool re = pos < m;
      const int r = re ? pos : pos - m;
      x1r = 0.0; x1i = 0.0; x2r = 0.0; x2i = 0.0;
      if (colok && pos < 2 * m) {
        const cpx<double> g1 = Gh[((int64_t)wl * nn + (int64_t)kpq * nocc + b_l) * Nn + (int64_t)kq * m + r];
        const cpx<double> g2 = Gh[((int64_t)wl * nn + (int64_t)k * nocc + b_l) * Nn + (int64_t)kp * m + r];
        x1r = re ? g1.re : -g1.im; x1i = re ? g1.im : g1.re;
        x2r = re ? g2.re : -g2.im; x2i = re ? g2.im : g2.re;
      }
    };
    double a1 = 0.0, a2 = 0.0;
    int nf = 0;  // a non-finite entry (fmax would drop a NaN)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double x1r, x1i, x2r, x2i;
        load(kb, i, x1r, x1i, x2r, x2i);
        if constexpr (!RELOAD) {
          hv[kb][i][0] = x1r; hv[kb][i][1] = x1i; hv[kb][i][2] = x2r; hv[kb][i][3] = x2i;
        }
        a1 = fmax(a1, fmax(fabs(x1r), fabs(x1i)));
        a2 = fmax(a2, fmax(fabs(x2r), fabs(x2i)));
        nf |= !(isfinite(x1r) && isfinite(x1i) && isfinite(x2r) && isfinite(x2i));
      }
    // row maxima over the four lane groups holding the same column
    a1 = fmax(a1, __shfl_xor(a1, 16, 64));
    a1 = fmax(a1, __shfl_xor(a1, 32, 64));
    a2 = fmax(a2, __shfl_xor(a2, 16, 64));
    a2 = fmax(a2, __shfl_xor(a2, 32, 64));
    nf |= __shfl_xor(nf, 16, 64);
    nf |= __shfl_xor(nf, 32, 64);
    bad = nf || !isfinite(a1) || !isfinite(a2);
    e1 = bad ? 0 : i8_exponent(a1);
    e2 = bad ? 0 : i8_exponent(a2);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int w1r[I8_ND] = {}, w1i[I8_ND] = {}, w2r[I8_ND] = {}, w2i[I8_ND] = {};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double x1r, x1i, x2r, x2i;
          if constexpr (RELOAD) {
            load(kb, 4 * q + u, x1r, x1i, x2r, x2i);
          } else {
            x1r = hv[kb][4 * q + u][0]; x1i = hv[kb][4 * q + u][1];
            x2r = hv[kb][4 * q + u][2]; x2i = hv[kb][4 * q + u][3];
          }
          int d[I8_ND];
          static_assert(sizeof(d) == I8_ND * sizeof(int), "");
          i8_digits(bad ? 0.0 : x1r, e1, d);
#pragma unroll
          for (int j = 0; j < I8_ND; ++j) w1r[j] |= (d[j] & 0xff) << (8 * u);
          i8_digits(bad ? 0.0 : x1i, e1, d);
#pragma unroll
          for (int j = 0; j < I8_ND; ++j) w1i[j] |= (d[j] & 0xff) << (8 * u);
          i8_digits(bad ? 0.0 : x2r, e2, d);
#pragma unroll
          for (int j = 0; j < I8_ND; ++j) w2r[j] |= (d[j] & 0xff) << (8 * u);
          i8_digits(bad ? 0.0 : x2i, e2, d);
#pragma unroll
          for (int j = 0; j < I8_ND; ++j) w2i[j] |= (d[j] & 0xff) << (8 * u);
        }
#pragma unroll
        for (int j = 0; j < I8_ND; ++j) {
          b1r[kb][j][q] = w1r[j]; b1i[kb][j][q] = w1i[j];
          b2r[kb][j][q] = w2r[j]; b2i[kb][j][q] = w2i[j];
        }
      }
  }

  // slab rows (g, a) of chunk c: rows [(slab C + c Gs) nocc, + Gs nocc) of the digit array
  const int64_t srow0 = ((int64_t)Q * nk + k) * C * nocc;
  const int64_t srow1 = ((int64_t)mQ * nk + kpq) * C * nocc;
  const int nch = (C + Gs - 1) / Gs;
  const int rows = Gs * nocc;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 pu[NU];
  int pe = 0;
  auto fetch = [&](int c) {
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int u = tid + 256 * e;
      const int sl = u / (16 * ROWB / 16), rem = u % (16 * ROWB / 16);
      const int row = rem / (ROWB / 16), off = (rem % (ROWB / 16)) * 16;
      u4 v = {0u, 0u, 0u, 0u};
      if (u < UNITS && row < rows && c * Gs + row / nocc < C)
        v = *reinterpret_cast<const u4*>(L8 + ((sl ? srow1 : srow0) + (int64_t)c * rows + row) * ROWG + off);
      pu[e] = v;
    }
    if (tid < 32) {
      const int sl = tid >> 4, row = tid & 15;
      pe = (row < rows && c * Gs + row / nocc < C) ? L8e[(sl ? srow1 : srow0) + (int64_t)c * rows + row] : 0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NU; ++e) {
      const int u = tid + 256 * e;
      const int sl = u / (16 * ROWB / 16), rem = u % (16 * ROWB / 16);
      const int row = rem / (ROWB / 16), off = (rem % (ROWB / 16)) * 16;
      if (u < UNITS) *reinterpret_cast<u4*>(&LA[buf][sl][row][off]) = pu[e];
    }
    if (tid < 32) LE[buf][tid >> 4][tid & 15] = pe;
  };

  // T1 of one slab on this wave's 16 x 16 tile: rows 4 (lane / 16) + v, column lane % 16
  auto tile = [&](int buf, int sl, const v4i (&br)[KB][I8_ND], const v4i (&bi)[KB][I8_ND],
                  int eb, double (&tr)[4], double (&ti)[4]) {
    v4i cr[I8_ND], ci[I8_ND];
#pragma unroll
    for (int l = 0; l < I8_ND; ++l) { cr[l] = v4i{0, 0, 0, 0}; ci[l] = cr[l]; }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int i = 0; i < I8_ND; ++i) {
        const v4i a = *reinterpret_cast<const v4i*>(&LA[buf][sl][col][i * KP8 + 64 * kb + 16 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j + i < I8_ND; ++j) {
          cr[i + j] = mfma_i8(a, br[kb][j], cr[i + j]);
          ci[i + j] = mfma_i8(a, bi[kb][j], ci[i + j]);
        }
      }
    // D = sum_l acc_l 128^(ND-1-l): levels (0, 1) and (2, 3) pair up exactly in int32
    // (levels 0 and 2 stay below 2^21, every level below 2^21.4: |acc 128 + acc'| < 2^29),
    // the rest is exact in FP64 (|D| < 2^49)
    static_assert(I8_ND == 4 || I8_ND == 5, "level grouping for four or five digits");
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r01 = cr[0][v] * 128 + cr[1][v], r23 = cr[2][v] * 128 + cr[3][v];
      const int i01 = ci[0][v] * 128 + ci[1][v], i23 = ci[2][v] * 128 + ci[3][v];
      double dr = fma((double)r01, 16384.0, (double)r23);
      double di = fma((double)i01, 16384.0, (double)i23);
      if constexpr (I8_ND == 5) {
        dr = fma(dr, 128.0, (double)cr[4][v]);
        di = fma(di, 128.0, (double)ci[4][v]);
      }
      const int ex = LE[buf][sl][4 * (lane >> 4) + v] + eb - 7 * (I8_ND + 1);
      tr[v] = ldexp(dr, ex);
      ti[v] = ldexp(di, ex);
    }
  };

  double sr = 0.0, si = 0.0;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) fetch(c + 1);
    double t2r[4], t2i[4], t1r[4], t1i[4];
    tile(buf, 1, b2r, b2i, e2, t2r, t2i);
    // T1 of the partner triple to the wave-private tile
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * (lane >> 4) + v;
      XB[wave][0][row][col] = t2r[v];
      XB[wave][1][row][col] = t2i[v];
    }
    tile(buf, 0, b1r, b1i, e1, t1r, t1i);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int g0 = c * Gs;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * (lane >> 4) + v;
      const int g_s = row / nocc, a = row % nocc;
      if (colok && g_s < Gs && g0 + g_s < C) {
        const int rp = g_s * nocc + b_l, cp = ws_l * nocc + a;
        const double pr2 = XB[wave][0][rp][cp], pi2 = XB[wave][1][rp][cp];
        sr += t1r[v] * pr2 - t1i[v] * pi2;
        si += t1r[v] * pi2 + t1i[v] * pr2;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (c + 1 < nch) stash(buf ^ 1);
    __syncthreads();
  }
  // a column with a non-finite Green's function entry: a non-finite energy, as in FP64
  if (bad) { sr = __builtin_nan(""); si = sr; }

  // per-walker reduction: lanes of a wave with the same column walker
  red[0][tid] = sr;
  red[1][tid] = si;
  __syncthreads();
  if (tid < 4 * Ws) {
    const int wv = tid / Ws, wsi = tid % Ws;
    const int w = chunk * 4 * Ws + wv * Ws + wsi;
    if (w < W) {
      double ar = 0.0, ai = 0.0;
      for (int grp = 0; grp < 4; ++grp)
        for (int b = 0; b < nocc; ++b) {
          const int l = wv * 64 + grp * 16 + wsi * nocc + b;
          ar += red[0][l];
          ai += red[1][l];
        }
      part[(int64_t)t * W + w] = cpx<double>{-mult * ar, -mult * ai};
    }
  }
}

static size_t carve_energy(Carve& c, const afqmc_kpt_problem& p, void** X, void** parts,
                           void** xpart) {
  Dims d = dims_of(p);
  *X = c.take(16 * (size_t)d.W * d.nk * d.C);
  VbiasWs v;
  carve_vbias(c, d, v);
  *parts = v.parts;
  *xpart = c.take(16 * (size_t)d.nk * d.nk * d.nk * d.W);
  return c.off;
}

size_t energy_ws_bytes(const afqmc_kpt_problem& p) {
  Carve c(nullptr);
  void *a, *b, *x;
  return carve_energy(c, p, &a, &b, &x);
}

static int ks_class(int m) {
  const int KS = (m + 3) / 4;
  return KS <= 4 ? 4 : (KS <= 8 ? 8 : (KS <= 16 ? 16 : -1));
}

// Column tiles (16 / nocc walkers each) per wave of the BF16X3 exchange: two for K = 32
// (the slab of Lh is reused by twice the walkers), one for K = 64 (register budget).
static int exch_bf16_wt(const afqmc_kpt_problem& p) { return p.m <= 32 ? 2 : 1; }

static int exch_nchunk(const afqmc_kpt_problem& p) {
  const int Ws = 16 / p.nocc;
  return (p.nwalk + 4 * Ws - 1) / (4 * Ws);
}

// Exchange partials of every job; one launch per (precision, K-slice class).
static hipError_t launch_exchange(const Job* jobs, int n, void* const* xpart, hipStream_t s) {
  TimedScope ts(KC_EXCHANGE, s);
  return for_groups(
      n,
      [&](int i) {
        const afqmc_kpt_problem& p = jobs[i].p;
        if (jobs[i].int8) return 1024 + 8 * jobs[i].int8 + (p.m <= 32 ? 1 : 2);
        return p.prec * 64 + (p.prec == AFQMC_PREC_BF16X3
                                  ? (p.m <= 32 ? 1 : 2) + (p.nocc == 4 ? 4 : 0)
                                  : ks_class(p.m));
      },
      [&](const int* ids, int c) -> hipError_t {
        Batch<ExchArgs> B;
        B.nprob = c;
        long long cnt[AFQMC_MAXP];
        for (int q = 0; q < c; ++q) {
          const afqmc_kpt_problem& p = jobs[ids[q]].p;
          ExchArgs& a = B.a[q];
          a.nk = p.nk; a.m = p.m; a.nocc = p.nocc; a.C = p.nchol; a.W = p.nwalk;
          a.nchunk_w = exch_nchunk(p);
          if (p.prec == AFQMC_PREC_BF16X3) {
            const int per = 4 * exch_bf16_wt(p) * (16 / p.nocc);
            a.nchunk_w = (p.nwalk + per - 1) / per;
          }
          a.mesh = make_mesh(p);
          a.Lh = (p.prec == AFQMC_PREC_BF16X3) ? p.Lhs : (low_prec(p.prec) ? p.Lh32 : p.Lh);
          if (jobs[ids[q]].int8) a.Lh = p.Lh8;
          a.Gh = (const cpx<double>*)p.Gh;
          a.part = (cpx<double>*)xpart[ids[q]];
          cnt[q] = (long long)p.nk * p.nk * p.nk * a.nchunk_w;
        }
        const long long g = batch_close(B, cnt);
        if (g < 0) return hipErrorInvalidValue;
        if (g == 0) return hipSuccess;
        const bool f32 = low_prec(jobs[ids[0]].p.prec);
        const dim3 grid((unsigned)g), blk(256);
        if (jobs[ids[0]].int8) {
          const bool k1 = jobs[ids[0]].p.m <= 32;
          if (jobs[ids[0]].int8 == 5) {
            if (k1) hipLaunchKernelGGL((exchange_int8_kernel<1, 5>), grid, blk, 0, s, B);
            else hipLaunchKernelGGL((exchange_int8_kernel<2, 5>), grid, blk, 0, s, B);
          } else {
            if (k1) hipLaunchKernelGGL((exchange_int8_kernel<1, 4>), grid, blk, 0, s, B);
            else hipLaunchKernelGGL((exchange_int8_kernel<2, 4>), grid, blk, 0, s, B);
          }
          return hipGetLastError();
        }
        if (jobs[ids[0]].p.prec == AFQMC_PREC_BF16X3) {
          const bool k1 = jobs[ids[0]].p.m <= 32;
          if (jobs[ids[0]].p.nocc == 4) {
            if (k1) hipLaunchKernelGGL((exchange_bf16x3_q4_kernel<1, 2>), grid, blk, 0, s, B);
            else hipLaunchKernelGGL((exchange_bf16x3_q4_kernel<2, 1>), grid, blk, 0, s, B);
          } else {
            if (k1) hipLaunchKernelGGL((exchange_bf16x3_kernel<1, 2>), grid, blk, 0, s, B);
            else hipLaunchKernelGGL((exchange_bf16x3_kernel<2, 1>), grid, blk, 0, s, B);
          }
          return hipGetLastError();
        }
        switch (ks_class(jobs[ids[0]].p.m)) {
          case 4:
            if (f32) hipLaunchKernelGGL((exchange_kernel<float, 4>), grid, blk, 0, s, B);
            else hipLaunchKernelGGL((exchange_kernel<double, 4>), grid, blk, 0, s, B);
            break;
          case 8:
            if (f32) hipLaunchKernelGGL((exchange_kernel<float, 8>), grid, blk, 0, s, B);
            else hipLaunchKernelGGL((exchange_kernel<double, 8>), grid, blk, 0, s, B);
            break;
          case 16:
            if (f32) hipLaunchKernelGGL((exchange_kernel<float, 16>), grid, blk, 0, s, B);
            else hipLaunchKernelGGL((exchange_kernel<double, 16>), grid, blk, 0, s, B);
            break;
          default:
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
      });
}

hipError_t run_energy(const Job* jobs, int n, hipStream_t s) {
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    const Job* J = jobs + c0;
    void *X[AFQMC_MAXP], *parts[AFQMC_MAXP], *xpart[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      Carve cv(J[q].ws);
      carve_energy(cv, J[q].p, &X[q], &parts[q], &xpart[q]);
    }
    hipError_t e = launch_cholesky_trace(J, c, X, nullptr, parts, s);
    if (e != hipSuccess) return e;
    e = launch_exchange(J, c, xpart, s);
    if (e != hipSuccess) return e;
    TimedScope ts(KC_ENERGY_REST, s);
    Batch<EfinArgs> B;
    B.nprob = c;
    long long cnt[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const afqmc_kpt_problem& p = J[q].p;
      EfinArgs& a = B.a[q];
      a.nk = p.nk; a.m = p.m; a.nocc = p.nocc; a.C = p.nchol; a.W = p.nwalk;
      a.mesh = make_mesh(p);
      a.h1h = (const cpx<double>*)p.h1h;
      a.Gh = (const cpx<double>*)p.Gh;
      a.X = (const cpx<double>*)X[q];
      a.part = (const cpx<double>*)xpart[q];
      a.E = (cpx<double>*)J[q].E;
      cnt[q] = p.nwalk;
    }
    const long long g = batch_close(B, cnt);
    if (g < 0) return hipErrorInvalidValue;
    if (g == 0) continue;
    hipLaunchKernelGGL(energy_final_kernel, dim3((unsigned)g), dim3(256), 0, s, B);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!has_pairs(jobs, n)) return hipSuccess;
  // two-determinant walkers: the pair's energy from both halves' closed-shell parts
  std::vector<void*> X(n);
  for (int q = 0; q < n; ++q) {
    Carve cv(jobs[q].ws);
    void *parts, *xpart;
    carve_energy(cv, jobs[q].p, &X[q], &parts, &xpart);
  }
  return run_spin_energy(jobs, n, X.data(), s);
}

// ---------------------------------------------------------------------------
// Mixed estimate: one workgroup per problem, FP64 sums of w E_L and w over the walkers.
struct MixArgs {
  int W;
  const cpx<double>* E;  // [W][3]
  const double* weight;  // [W]
  cpx<double>* out;      // one value
};

__global__ __launch_bounds__(256) void mixed_energy_kernel(const Batch<MixArgs> B) {
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const MixArgs a = B.a[pb];
  const int tid = threadIdx.x;
  __shared__ double red[3][256];
  double sr = 0.0, si = 0.0, sw = 0.0;
  for (int w = tid; w < a.W; w += 256) {
    const double wt = a.weight[w];
    const cpx<double> e0 = a.E[3 * (int64_t)w], e1 = a.E[3 * (int64_t)w + 1],
                      e2 = a.E[3 * (int64_t)w + 2];
    if (wt != 0.0) {  // a zero weight drops the walker even if its energy is not finite
      sr += wt * (e0.re + e1.re + e2.re);
      si += wt * (e0.im + e1.im + e2.im);
      sw += wt;
    }
  }
  red[0][tid] = sr; red[1][tid] = si; red[2][tid] = sw;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) {
      red[0][tid] += red[0][tid + o];
      red[1][tid] += red[1][tid + o];
      red[2][tid] += red[2][tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double s = red[2][0];
    *a.out = (s != 0.0) ? cpx<double>{red[0][0] / s, red[1][0] / s}
                        : cpx<double>{__builtin_nan(""), __builtin_nan("")};
  }
}

hipError_t run_mixed_energy(const Job* jobs, int n, void* Emix, hipStream_t s) {
  TimedScope ts(KC_ENERGY_REST, s);
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    Batch<MixArgs> B;
    B.nprob = c;
    long long cnt[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const Job& j = jobs[c0 + q];
      B.a[q].W = j.p.nwalk;
      B.a[q].E = (const cpx<double>*)j.E;
      B.a[q].weight = j.p.weight;
      B.a[q].out = (cpx<double>*)Emix + c0 + q;
      cnt[q] = 1;
    }
    const long long g = batch_close(B, cnt);
    if (g <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mixed_energy_kernel, dim3((unsigned)g), dim3(256), 0, s, B);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Adjoint.  One workgroup per (k1, k2, walker chunk) accumulates over Q and g
//   K[(w al), rho] = sum_{b,g} T1_{(Q,k1,k2)}[w][b][al][g] Lh[-Q][k2-Q][b][rho][g]
// with T1 recomputed per g chunk (GEMM 1, K = m) and fed through a wave-private LDS tile
// into GEMM 2 (K = (b, g) of the chunk).  The epilogue adds the one-body and Coulomb terms
// and scales by 2 gE[w].
struct BwdArgs {
  int nk, m, nocc, C, W, nchunk_w;
  KMesh mesh;
  const void* Lh;            // [nk][nk][nocc][m][C] in the contraction precision
  const cpx<double>* LhD;    // the same in complex128 (Coulomb term)
  const cpx<double>* h1h;    // [nk][nocc][m]
  const cpx<double>* Gh;     // [W][nk*nocc][nk*m]
  const cpx<double>* X;      // [W][nk][C]
  const cpx<double>* gE;     // [W] or null (gE = 1)
  cpx<double>* gGh;          // like Gh
};

template <typename T, int KSMAX, int MT>
__global__ __launch_bounds__(256) void exchange_bwd_kernel(const Batch<BwdArgs> B) {
  typedef typename mfma16<T>::acc_t acc_t;
  constexpr int RP = 4 * KSMAX;
  constexpr int NC = MT * 16;
  constexpr int NLA = (16 * RP) / 256 > 0 ? (16 * RP) / 256 : 1;
  constexpr int NLB = (16 * NC) / 256;

  __shared__ T LA[2][2][RP][16];      // [buf][re/im][r][(g, al)]
  __shared__ T LB[2][2][16][NC + 1];  // [buf][re/im][(b, g)][rho]
  __shared__ T XB[4][2][16][17];

  long long bid;
  // launch order (consecutive workgroups on different XCDs): neighbouring triples, which
  // share a slab of Lh, run at the same time on all XCDs
  const int pb = batch_find(B, blockIdx.x, bid);
  const int nk = B.a[pb].nk, m = B.a[pb].m, nocc = B.a[pb].nocc, C = B.a[pb].C, W = B.a[pb].W;
  const int nchunk_w = B.a[pb].nchunk_w;
  const KMesh mesh = B.a[pb].mesh;
  const cpx<T>* __restrict__ Lh = (const cpx<T>*)B.a[pb].Lh;
  const cpx<double>* __restrict__ LhD = B.a[pb].LhD;
  const cpx<double>* __restrict__ h1h = B.a[pb].h1h;
  const cpx<double>* __restrict__ Gh = B.a[pb].Gh;
  const cpx<double>* __restrict__ X = B.a[pb].X;
  const cpx<double>* __restrict__ gE = B.a[pb].gE;
  cpx<double>* __restrict__ gGh = B.a[pb].gGh;
  const int chunk = (int)(bid % nchunk_w);
  const int k2 = (int)((bid / nchunk_w) % nk);
  const int k1 = (int)(bid / ((long long)nchunk_w * nk));

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int Gs = 16 / nocc, Ws = 16 / nocc;
  const int KS = (m + 3) >> 2;
  const int col = lane & 15;
  const int ws_l = col / nocc, b_l = col % nocc;
  const int wl = chunk * 4 * Ws + wave * Ws + ws_l;
  const bool colok = (ws_l < Ws) && (wl < W);
  const int64_t Nn = (int64_t)nk * m, nn = (int64_t)nk * nocc;
  const int nch = (C + Gs - 1) / Gs;

  acc_t o_r[MT], o_i[MT];
#pragma unroll
  for (int j = 0; j < MT; ++j) { o_r[j] = mfma16<T>::zero(); o_i[j] = mfma16<T>::zero(); }

  // LDS rows never written by a slab (beyond nocc * Gs) stay zero
  for (int i = tid; i < 2 * 2 * RP * 16; i += 256) (&LA[0][0][0][0])[i] = (T)0;
  for (int i = tid; i < 2 * 2 * 16 * (NC + 1); i += 256) (&LB[0][0][0][0])[i] = (T)0;
  __syncthreads();

  T par[NLA], pai[NLA], pbr[NLB], pbi[NLB];
  for (int Q = 0; Q < nk; ++Q) {
    const int mQ = mesh.neg(Q), kq1 = mesh.kmq(k1, Q), kq2 = mesh.kmq(k2, Q);
    T b1r[KSMAX], b1i[KSMAX];
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) {
      const int r = 4 * s + (lane >> 4);
      T xr = 0, xi = 0;
      if (s < KS && r < m && colok) {
        const cpx<double> g1 =
            Gh[((int64_t)wl * nn + (int64_t)kq2 * nocc + b_l) * Nn + (int64_t)kq1 * m + r];
        xr = (T)g1.re; xi = (T)g1.im;
      }
      b1r[s] = xr; b1i[s] = xi;
    }
    const cpx<T>* sa = Lh + ((int64_t)Q * nk + k1) * nocc * m * C;
    const cpx<T>* sb = Lh + ((int64_t)mQ * nk + kq2) * nocc * m * C;
    // LA element: (r, q = al * Gs + g_s); LB element: (b, rho, g_s), g fastest in memory
    auto fetch = [&](int c) {
      const int g0 = c * Gs;
#pragma unroll
      for (int e = 0; e < NLA; ++e) {
        const int idx = tid + 256 * e;
        const int r = idx / 16, q = idx % 16;
        const int al = q / Gs, g_s = q % Gs;
        T vr = 0, vi = 0;
        if (idx < 16 * RP && al < nocc && r < m && g0 + g_s < C) {
          const cpx<T> v = sa[((int64_t)al * m + r) * C + g0 + g_s];
          vr = v.re; vi = v.im;
        }
        par[e] = vr; pai[e] = vi;
      }
#pragma unroll
      for (int e = 0; e < NLB; ++e) {
        const int idx = tid + 256 * e;
        const int g_s = idx % Gs, rest = idx / Gs;
        const int rho = rest % NC, b = rest / NC;
        T vr = 0, vi = 0;
        if (b < nocc && rho < m && g0 + g_s < C) {
          const cpx<T> v = sb[((int64_t)b * m + rho) * C + g0 + g_s];
          vr = v.re; vi = v.im;
        }
        pbr[e] = vr; pbi[e] = vi;
      }
    };
    auto stash = [&](int buf) {
#pragma unroll
      for (int e = 0; e < NLA; ++e) {
        const int idx = tid + 256 * e;
        const int r = idx / 16, q = idx % 16;
        const int al = q / Gs, g_s = q % Gs;
        if (idx < 16 * RP && al < nocc) {
          LA[buf][0][r][g_s * nocc + al] = par[e];
          LA[buf][1][r][g_s * nocc + al] = pai[e];
        }
      }
#pragma unroll
      for (int e = 0; e < NLB; ++e) {
        const int idx = tid + 256 * e;
        const int g_s = idx % Gs, rest = idx / Gs;
        const int rho = rest % NC, b = rest / NC;
        if (b < nocc) {
          LB[buf][0][b * Gs + g_s][rho] = pbr[e];
          LB[buf][1][b * Gs + g_s][rho] = pbi[e];
        }
      }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      const int buf = c & 1;
      if (c + 1 < nch) fetch(c + 1);
      acc_t tr_ = mfma16<T>::zero(), ti_ = mfma16<T>::zero();
#pragma unroll
      for (int s = 0; s < KSMAX; ++s) {
        if (s < KS) {
          const int r = 4 * s + (lane >> 4);
          cmfma<T>(LA[buf][0][r][col], LA[buf][1][r][col], b1r[s], b1i[s], tr_, ti_);
        }
      }
      // T1 tile: rows (g, al), cols (w, b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = mfma16<T>::drow(lane, v);
        XB[wave][0][row][col] = tr_[v];
        XB[wave][1][row][col] = ti_[v];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // GEMM 2: A[(w, al)][(b, g)] = T1[(g, al)][(w, b)], B[(b, g)][rho] from LB
      const int rw = lane & 15;  // A row for this lane: (w_s, al)
      const int w_s = rw / nocc, al = rw % nocc;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int kk = 4 * ks + (lane >> 4);
        const int b = kk / Gs, g_s = kk % Gs;
        T xr = 0, xi = 0;
        if (w_s < Ws && b < nocc) {
          xr = XB[wave][0][g_s * nocc + al][w_s * nocc + b];
          xi = XB[wave][1][g_s * nocc + al][w_s * nocc + b];
        }
#pragma unroll
        for (int j = 0; j < MT; ++j)
          cmfma<T>(xr, xi, LB[buf][0][kk][j * 16 + col], LB[buf][1][kk][j * 16 + col], o_r[j], o_i[j]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (c + 1 < nch) stash(buf ^ 1);
      __syncthreads();
    }
  }

  // epilogue: rows (w, al), cols rho
  const int Q0 = mesh.kmq(k1, k2);  // k1 - k2
  const int mQ0 = mesh.neg(Q0);
#pragma unroll
  for (int j = 0; j < MT; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = mfma16<T>::drow(lane, v);
      const int w_s = row / nocc, al = row % nocc;
      const int rho = j * 16 + col;
      const int w = chunk * 4 * Ws + wave * Ws + w_s;
      if (w_s >= Ws || w >= W || rho >= m) continue;
      double vr = -(double)o_r[j][v], vi = -(double)o_i[j][v];
      if (k1 == k2) {
        const cpx<double> h = h1h[((int64_t)k1 * nocc + al) * m + rho];
        vr += h.re; vi += h.im;
      }
      const cpx<double>* lc = LhD + ((((int64_t)Q0 * nk + k1) * nocc + al) * m + rho) * C;
      const cpx<double>* xc = X + ((int64_t)w * nk + mQ0) * C;
      double cr = 0, ci = 0;
      for (int g = 0; g < C; ++g) {
        const cpx<double> l = lc[g], x = xc[g];
        cr += l.re * x.re - l.im * x.im;
        ci += l.re * x.im + l.im * x.re;
      }
      vr += cr; vi += ci;
      double sr = 2.0, si = 0.0;
      if (gE) { sr = 2.0 * gE[w].re; si = 2.0 * gE[w].im; }
      gGh[((int64_t)w * nn + (int64_t)k1 * nocc + al) * Nn + (int64_t)k2 * m + rho] =
          cpx<double>{sr * vr - si * vi, sr * vi + si * vr};
    }
}

static size_t carve_backward(Carve& c, const afqmc_kpt_problem& p, void** X, void** parts) {
  Dims d = dims_of(p);
  *X = c.take(16 * (size_t)d.W * d.nk * d.C);
  VbiasWs v;
  carve_vbias(c, d, v);
  *parts = v.parts;
  return c.off;
}

size_t backward_ws_bytes(const afqmc_kpt_problem& p) {
  Carve c(nullptr);
  void *a, *b;
  return carve_backward(c, p, &a, &b);
}

static hipError_t launch_bwd(const Job* jobs, int n, void* const* X, hipStream_t s) {
  TimedScope ts(KC_EXCHANGE_BWD, s);
  return for_groups(
      n,
      [&](int i) {
        return (jobs[i].p.prec * 64 + ks_class(jobs[i].p.m)) * 8 + (jobs[i].p.m + 15) / 16;
      },
      [&](const int* ids, int c) -> hipError_t {
        Batch<BwdArgs> B;
        B.nprob = c;
        long long cnt[AFQMC_MAXP];
        for (int q = 0; q < c; ++q) {
          const Job& j = jobs[ids[q]];
          const afqmc_kpt_problem& p = j.p;
          BwdArgs& a = B.a[q];
          a.nk = p.nk; a.m = p.m; a.nocc = p.nocc; a.C = p.nchol; a.W = p.nwalk;
          a.nchunk_w = exch_nchunk(p);
          a.mesh = make_mesh(p);
          a.Lh = low_prec(p.prec) ? p.Lh32 : p.Lh;
          a.LhD = (const cpx<double>*)p.Lh;
          a.h1h = (const cpx<double>*)p.h1h;
          a.Gh = (const cpx<double>*)p.Gh;
          a.X = (const cpx<double>*)X[ids[q]];
          a.gE = (const cpx<double>*)j.gE;
          a.gGh = (cpx<double>*)j.gGh;
          cnt[q] = (long long)p.nk * p.nk * a.nchunk_w;
        }
        const long long g = batch_close(B, cnt);
        if (g < 0) return hipErrorInvalidValue;
        if (g == 0) return hipSuccess;
        const afqmc_kpt_problem& p0 = jobs[ids[0]].p;
        const bool f32 = low_prec(p0.prec);
        const int ks = ks_class(p0.m), MT = (p0.m + 15) / 16;
        const dim3 grid((unsigned)g), blk(256);
#define AFQMC_BWD(KSV, MTV)                                                                \
  if (ks == KSV && MT == MTV) {                                                            \
    if (f32) hipLaunchKernelGGL((exchange_bwd_kernel<float, KSV, MTV>), grid, blk, 0, s, B); \
    else hipLaunchKernelGGL((exchange_bwd_kernel<double, KSV, MTV>), grid, blk, 0, s, B);    \
    return hipGetLastError();                                                              \
  }
        AFQMC_BWD(4, 1)
        AFQMC_BWD(8, 2)
        AFQMC_BWD(16, 3)
        AFQMC_BWD(16, 4)
#undef AFQMC_BWD
        return hipErrorInvalidValue;
      });
}

hipError_t run_energy_backward(const Job* jobs, int n, hipStream_t s) {
  std::vector<void*> X(n), parts(n);
  for (int q = 0; q < n; ++q) {
    Carve cv(jobs[q].ws);
    carve_backward(cv, jobs[q].p, &X[q], &parts[q]);
  }
  // the traces of every problem first: a two-determinant pair's Coulomb term needs both
  // halves' (the pair's X, the mean of the two closed-shell traces, in both halves' slots)
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    const hipError_t e = launch_cholesky_trace(jobs + c0, c, X.data() + c0, nullptr,
                                               parts.data() + c0, s);
    if (e != hipSuccess) return e;
  }
  const bool pairs = has_pairs(jobs, n);
  if (pairs) {
    std::vector<double*> a, b;
    std::vector<int64_t> cnt;
    for (int i = 0; i + 1 < n; ++i) {
      if (jobs[i].p.spin != AFQMC_SPIN_UP) continue;
      a.push_back((double*)X[i]);
      b.push_back((double*)X[i + 1]);
      cnt.push_back(2 * (int64_t)jobs[i].p.nwalk * jobs[i].p.nk * jobs[i].p.nchol);
    }
    const hipError_t e = run_pair_mean(a.data(), b.data(), cnt.data(), (int)a.size(), s);
    if (e != hipSuccess) return e;
  }
  for (int c0 = 0; c0 < n; c0 += AFQMC_MAXP) {
    const int c = (n - c0 < AFQMC_MAXP) ? n - c0 : AFQMC_MAXP;
    const hipError_t e = launch_bwd(jobs + c0, c, X.data() + c0, s);
    if (e != hipSuccess) return e;
  }
  // each half's closed-shell adjoint with the pair's X is twice that spin's derivative
  return pairs ? run_spin_adjoint_scale(jobs, n, s) : hipSuccess;
}

}  // namespace afqmc
