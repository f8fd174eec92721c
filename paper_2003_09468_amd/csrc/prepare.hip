// One-time preparation of the static data (k-point section: half-transformed Cholesky
// matrix; introduction: one-body propagator exp(-dt/2 H1') with H1' = H1 + v0).
//
//   Lh[Q][k][a][r][g] = sum_p conj(A[k][p][a]) L[Q][k][p][r][g]      (batched GEMM)
//   h1h[k]            = A[k]^H H1[k]                                 (batched GEMM)
//   V0[k]             = -1/2 sum_{Q,g} L[Q][k][:,:,g] L[Q][k][:,:,g]^H (GEMM, K = nk*m*nchol)
//   bhalf[k]          = exp(-dt/2 (H1[k] + V0[k]))
// The exponential uses the Taylor series with scaling and squaring (Moler and Van Loan,
// "Nineteen dubious ways to compute the exponential of a matrix"): the matrix is scaled
// by 2^-s so that its 1-norm is at most 1/4, summed to 18th order (remainder below 1e-27
// relative) and squared s times, all in FP64.
#include <math.h>

#include "cgemm.h"
#include "internal.h"

namespace afqmc {

// Y[b][row][col] = sum_p conj(A[kb][p][row]) X[b][p][col]; batch b over (Q, k) or k.
struct OpHalfRot {
  typedef double T;
  static constexpr bool A_KCONTIG = false;  // A(row=a, k=p) = conj(A[k][p][a]): along a
  static constexpr bool B_NCONTIG = true;
  int M, N, K, nbatch;  // M = nocc, K = m, N = cols of X
  int nk;
  const cpx<double>* Atr;  // [nk][m][nocc]
  const cpx<double>* X;    // [nbatch][m][N]
  cpx<double>* Y;          // [nbatch][nocc][N]
  cpx<float>* Y32;         // optional complex64 copy
  __device__ void load_a(int b, int row, int k, double& re, double& im) const {
    const cpx<double> v = Atr[((int64_t)(b % nk) * K + k) * M + row];
    re = v.re; im = -v.im;
  }
  __device__ void load_b(int b, int k, int col, double& re, double& im) const {
    const cpx<double> v = X[((int64_t)b * K + k) * N + col];
    re = v.re; im = v.im;
  }
  __device__ void store(int b, int row, int col, double re, double im) const {
    const int64_t idx = ((int64_t)b * M + row) * N + col;
    Y[idx] = cpx<double>{re, im};
    if (Y32) Y32[idx] = cpx<float>{(float)re, (float)im};
  }
};

// V0[k][p][q] = -1/2 sum_{Q, (r g)} L[Q][k][p][(r g)] conj(L[Q][k][q][(r g)])
struct OpV0 {
  typedef double T;
  static constexpr bool A_KCONTIG = true;
  static constexpr bool B_NCONTIG = false;
  int M, N, K, nbatch;  // M = N = m, K = nk * m * C, nbatch = nk
  int nk, m;
  int64_t mc;  // m * C
  const cpx<double>* L;
  cpx<double>* V0;
  __device__ const cpx<double>& at(int kb, int row, int k) const {
    const int Q = (int)(k / mc);
    const int64_t rg = k % mc;
    return L[(((int64_t)Q * nk + kb) * m + row) * mc + rg];
  }
  __device__ void load_a(int b, int row, int k, double& re, double& im) const {
    const cpx<double> v = at(b, row, k);
    re = v.re; im = v.im;
  }
  __device__ void load_b(int b, int k, int col, double& re, double& im) const {
    const cpx<double> v = at(b, col, k);
    re = v.re; im = -v.im;
  }
  __device__ void store(int b, int row, int col, double re, double im) const {
    V0[((int64_t)b * M + row) * N + col] = cpx<double>{-0.5 * re, -0.5 * im};
  }
};

__global__ void to_c64_kernel(int64_t n, const cpx<double>* __restrict__ x, cpx<float>* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = cpx<float>{(float)x[i].re, (float)x[i].im};
}

// BF16 split planes of Lh for the three-pass exchange:
//   Lhs[Q][k][g][a][plane][r], planes (re hi, re lo, im hi, im lo) of the FP32-rounded
//   value, hi = bf16(x), lo = bf16(x - hi) (round to nearest even), r padded to KP with 0.
__global__ void lh_split_kernel(int nk, int m, int nocc, int C, int KP,
                                const cpx<double>* __restrict__ Lh,
                                unsigned short* __restrict__ Lhs) {
  const int64_t total = (int64_t)nk * nk * C * nocc * KP;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i % KP);
    const int a = (int)((i / KP) % nocc);
    const int g = (int)((i / ((int64_t)KP * nocc)) % C);
    const int64_t qk = i / ((int64_t)KP * nocc * C);
    float xr = 0.f, xi = 0.f;
    if (r < m) {
      const cpx<double> v = Lh[((qk * nocc + a) * m + r) * C + g];
      xr = (float)v.re;
      xi = (float)v.im;
    }
    unsigned short rh, rl, ih, il;
    bf16_split(xr, rh, rl);
    bf16_split(xi, ih, il);
    unsigned short* o = Lhs + ((((qk * C + g) * nocc + a) * 4) * KP + r);
    o[0] = rh;
    o[KP] = rl;
    o[2 * KP] = ih;
    o[3 * KP] = il;
  }
}

// Int8 digits of Lh for the INT8X5 exchange: row (Q, k, g, a) over kk < KP8 of
// [Re Lh[Q][k][a][:][g] | Im Lh[Q][k][a][:][g] | 0], scaled by 2^e (2^(e-2) <= max |x| <
// 2^(e-1)) and cut into five signed 7-bit digits x 2^-e = sum_i d_i 128^-(i+1) + rest (each
// step exact: multiply by 128, round to nearest, subtract).  One thread per row.
__global__ void lh_int8_kernel(int nk, int m, int nocc, int C, int KP8,
                               const cpx<double>* __restrict__ Lh, signed char* __restrict__ L8) {
  constexpr int ND = 5;
  const int64_t nrows = (int64_t)nk * nk * C * nocc;
  int* __restrict__ ex = (int*)(L8 + nrows * ND * KP8);
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < nrows;
       row += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(row % nocc);
    const int g = (int)((row / nocc) % C);
    const int64_t qk = row / ((int64_t)nocc * C);
    const cpx<double>* src = Lh + (qk * nocc + a) * m * C + g;  // element r at src[r * C]
    double amax = 0.0;
    for (int r = 0; r < m; ++r) {
      const cpx<double> v = src[(int64_t)r * C];
      amax = fmax(amax, fmax(fabs(v.re), fabs(v.im)));
    }
    const int e = amax > 0.0 ? ilogb(amax) + 2 : 0;
    ex[row] = e;
    signed char* o = L8 + row * ND * KP8;
    for (int kk = 0; kk < KP8; ++kk) {
      double x = 0.0;
      if (kk < m) x = src[(int64_t)kk * C].re;
      else if (kk < 2 * m) x = src[(int64_t)(kk - m) * C].im;
      double r = ldexp(x, -e);
      for (int i = 0; i < ND; ++i) {
        r *= 128.0;
        const double q = rint(r);
        r -= q;
        o[i * KP8 + kk] = (signed char)(int)q;
      }
    }
  }
}

// The Q of each slot of the half store (the Q with index <= that of -Q, increasing); one
// thread.
__global__ void ls_slot_kernel(int nk, KMesh mesh, int* __restrict__ slotq) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int s = 0;
  for (int Q = 0; Q < nk; ++Q)
    if (Q <= mesh.neg(Q)) slotq[s++] = Q;
}

// BF16 split planes of L for the three-pass HS potential, half store, by chunks of 32 g:
//   Ls[slot][g / 32][(k p r)][plane][g % 32] = split of L[Q(slot)][k][p][r][g], g
//   zero-padded to CP = 32 ceil(C / 32), so that one chunk of consecutive columns is one
//   contiguous block.
__global__ void l_split_kernel(int64_t ncols, int64_t ncq, int C, int CP,
                               const cpx<double>* __restrict__ L, const int* __restrict__ slotq,
                               unsigned short* __restrict__ Ls) {
  const int64_t total = ncols * CP;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(i % CP);
    const int64_t cg = i / CP;  // (slot, k, p, r)
    const int64_t Q = cg / ncq, col = cg % ncq;
    float xr = 0.f, xi = 0.f;
    if (g < C) {
      const cpx<double> v = L[((int64_t)slotq[Q] * ncq + col) * C + g];
      xr = (float)v.re;
      xi = (float)v.im;
    }
    unsigned short rh, rl, ih, il;
    bf16_split(xr, rh, rl);
    bf16_split(xi, ih, il);
    unsigned short* o = Ls + ((((Q * (CP / 32) + g / 32) * ncq + col) * 4) * 32 + (g % 32));
    o[0] = rh;
    o[32] = rl;
    o[64] = ih;
    o[96] = il;
  }
}

// One workgroup per k.  Scratch: [nk][4][m][m] complex128 (X, T, E, tmp).
__global__ __launch_bounds__(256) void expm_kernel(int m, double scale,
                                                   const cpx<double>* __restrict__ H1,
                                                   const cpx<double>* __restrict__ V0,
                                                   cpx<double>* __restrict__ scr,
                                                   cpx<double>* __restrict__ out) {
  const int k = blockIdx.x, tid = threadIdx.x;
  const int mm = m * m;
  cpx<double>* X = scr + (int64_t)k * 4 * mm;
  cpx<double>* Tm = X + mm;
  cpx<double>* E = Tm + mm;
  cpx<double>* Y = E + mm;
  __shared__ double red[256];
  __shared__ int s_sh;
  // X = scale * (H1 + V0)
  for (int i = tid; i < mm; i += 256) {
    const cpx<double> h = H1[(int64_t)k * mm + i], v = V0[(int64_t)k * mm + i];
    X[i] = cpx<double>{scale * (h.re + v.re), scale * (h.im + v.im)};
  }
  __syncthreads();
  // 1-norm (max column sum)
  double cmax = 0.0;
  for (int c = tid; c < m; c += 256) {
    double sum = 0.0;
    for (int r = 0; r < m; ++r) sum += hypot(X[r * m + c].re, X[r * m + c].im);
    cmax = fmax(cmax, sum);
  }
  red[tid] = cmax;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) red[tid] = fmax(red[tid], red[tid + o]);
    __syncthreads();
  }
  if (tid == 0) {
    int s = 0;
    double nrm = red[0];
    while (nrm > 0.25 && s < 60) { nrm *= 0.5; ++s; }
    s_sh = s;
  }
  __syncthreads();
  const int s = s_sh;
  const double f = ldexp(1.0, -s);
  for (int i = tid; i < mm; i += 256) {
    X[i].re *= f; X[i].im *= f;
    const int r = i / m, c = i % m;
    Tm[i] = X[i];
    E[i] = cpx<double>{X[i].re + (r == c ? 1.0 : 0.0), X[i].im};
  }
  __syncthreads();
  for (int j = 2; j <= 18; ++j) {
    // Y = X T / j
    for (int i = tid; i < mm; i += 256) {
      const int r = i / m, c = i % m;
      double ar = 0, ai = 0;
      for (int q = 0; q < m; ++q) {
        const cpx<double> a = X[r * m + q], b = Tm[q * m + c];
        ar += a.re * b.re - a.im * b.im;
        ai += a.re * b.im + a.im * b.re;
      }
      Y[i] = cpx<double>{ar / j, ai / j};
    }
    __syncthreads();
    for (int i = tid; i < mm; i += 256) {
      Tm[i] = Y[i];
      E[i].re += Y[i].re;
      E[i].im += Y[i].im;
    }
    __syncthreads();
  }
  for (int it = 0; it < s; ++it) {
    for (int i = tid; i < mm; i += 256) {
      const int r = i / m, c = i % m;
      double ar = 0, ai = 0;
      for (int q = 0; q < m; ++q) {
        const cpx<double> a = E[r * m + q], b = E[q * m + c];
        ar += a.re * b.re - a.im * b.im;
        ai += a.re * b.im + a.im * b.re;
      }
      Y[i] = cpx<double>{ar, ai};
    }
    __syncthreads();
    for (int i = tid; i < mm; i += 256) E[i] = Y[i];
    __syncthreads();
  }
  for (int i = tid; i < mm; i += 256) out[(int64_t)k * mm + i] = E[i];
}

size_t prepare_ws_bytes(const afqmc_kpt_problem& p) {
  return align_up(16 * (size_t)p.nk * p.m * p.m) + align_up(16 * 4 * (size_t)p.nk * p.m * p.m);
}

hipError_t run_prepare(const afqmc_kpt_problem& p, const void* H1, void* ws, hipStream_t s) {
  Carve c(ws);
  void* V0 = c.take(16 * (size_t)p.nk * p.m * p.m);
  void* scr = c.take(16 * 4 * (size_t)p.nk * p.m * p.m);
  // the reduced copies that the step and the energy precision read
  const int sp = step_prec(p.prec), ep = energy_prec(p.prec);
  const bool f32 = low_prec(sp) || low_prec(ep);
  hipError_t e;
  {  // Lh = A^H L, batch (Q, k)
    OpHalfRot op;
    op.M = p.nocc; op.K = p.m; op.N = p.m * p.nchol;
    op.nbatch = p.nk * p.nk;
    op.nk = p.nk;
    op.Atr = (const cpx<double>*)p.A;
    op.X = (const cpx<double>*)p.L;
    op.Y = (cpx<double>*)p.Lh;
    op.Y32 = f32 ? (cpx<float>*)p.Lh32 : nullptr;
    e = launch_cgemm<16, 64, 16, 1, 4>(op, s);
    if (e != hipSuccess) return e;
  }
  {  // h1h = A^H H1, batch k
    OpHalfRot op;
    op.M = p.nocc; op.K = p.m; op.N = p.m;
    op.nbatch = p.nk;
    op.nk = p.nk;
    op.Atr = (const cpx<double>*)p.A;
    op.X = (const cpx<double>*)H1;
    op.Y = (cpx<double>*)p.h1h;
    op.Y32 = nullptr;
    e = launch_cgemm<16, 64, 16, 1, 4>(op, s);
    if (e != hipSuccess) return e;
  }
  {  // V0
    OpV0 op;
    op.M = p.m; op.N = p.m;
    op.K = p.nk * p.m * p.nchol;
    op.nbatch = p.nk;
    op.nk = p.nk; op.m = p.m;
    op.mc = (int64_t)p.m * p.nchol;
    op.L = (const cpx<double>*)p.L;
    op.V0 = (cpx<double>*)V0;
    e = launch_cgemm<32, 32, 16, 2, 2>(op, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(expm_kernel, dim3(p.nk), dim3(256), 0, s, p.m, -0.5 * p.dt,
                     (const cpx<double>*)H1, (const cpx<double>*)V0, (cpx<double>*)scr,
                     (cpx<double>*)p.bhalf);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (sp == AFQMC_PREC_FP32) {  // BF16X3 reads the split planes of L instead
    const int64_t n = (int64_t)p.nk * p.nk * p.m * p.m * p.nchol;
    hipLaunchKernelGGL(to_c64_kernel, dim3(4096), dim3(256), 0, s, n, (const cpx<double>*)p.L,
                       (cpx<float>*)p.L32);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (sp == AFQMC_PREC_BF16X3 || ep == AFQMC_PREC_BF16X3) {
    const int KP = 32 * ((p.m + 31) / 32);
    hipLaunchKernelGGL(lh_split_kernel, dim3(4096), dim3(256), 0, s, p.nk, p.m, p.nocc,
                       p.nchol, KP, (const cpx<double>*)p.Lh, (unsigned short*)p.Lhs);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (int8_digits(ep)) {  // five digits stored; INT8X4 reads the first four
    const int KP8 = 64 * ((2 * p.m + 63) / 64);
    hipLaunchKernelGGL(lh_int8_kernel, dim3(2048), dim3(256), 0, s, p.nk, p.m, p.nocc, p.nchol,
                       KP8, (const cpx<double>*)p.Lh, (signed char*)p.Lh8);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (sp == AFQMC_PREC_BF16X3) {
    const int CP = 32 * ((p.nchol + 31) / 32);
    const int64_t ncq = (int64_t)p.nk * p.m * p.m, ncols = ls_slots(p) * ncq;
    int* slotq = (int*)((char*)p.Ls + ls_plane_bytes(p));
    hipLaunchKernelGGL(ls_slot_kernel, dim3(1), dim3(64), 0, s, p.nk, make_mesh(p), slotq);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(l_split_kernel, dim3(4096), dim3(256), 0, s, ncols, ncq, p.nchol, CP,
                       (const cpx<double>*)p.L, (const int*)slotq, (unsigned short*)p.Ls);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace afqmc
