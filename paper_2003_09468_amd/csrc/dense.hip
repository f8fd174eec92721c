// The standard (dense) representation of a k-point system, on the device.
//
// The paper's standard representation uses one set of Cholesky vectors of the whole
// supercell basis (Nk m orbitals).  With one real field per vector its HS construction
// needs Hermitian vectors; the supercell operators LL_Q of the k-point factorisation are
// Hermitian only for Q = -Q (LL_{-Q} = LL_Q^H, "k-Point Representation"), so each pair
// (Q, -Q) becomes the two Hermitian vectors A = (LL_Q + LL_Q^H) / sqrt 2 and
// B = i (LL_Q - LL_Q^H) / sqrt 2, which carry the same two-body integrals and the same V0.
// The dense system then runs through the same entry points as a 1x1x1 mesh.
#include <math.h>

#include "internal.h"
#include "kcommon.h"

namespace afqmc {

namespace {

// Slot of dense vector gd: the Q (index <= that of -Q) it comes from, whether Q = -Q, and
// its Cholesky index g and part (0: LL_Q or A, 1: B).  Slots in increasing Q, C vectors for
// a self-paired Q, 2C (A then B) for a pair.
struct DenseSlot {
  int Q, self, g, part;
};

__device__ __forceinline__ DenseSlot dense_slot(int gd, int nk, int C, const KMesh& mesh) {
  int base = 0;
  for (int Q = 0; Q < nk; ++Q) {
    const int nq = mesh.neg(Q);
    if (Q > nq) continue;
    const int n = (Q == nq) ? C : 2 * C;
    if (gd < base + n) {
      const int o = gd - base;
      return DenseSlot{Q, Q == nq ? 1 : 0, o % C, o / C};
    }
    base += n;
  }
  return DenseSlot{0, 1, 0, 0};  // not reached for gd < nk C
}

// Ld[P][R][gd] (P = (k p), R = (k' r)) from L[Q][k][p][r][g]: LL_Q[P][R] = L[Q][k][p][r][g]
// when k' = k - Q, else 0.
__global__ void dense_cholesky_kernel(int nk, int m, int C, KMesh mesh,
                                      const cpx<double>* __restrict__ L,
                                      cpx<double>* __restrict__ Ld) {
  const int64_t N = (int64_t)nk * m, G = (int64_t)nk * C;
  const int64_t total = N * N * G;
  const double s2 = 0.70710678118654752440;  // 1 / sqrt 2
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int gd = (int)(i % G);
    const int64_t PR = i / G;
    const int P = (int)(PR / N), R = (int)(PR % N);
    const int k = P / m, p = P % m, kk = R / m, r = R % m;
    const DenseSlot sl = dense_slot(gd, nk, C, mesh);
    // LL_Q[P][R] and LL_Q^H[P][R] = conj(LL_Q[R][P])
    cpx<double> a{0.0, 0.0}, b{0.0, 0.0};
    if (kk == mesh.kmq(k, sl.Q))
      a = L[((((int64_t)sl.Q * nk + k) * m + p) * m + r) * C + sl.g];
    if (k == mesh.kmq(kk, sl.Q)) {
      const cpx<double> t = L[((((int64_t)sl.Q * nk + kk) * m + r) * m + p) * C + sl.g];
      b = cpx<double>{t.re, -t.im};
    }
    cpx<double> v;
    if (sl.self) v = a;
    else if (sl.part == 0) v = cpx<double>{(a.re + b.re) * s2, (a.im + b.im) * s2};
    else v = cpx<double>{-(a.im - b.im) * s2, (a.re - b.re) * s2};  // i (a - b) / sqrt 2
    Ld[i] = v;
  }
}

// H1d[P][R] = H1[k][p][r] for k = k' (else 0); Ad[P][(k' a)] = A[k][p][a] for k = k'.
__global__ void dense_one_body_kernel(int nk, int m, int nocc,
                                      const cpx<double>* __restrict__ H1,
                                      const cpx<double>* __restrict__ A,
                                      cpx<double>* __restrict__ H1d, cpx<double>* __restrict__ Ad) {
  const int64_t N = (int64_t)nk * m, n = (int64_t)nk * nocc;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N * N + N * n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < N * N) {
      const int P = (int)(i / N), R = (int)(i % N);
      const int k = P / m, kk = R / m;
      H1d[i] = (k == kk) ? H1[((int64_t)k * m + P % m) * m + R % m] : cpx<double>{0.0, 0.0};
    } else {
      const int64_t j = i - N * N;
      const int P = (int)(j / n), c = (int)(j % n);
      const int k = P / m, kk = c / nocc;
      Ad[j] = (k == kk) ? A[((int64_t)k * m + P % m) * nocc + c % nocc] : cpx<double>{0.0, 0.0};
    }
  }
}

// Dense fields xd[w][0][gd][+/-] from x[w][Q][g][+/-]: for a pair,
// x_A = (x+_Q + x+_{-Q}) / sqrt 2, x_B = (x-_{-Q} - x-_Q) / sqrt 2; for Q = -Q, x+_Q; the
// minus fields of the Hermitian vectors are 0.
__global__ void dense_fields_kernel(int W, int nk, int C, KMesh mesh,
                                    const double* __restrict__ x, double* __restrict__ xd) {
  const int64_t G = (int64_t)nk * C, total = (int64_t)W * G;
  const double s2 = 0.70710678118654752440;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int gd = (int)(i % G);
    const int64_t w = i / G;
    const DenseSlot sl = dense_slot(gd, nk, C, mesh);
    const double* xw = x + w * G * 2;
    const int mq = mesh.neg(sl.Q);
    double v;
    if (sl.self) v = xw[((int64_t)sl.Q * C + sl.g) * 2 + 0];
    else if (sl.part == 0)
      v = (xw[((int64_t)sl.Q * C + sl.g) * 2 + 0] + xw[((int64_t)mq * C + sl.g) * 2 + 0]) * s2;
    else
      v = (xw[((int64_t)mq * C + sl.g) * 2 + 1] - xw[((int64_t)sl.Q * C + sl.g) * 2 + 1]) * s2;
    xd[i * 2 + 0] = v;
    xd[i * 2 + 1] = 0.0;
  }
}

}  // namespace

hipError_t run_dense_system(const afqmc_kpt_problem& p, const void* H1, void* Ld, void* H1d,
                            void* Ad, hipStream_t s) {
  hipLaunchKernelGGL(dense_cholesky_kernel, dim3(4096), dim3(256), 0, s, p.nk, p.m, p.nchol,
                     make_mesh(p), (const cpx<double>*)p.L, (cpx<double>*)Ld);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dense_one_body_kernel, dim3(256), dim3(256), 0, s, p.nk, p.m, p.nocc,
                     (const cpx<double>*)H1, (const cpx<double>*)p.A, (cpx<double>*)H1d,
                     (cpx<double>*)Ad);
  return hipGetLastError();
}

hipError_t run_dense_fields(const afqmc_kpt_problem& p, const double* x, double* xd,
                            hipStream_t s) {
  hipLaunchKernelGGL(dense_fields_kernel, dim3(512), dim3(256), 0, s, p.nwalk, p.nk, p.nchol,
                     make_mesh(p), x, xd);
  return hipGetLastError();
}

}  // namespace afqmc
