// Non-uniform band counts per k-point.
//
// The k-point representation counts an average number of bands per k-point; with mk[k]
// bands at k the Cholesky block (Q, k) is mk[k] x mk[k-Q] and the one-body block at k is
// mk[k] x mk[k].  The library's kernels take one band count m for every k-point: a ragged
// system enters as the uniform system with m >= max mk bands whose extra bands are zero
// rows and columns of L, H1 and the trial and zero rows of the walkers.  Those bands carry
// no matrix element, so the propagator keeps the walkers' zero rows zero (its one-body
// factor is the identity there, its two-body exponent zero), and every overlap, trace and
// contraction of the method is that of the ragged system.  The kernels here write the
// padded arrays from packed ragged ones, and the ragged walkers and Green's functions back.
#include "internal.h"
#include "kcommon.h"

namespace afqmc {

namespace {

// Band tables of one call: counts, prefix offsets of the packed blocks (kernel arguments,
// nk <= AFQMC_PAD_MAX_NK).
struct PadTab {
  int nk, m, nocc, C, W;
  KMesh mesh;
  unsigned char mk[AFQMC_PAD_MAX_NK];
  int64_t koff[AFQMC_PAD_MAX_NK + 1];  // sum_{k' < k} mk[k']            (bands before k)
  int64_t hoff[AFQMC_PAD_MAX_NK + 1];  // sum_{k' < k} mk[k']^2          (H1 blocks)
  int64_t qoff[AFQMC_PAD_MAX_NK + 1];  // sum_{Q' < Q} sum_k mk[k] mk[k-Q'] nchol (L rows of Q)
};

// One workgroup per (Q, k) block of the padded L.
__global__ __launch_bounds__(256) void pad_l_kernel(const PadTab t,
                                                    const cpx<double>* __restrict__ src,
                                                    cpx<double>* __restrict__ dst) {
  const int Q = blockIdx.x / t.nk, k = blockIdx.x % t.nk;
  __shared__ int64_t base;
  if (threadIdx.x == 0) {
    int64_t o = t.qoff[Q];
    for (int kk = 0; kk < k; ++kk) o += (int64_t)t.mk[kk] * t.mk[t.mesh.kmq(kk, Q)] * t.C;
    base = o;
  }
  __syncthreads();
  const int mr = t.mk[k], mc = t.mk[t.mesh.kmq(k, Q)];
  const int64_t nblk = (int64_t)t.m * t.m * t.C;
  cpx<double>* out = dst + (int64_t)blockIdx.x * nblk;
  for (int64_t i = threadIdx.x; i < nblk; i += 256) {
    const int g = (int)(i % t.C);
    const int64_t pr = i / t.C;
    const int p = (int)(pr / t.m), r = (int)(pr % t.m);
    out[i] = (p < mr && r < mc) ? src[base + ((int64_t)p * mc + r) * t.C + g]
                                : cpx<double>{0.0, 0.0};
  }
}

// H1 [nk][m][m] and A [nk][m][nocc] from their packed blocks (grid-stride).
__global__ __launch_bounds__(256) void pad_h1_a_kernel(const PadTab t,
                                                       const cpx<double>* __restrict__ H1r,
                                                       const cpx<double>* __restrict__ Ar,
                                                       cpx<double>* __restrict__ H1,
                                                       cpx<double>* __restrict__ A) {
  const int64_t nh = H1 ? (int64_t)t.nk * t.m * t.m : 0;
  const int64_t na = A ? (int64_t)t.nk * t.m * t.nocc : 0;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < nh + na; i += gridDim.x * 256LL) {
    if (i < nh) {
      const int k = (int)(i / ((int64_t)t.m * t.m));
      const int p = (int)((i / t.m) % t.m), q = (int)(i % t.m);
      const int mq = t.mk[k];
      H1[i] = (p < mq && q < mq) ? H1r[t.hoff[k] + (int64_t)p * mq + q] : cpx<double>{0.0, 0.0};
    } else {
      const int64_t j = i - nh;
      const int k = (int)(j / ((int64_t)t.m * t.nocc));
      const int p = (int)((j / t.nocc) % t.m), a = (int)(j % t.nocc);
      A[j] = (p < t.mk[k]) ? Ar[(t.koff[k] + p) * t.nocc + a] : cpx<double>{0.0, 0.0};
    }
  }
}

// Walkers: padded [W][nk m][n] from ragged [W][sum mk][n] (to_pad), or back.
__global__ __launch_bounds__(256) void pad_u_kernel(const PadTab t, bool to_pad,
                                                    const cpx<double>* __restrict__ src,
                                                    cpx<double>* __restrict__ dst) {
  const int64_t n = (int64_t)t.nk * t.nocc, Mp = (int64_t)t.nk * t.m, Mr = t.koff[t.nk];
  const int64_t total = (int64_t)t.W * (to_pad ? Mp : Mr) * n;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < total; i += gridDim.x * 256LL) {
    const int64_t j = i % n, row = (i / n) % (to_pad ? Mp : Mr), w = i / (n * (to_pad ? Mp : Mr));
    if (to_pad) {
      const int k = (int)(row / t.m), p = (int)(row % t.m);
      dst[i] = (p < t.mk[k]) ? src[(w * Mr + t.koff[k] + p) * n + j] : cpx<double>{0.0, 0.0};
    } else {
      int k = 0;  // the k-point of ragged row `row`
      while (k + 1 < t.nk && t.koff[k + 1] <= row) ++k;
      dst[i] = src[(w * Mp + (int64_t)k * t.m + (row - t.koff[k])) * n + j];
    }
  }
}

// Half-rotated Green's functions: padded [W][n][nk m] -> ragged [W][n][sum mk].
__global__ __launch_bounds__(256) void unpad_gh_kernel(const PadTab t,
                                                       const cpx<double>* __restrict__ src,
                                                       cpx<double>* __restrict__ dst) {
  const int64_t n = (int64_t)t.nk * t.nocc, Mp = (int64_t)t.nk * t.m, Mr = t.koff[t.nk];
  const int64_t total = (int64_t)t.W * n * Mr;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < total; i += gridDim.x * 256LL) {
    const int64_t col = i % Mr, row = i / Mr;  // row = w n + a
    int k = 0;
    while (k + 1 < t.nk && t.koff[k + 1] <= col) ++k;
    dst[i] = src[row * Mp + (int64_t)k * t.m + (col - t.koff[k])];
  }
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

PadTab make_tab(const afqmc_kpt_problem& p, const int32_t* mk) {
  PadTab t;
  t.nk = p.nk; t.m = p.m; t.nocc = p.nocc; t.C = p.nchol; t.W = p.nwalk;
  t.mesh = make_mesh(p);
  t.koff[0] = t.hoff[0] = t.qoff[0] = 0;
  for (int k = 0; k < p.nk; ++k) {
    t.mk[k] = (unsigned char)mk[k];
    t.koff[k + 1] = t.koff[k] + mk[k];
    t.hoff[k + 1] = t.hoff[k] + (int64_t)mk[k] * mk[k];
  }
  for (int Q = 0; Q < p.nk; ++Q) {
    int64_t s = 0;
    for (int k = 0; k < p.nk; ++k) s += (int64_t)mk[k] * mk[t.mesh.kmq(k, Q)] * p.nchol;
    t.qoff[Q + 1] = t.qoff[Q] + s;
  }
  return t;
}

}  // namespace

hipError_t run_pad_bands(const afqmc_kpt_problem& p, const int32_t* mk, const void* Lr,
                         const void* H1r, const void* Ar, const void* Ur, void* L, void* H1,
                         void* A, void* U, hipStream_t s) {
  const PadTab t = make_tab(p, mk);
  if (Lr) {
    hipLaunchKernelGGL(pad_l_kernel, dim3((unsigned)(p.nk * p.nk)), dim3(256), 0, s, t,
                       (const cpx<double>*)Lr, (cpx<double>*)L);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (H1r || Ar) {
    const int64_t n = (H1r ? (int64_t)p.nk * p.m * p.m : 0) + (Ar ? (int64_t)p.nk * p.m * p.nocc : 0);
    hipLaunchKernelGGL(pad_h1_a_kernel, dim3(grid_for(n)), dim3(256), 0, s, t,
                       (const cpx<double>*)H1r, (const cpx<double>*)Ar,
                       H1r ? (cpx<double>*)H1 : nullptr, Ar ? (cpx<double>*)A : nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (Ur) {
    const int64_t n = (int64_t)p.nwalk * p.nk * p.m * p.nk * p.nocc;
    hipLaunchKernelGGL(pad_u_kernel, dim3(grid_for(n)), dim3(256), 0, s, t, true,
                       (const cpx<double>*)Ur, (cpx<double>*)U);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_unpad_bands(const afqmc_kpt_problem& p, const int32_t* mk, const void* U,
                           const void* Gh, void* Ur, void* Ghr, hipStream_t s) {
  const PadTab t = make_tab(p, mk);
  const int64_t n = (int64_t)p.nwalk * t.koff[p.nk] * p.nk * p.nocc;
  if (U) {
    hipLaunchKernelGGL(pad_u_kernel, dim3(grid_for(n)), dim3(256), 0, s, t, false,
                       (const cpx<double>*)U, (cpx<double>*)Ur);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (Gh) {
    hipLaunchKernelGGL(unpad_gh_kernel, dim3(grid_for(n)), dim3(256), 0, s, t,
                       (const cpx<double>*)Gh, (cpx<double>*)Ghr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace afqmc
