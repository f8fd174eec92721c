// Two-determinant (collinear, spin-unrestricted) walkers.
//
// The Hamiltonian sums over the spins of both electrons ("Introduction to AFQMC").  A
// closed-shell walker keeps one determinant for both spins; a collinear walker keeps one
// per spin, each against its own block-diagonal trial, in the same single-particle basis
// (spin-independent one-body blocks and Cholesky vectors, "k-Point Representation").  The
// library holds such a walker set as two problems, the up half directly followed by the
// down half.  Every stage runs on each half as for a closed shell, whose factors assume
// two equal spins:
//   force bias: X_cs = 2 tr(Lh^s Gh^s), the pair's X = tr(Lh^up Gh^up) + tr(Lh^dn Gh^dn)
//               = (X_cs^up + X_cs^dn) / 2, and the same mean for xbar (linear in X);
//   one-body and exchange energies: the closed shell's are twice one spin's, the pair's
//               are the sums over the spins = the means of the two halves' values;
//   Coulomb energy: 1/2 sum_{Q,g} X_Q X_-Q of the pair's X (not of either half's);
//   adjoint: dE/dGh^s = h1h^s + Lh^s X - exchange^s of the pair's X = half the closed
//               shell's expression evaluated with X_cs := the pair's X.
// The kernels here apply these couplings between the halves' stages; the weight update
// of a pair (the product of the two overlaps) is in the weight kernel.
#include <vector>

#include "internal.h"
#include "kcommon.h"

namespace afqmc {

namespace {

// a[i] = b[i] = (a[i] + b[i]) / 2 over n doubles
struct PairMeanArgs {
  double* a;
  double* b;
  int64_t n;
  long long nblk;
};

__global__ __launch_bounds__(256) void pair_mean_kernel(const Batch<PairMeanArgs> B) {
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const PairMeanArgs a = B.a[pb];
  for (int64_t i = loc * 256 + threadIdx.x; i < a.n; i += a.nblk * 256) {
    const double v = 0.5 * (a.a[i] + a.b[i]);
    a.a[i] = v;
    a.b[i] = v;
  }
}

// a[i] *= f over n doubles
struct ScaleArgs {
  double* a;
  int64_t n;
  double f;
  long long nblk;
};

__global__ __launch_bounds__(256) void scale_kernel(const Batch<ScaleArgs> B) {
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const ScaleArgs a = B.a[pb];
  for (int64_t i = loc * 256 + threadIdx.x; i < a.n; i += a.nblk * 256) a.a[i] *= a.f;
}

// One workgroup per walker of a pair: E1 and EX the means of the halves' closed-shell
// values, EC = 1/2 sum_{Q,g} X_Qg X_{-Q}g with X = (X_cs^up + X_cs^dn) / 2; both halves'
// rows receive the pair's energy.
struct SpinEnergyArgs {
  int W, nk, C;
  KMesh mesh;
  const cpx<double>* Xa;  // [W][nk][C], closed-shell traces of the up half
  const cpx<double>* Xb;  // the down half's
  cpx<double>* Ea;        // [W][3]
  cpx<double>* Eb;
};

__global__ __launch_bounds__(256) void spin_energy_kernel(const Batch<SpinEnergyArgs> B) {
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const SpinEnergyArgs a = B.a[pb];
  const int w = (int)loc, tid = threadIdx.x;
  const int64_t G = (int64_t)a.nk * a.C;
  const cpx<double>* xa = a.Xa + (int64_t)w * G;
  const cpx<double>* xb = a.Xb + (int64_t)w * G;
  double sr = 0.0, si = 0.0;
  for (int64_t i = tid; i < G; i += 256) {
    const int Q = (int)(i / a.C), g = (int)(i % a.C);
    const int64_t j = (int64_t)a.mesh.neg(Q) * a.C + g;
    const double pr = 0.5 * (xa[i].re + xb[i].re), pi = 0.5 * (xa[i].im + xb[i].im);
    const double qr = 0.5 * (xa[j].re + xb[j].re), qi = 0.5 * (xa[j].im + xb[j].im);
    sr += pr * qr - pi * qi;
    si += pr * qi + pi * qr;
  }
  __shared__ double rr[256], ri[256];
  rr[tid] = sr;
  ri[tid] = si;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) { rr[tid] += rr[tid + o]; ri[tid] += ri[tid + o]; }
    __syncthreads();
  }
  if (tid == 0) {
    cpx<double>* ea = a.Ea + 3 * (int64_t)w;
    cpx<double>* eb = a.Eb + 3 * (int64_t)w;
    const cpx<double> e1{0.5 * (ea[0].re + eb[0].re), 0.5 * (ea[0].im + eb[0].im)};
    const cpx<double> ec{0.5 * rr[0], 0.5 * ri[0]};
    const cpx<double> ex{0.5 * (ea[2].re + eb[2].re), 0.5 * (ea[2].im + eb[2].im)};
    ea[0] = e1; ea[1] = ec; ea[2] = ex;
    eb[0] = e1; eb[1] = ec; eb[2] = ex;
  }
}

long long blocks_for(int64_t n) {
  const long long b = (long long)((n + 255) / 256);
  return b < 1 ? 1 : (b > 2048 ? 2048 : b);
}

}  // namespace

bool has_pairs(const Job* jobs, int n) {
  for (int i = 0; i < n; ++i)
    if (jobs[i].p.spin == AFQMC_SPIN_UP) return true;
  return false;
}

hipError_t run_pair_mean(double* const* a, double* const* b, const int64_t* n, int cnt,
                         hipStream_t s) {
  for (int c0 = 0; c0 < cnt; c0 += AFQMC_MAXP) {
    const int c = (cnt - c0 < AFQMC_MAXP) ? cnt - c0 : AFQMC_MAXP;
    Batch<PairMeanArgs> B;
    B.nprob = c;
    long long nb[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      nb[q] = blocks_for(n[c0 + q]);
      B.a[q] = PairMeanArgs{a[c0 + q], b[c0 + q], n[c0 + q], nb[q]};
    }
    const long long g = batch_close(B, nb);
    if (g < 0) return hipErrorInvalidValue;
    if (g == 0) continue;
    hipLaunchKernelGGL(pair_mean_kernel, dim3((unsigned)g), dim3(256), 0, s, B);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_spin_fields(const Job* jobs, int n, hipStream_t s) {
  std::vector<double*> a, b;
  std::vector<int64_t> cnt;
  for (int i = 0; i + 1 < n; ++i) {
    if (jobs[i].p.spin != AFQMC_SPIN_UP) continue;
    const Job &u = jobs[i], &d = jobs[i + 1];
    const int64_t G = (int64_t)u.p.nwalk * u.p.nk * u.p.nchol;
    if (u.xbar && d.xbar) {  // [W][nk][C][2] complex128
      a.push_back((double*)u.xbar); b.push_back((double*)d.xbar); cnt.push_back(4 * G);
    }
    if (u.X && d.X) {  // [W][nk][C] complex128
      a.push_back((double*)u.X); b.push_back((double*)d.X); cnt.push_back(2 * G);
    }
  }
  if (a.empty()) return hipSuccess;
  return run_pair_mean(a.data(), b.data(), cnt.data(), (int)a.size(), s);
}

hipError_t run_spin_energy(const Job* jobs, int n, void* const* X, hipStream_t s) {
  std::vector<int> up;
  for (int i = 0; i + 1 < n; ++i)
    if (jobs[i].p.spin == AFQMC_SPIN_UP) up.push_back(i);
  for (size_t c0 = 0; c0 < up.size(); c0 += AFQMC_MAXP) {
    const int c = (int)((up.size() - c0 < AFQMC_MAXP) ? up.size() - c0 : AFQMC_MAXP);
    Batch<SpinEnergyArgs> B;
    B.nprob = c;
    long long cnt[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const int i = up[c0 + q];
      const afqmc_kpt_problem& p = jobs[i].p;
      SpinEnergyArgs& a = B.a[q];
      a.W = p.nwalk; a.nk = p.nk; a.C = p.nchol;
      a.mesh = make_mesh(p);
      a.Xa = (const cpx<double>*)X[i];
      a.Xb = (const cpx<double>*)X[i + 1];
      a.Ea = (cpx<double>*)jobs[i].E;
      a.Eb = (cpx<double>*)jobs[i + 1].E;
      cnt[q] = p.nwalk;
    }
    const long long g = batch_close(B, cnt);
    if (g < 0) return hipErrorInvalidValue;
    if (g == 0) continue;
    hipLaunchKernelGGL(spin_energy_kernel, dim3((unsigned)g), dim3(256), 0, s, B);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_spin_adjoint_scale(const Job* jobs, int n, hipStream_t s) {
  std::vector<int> idx;
  for (int i = 0; i < n; ++i)
    if (jobs[i].p.spin != AFQMC_SPIN_CLOSED && jobs[i].gGh) idx.push_back(i);
  for (size_t c0 = 0; c0 < idx.size(); c0 += AFQMC_MAXP) {
    const int c = (int)((idx.size() - c0 < AFQMC_MAXP) ? idx.size() - c0 : AFQMC_MAXP);
    Batch<ScaleArgs> B;
    B.nprob = c;
    long long nb[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const Job& j = jobs[idx[c0 + q]];
      const int64_t nd = 2 * (int64_t)j.p.nwalk * j.p.nk * j.p.nocc * j.p.nk * j.p.m;
      nb[q] = blocks_for(nd);
      B.a[q] = ScaleArgs{(double*)j.gGh, nd, 0.5, nb[q]};
    }
    const long long g = batch_close(B, nb);
    if (g < 0) return hipErrorInvalidValue;
    if (g == 0) continue;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)g), dim3(256), 0, s, B);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace afqmc
