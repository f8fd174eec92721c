// Population control by the comb: one uniform number per system picks nwalk equally
// spaced points on the cumulative weight, and each point copies the walker whose weight
// interval holds it (stochastic reconfiguration; every new weight is the mean weight).
#include <math.h>

#include <vector>

#include "internal.h"
#include "kcommon.h"

namespace afqmc {

namespace {

struct CombArgs {
  int W;
  double xi;
  const double* weight;  // [W]
  double* cum;           // [W] workspace: cumulative weights
  int* par;              // [W] workspace: parent of each copy
  int* par_out;          // [W] caller's copy of par, or null
  double* neww;          // [1] workspace: the new weight, or -1 (population unchanged)
};

// One workgroup per system.  The cumulative sum is sequential in walker order (the order
// fixes the rounding of the comb's boundaries); each copy then binary-searches it.
__global__ __launch_bounds__(256) void comb_kernel(const Batch<CombArgs> B) {
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const CombArgs a = B.a[pb];
  __shared__ double s_tot;
  __shared__ int s_last, s_ok;
  if (threadIdx.x == 0) {
    double c = 0.0;
    int last = -1, ok = 1;
    for (int i = 0; i < a.W; ++i) {
      const double w = a.weight[i];
      if (!(w >= 0.0) || !__builtin_isfinite(w)) ok = 0;
      c += w;
      a.cum[i] = c;
      if (w > 0.0) last = i;
    }
    ok = ok && c > 0.0 && __builtin_isfinite(c);
    s_tot = c;
    s_last = last;
    s_ok = ok;
    *a.neww = ok ? c / a.W : -1.0;
  }
  __syncthreads();
  const double step = s_tot / a.W;
  for (int j = threadIdx.x; j < a.W; j += 256) {
    int i = j;
    if (s_ok) {
      const double z = ((double)j + a.xi) * step;
      int lo = 0, hi = a.W;  // first i with cum[i] > z (a zero-weight interval is empty)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.cum[mid] > z) hi = mid;
        else lo = mid + 1;
      }
      i = lo < s_last ? lo : s_last;  // rounding can put the last point at c
    }
    a.par[j] = i;
    if (a.par_out) a.par_out[j] = i;
  }
}

struct PopCopyArgs {
  int W;
  int64_t E;             // complex entries of one walker's U (= of its Gh)
  const int* par;        // [W]
  cpx<double>* U;        // [W][E]
  cpx<double>* Gh;       // [W][E]
  cpx<double>* logdet;   // [W]
  int* status;           // [W]
  double* weight;        // [W]
  cpx<double>* tU;       // [W][E] workspace
  cpx<double>* tG;       // [W][E] workspace
  cpx<double>* tL;       // [W] workspace
  int* tS;               // [W] workspace
  const double* neww;    // [1]
  long long nblk;        // workgroups of this system
};

// GATHER: the parents' state into the workspace; otherwise the workspace back in place
// (with the new weights).  Grid-stride over the system's entries.
template <bool GATHER>
__global__ __launch_bounds__(256) void pop_copy_kernel(const Batch<PopCopyArgs> B) {
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const PopCopyArgs a = B.a[pb];
  const int64_t total = (int64_t)a.W * a.E;
  for (int64_t idx = loc * 256 + threadIdx.x; idx < total; idx += a.nblk * 256) {
    const int64_t w = idx / a.E, e = idx % a.E;
    if (GATHER) {
      const int64_t src = (int64_t)a.par[w] * a.E + e;
      a.tU[idx] = a.U[src];
      a.tG[idx] = a.Gh[src];
    } else {
      a.U[idx] = a.tU[idx];
      a.Gh[idx] = a.tG[idx];
    }
  }
  for (int64_t w = loc * 256 + threadIdx.x; w < a.W; w += a.nblk * 256) {
    if (GATHER) {
      a.tL[w] = a.logdet[a.par[w]];
      a.tS[w] = a.status[a.par[w]];
    } else {
      a.logdet[w] = a.tL[w];
      a.status[w] = a.tS[w];
      const double nw = *a.neww;
      if (nw > 0.0) a.weight[w] = nw;
    }
  }
}

struct PopWs {
  double* cum; int* par; double* neww; cpx<double>* tU; cpx<double>* tG; cpx<double>* tL; int* tS;
};

size_t carve_population(Carve& c, const afqmc_kpt_problem& p, PopWs& w) {
  const size_t W = (size_t)p.nwalk, E = (size_t)p.nk * p.m * (size_t)p.nk * p.nocc;
  w.cum = (double*)c.take(8 * W);
  w.par = (int*)c.take(4 * W);
  w.neww = (double*)c.take(8);
  w.tU = (cpx<double>*)c.take(16 * W * E);
  w.tG = (cpx<double>*)c.take(16 * W * E);
  w.tL = (cpx<double>*)c.take(16 * W);
  w.tS = (int*)c.take(4 * W);
  return c.off;
}

}  // namespace

size_t population_ws_bytes(const afqmc_kpt_problem& p) {
  Carve c(nullptr);
  PopWs w;
  return carve_population(c, p, w);
}

hipError_t run_population(const afqmc_kpt_problem* p, int nprob, const double* xi,
                          int32_t* const* parent, void* ws, hipStream_t s) {
  char* base = (char*)ws;
  for (int c0 = 0; c0 < nprob; c0 += AFQMC_MAXP) {
    const int c = (nprob - c0 < AFQMC_MAXP) ? nprob - c0 : AFQMC_MAXP;
    Batch<CombArgs> Bc;
    Batch<PopCopyArgs> Bp;
    Bc.nprob = Bp.nprob = c;
    long long cc[AFQMC_MAXP], cp[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      const int i = c0 + q;
      const afqmc_kpt_problem& pi = p[i];
      // this system's workspace region follows those of the systems before it
      size_t off = 0;
      for (int k = 0; k < i; ++k) off += align_up(population_ws_bytes(p[k]));
      Carve cv(base + off);
      PopWs w;
      carve_population(cv, pi, w);
      CombArgs& a = Bc.a[q];
      a.W = pi.nwalk;
      a.xi = xi[i];
      a.weight = pi.weight;
      a.cum = w.cum;
      a.par = w.par;
      a.par_out = parent ? parent[i] : nullptr;
      a.neww = w.neww;
      cc[q] = 1;
      PopCopyArgs& b = Bp.a[q];
      b.W = pi.nwalk;
      b.E = (int64_t)pi.nk * pi.m * (int64_t)pi.nk * pi.nocc;
      b.par = w.par;
      b.U = (cpx<double>*)pi.U;
      b.Gh = (cpx<double>*)pi.Gh;
      b.logdet = (cpx<double>*)pi.logdet;
      b.status = pi.status;
      b.weight = pi.weight;
      b.tU = w.tU; b.tG = w.tG; b.tL = w.tL; b.tS = w.tS;
      b.neww = w.neww;
      const long long need = ((long long)b.W * b.E + 255) / 256;
      b.nblk = need < 2048 ? (need > 0 ? need : 1) : 2048;
      cp[q] = b.nblk;
    }
    long long g = batch_close(Bc, cc);
    if (g <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(comb_kernel, dim3((unsigned)g), dim3(256), 0, s, Bc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    g = batch_close(Bp, cp);
    if (g <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pop_copy_kernel<true>, dim3((unsigned)g), dim3(256), 0, s, Bp);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pop_copy_kernel<false>, dim3((unsigned)g), dim3(256), 0, s, Bp);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Energy shift between blocks: E_T <- (1 - blend) E_T + blend Re(Emix), per system, when the
// system's mixed estimate is finite.  One thread per system.
struct EtrialArgs {
  double* et;               // [1]
  const cpx<double>* emix;  // [1]
  double blend;
};

__global__ __launch_bounds__(64) void etrial_kernel(const Batch<EtrialArgs> B) {
  if (threadIdx.x != 0) return;
  long long loc;
  const int pb = batch_find(B, blockIdx.x, loc);
  const EtrialArgs a = B.a[pb];
  const cpx<double> e = a.emix[0];
  if (__builtin_isfinite(e.re) && __builtin_isfinite(e.im))
    a.et[0] = (1.0 - a.blend) * a.et[0] + a.blend * e.re;
}

hipError_t run_update_etrial(const afqmc_kpt_problem* p, int nprob, const void* Emix,
                             double blend, hipStream_t s) {
  for (int c0 = 0; c0 < nprob; c0 += AFQMC_MAXP) {
    const int c = (nprob - c0 < AFQMC_MAXP) ? nprob - c0 : AFQMC_MAXP;
    Batch<EtrialArgs> B;
    B.nprob = c;
    long long cnt[AFQMC_MAXP];
    for (int q = 0; q < c; ++q) {
      B.a[q].et = p[c0 + q].etrial;
      B.a[q].emix = (const cpx<double>*)Emix + c0 + q;
      B.a[q].blend = blend;
      cnt[q] = 1;
    }
    const long long g = batch_close(B, cnt);
    if (g <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(etrial_kernel, dim3((unsigned)g), dim3(64), 0, s, B);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Blocking analysis on the host (error bars of a serially correlated series): level 0 is
// the series, level l + 1 the means of neighbouring pairs of level l; sample variance with
// the n - 1 denominator; the first level with B^3 > 2 n (err_l / err_0)^4 is the one to
// quote (Lee, Needs and Towler).
int reblock_host(const double* x, int64_t n, afqmc_reblock_level* levels, int max_levels,
                 int* optimal) {
  std::vector<double> cur(x, x + n), nxt;
  int nl = 0, opt = -1;
  double err0 = 0.0;
  while ((int64_t)cur.size() >= 2) {
    const int64_t m = (int64_t)cur.size();
    double sum = 0.0;
    for (int64_t i = 0; i < m; ++i) sum += cur[i];
    const double mean = sum / (double)m;
    double ss = 0.0;
    for (int64_t i = 0; i < m; ++i) ss += (cur[i] - mean) * (cur[i] - mean);
    const double err = sqrt(ss / (double)(m - 1) / (double)m);
    if (nl == 0) err0 = err;
    if (nl < max_levels)
      levels[nl] = afqmc_reblock_level{m, mean, err, err / sqrt(2.0 * (double)(m - 1))};
    if (opt < 0) {
      const double r = err0 > 0.0 ? err / err0 : 1.0;
      const double B = ldexp(1.0, nl);
      if (B * B * B > 2.0 * (double)n * r * r * r * r) opt = nl;
    }
    ++nl;
    const int64_t h = m / 2;
    nxt.resize(h);
    for (int64_t i = 0; i < h; ++i) nxt[i] = 0.5 * (cur[2 * i] + cur[2 * i + 1]);
    cur.swap(nxt);
  }
  *optimal = opt;
  return nl;
}

}  // namespace afqmc
