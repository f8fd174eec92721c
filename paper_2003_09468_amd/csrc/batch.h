// Problem batches.  One launch serves up to AFQMC_MAXP problems (systems of different
// nk, m, nchol or walker count): the kernel receives every problem's arguments by value and
// the index of the first workgroup of each problem, and each workgroup finds its problem
// by a scan of that short table.  The problem index is made wave-uniform, so the
// arguments of the problem are scalar loads from the kernel-argument segment.
#pragma once

#include "kcommon.h"

namespace afqmc {

#define AFQMC_MAXP 8

template <class A>
struct Batch {
  A a[AFQMC_MAXP];
  long long first[AFQMC_MAXP + 1];  // first workgroup of each problem; first[nprob] = grid
  int nprob;
};

// Problem of global workgroup gid and the workgroup's index inside that problem.
template <class A>
__device__ __forceinline__ int batch_find(const Batch<A>& B, long long gid, long long& local) {
  int p = 0;
  while (p + 1 < B.nprob && gid >= B.first[p + 1]) ++p;
  p = __builtin_amdgcn_readfirstlane(p);
  local = gid - B.first[p];
  return p;
}

// Host: prefix sums of the per-problem workgroup counts; returns the grid size (0 if
// nothing to do, -1 if it exceeds the 32-bit grid limit).
template <class A>
long long batch_close(Batch<A>& B, const long long* count) {
  long long t = 0;
  for (int i = 0; i < B.nprob; ++i) {
    B.first[i] = t;
    t += count[i] > 0 ? count[i] : 0;
  }
  B.first[B.nprob] = t;
  return t > 0x7fffffffLL ? -1 : t;
}

}  // namespace afqmc
