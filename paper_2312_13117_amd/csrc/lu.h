// Batched LU / solve entry points shared by the host plan (see lu.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace nep {

constexpr int LU_NB = 64;   // panel width

// Per-step row-exchange record: [cnt, pos[2*NB], src[2*NB]] ints per step per matrix.
constexpr long long perm_ints_per_step() { return 1 + 4 * LU_NB; }

// Optional per-launch timing of the trailing-update kernel: events recorded on the
// launch stream around every launch, read back by the host after synchronisation.
struct LuTimers {
  static constexpr int MAXP = 2048;
  bool ev_enabled = false;
  int npairs = 0;
  hipEvent_t* ev = nullptr;   // 2 * MAXP events, created by the owner
  long long gemm_launches = 0;
  double gemm_flops = 0;
};

template <typename T>
hipError_t lu_factor_batch(c2<T>* W, long long mstride, int n, int nbatch, int* ipiv, int* perm,
                           long long perm_stride, c2<T>* Linv, c2<T>* Uinv, long long inv_stride, int* info,
                           hipStream_t st, LuTimers* tm);

template <typename T>
hipError_t lu_solve_batch(const c2<T>* W, long long mstride, int n, int nbatch, const int* perm,
                          long long perm_stride, const c2<T>* Linv, const c2<T>* Uinv, long long inv_stride,
                          double2* X, long long xstride, int m, bool trans, const int* active, hipStream_t st);

}  // namespace nep
