// Batched LU / solve entry points shared by the host plan (see lu.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace nep {

constexpr int LU_NB = 64;   // panel width
// The solve runs step by step over many workgroups per matrix for orders >= 256 with
// at most 8 right-hand sides (measured: delay workload, m = 1, solve and refinement
// phases 1.4-1.6x faster split), and for orders >= LU_SOLVE_MFMA_N with 9 to 32 on the
// matrix cores (dense workload, m = 20: 1.4x faster than one workgroup per matrix; the
// same steps on the vector units gave no gain there).
constexpr int LU_SOLVE_SPLIT_N = 256, LU_SOLVE_SPLIT_M = 8;
constexpr int LU_SOLVE_MFMA_N = 512;

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

// Pivot choice of the panel factorisation: LAPACK-style partial pivoting (one
// workgroup per panel), or tournament pivoting (row chunks factored in parallel,
// their pivot candidates merged pairwise; the factors then satisfy P A = L U with
// the tournament's pivot rows).
enum { LU_PIVOT_PARTIAL = 0, LU_PIVOT_TOURNAMENT = 1 };

// Scratch bytes per matrix for lu_factor_batch (either pivot choice).
size_t lu_factor_scratch_bytes(int n, size_t elem_bytes);

template <typename T>
hipError_t lu_factor_batch(c2<T>* W, long long mstride, int n, int nbatch, void* scratch, int* perm,
                           long long perm_stride, c2<T>* Linv, c2<T>* Uinv, long long inv_stride, int* info,
                           int pivot, hipStream_t st, LuTimers* tm);

template <typename T>
hipError_t lu_solve_batch(const c2<T>* W, long long mstride, int n, int nbatch, const int* perm,
                          long long perm_stride, const c2<T>* Linv, const c2<T>* Uinv, long long inv_stride,
                          double2* X, long long xstride, int m, bool trans, const int* active, hipStream_t st);

}  // namespace nep
