// Sweep kernels' launchers (see sweep.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace nep {

constexpr int MAX_TERMS = 4;
enum { PHI_ONE = 0, PHI_Z = 1, PHI_Z2 = 2, PHI_NEG_Z = 3, PHI_EXP_NEG_TAU_Z = 4 };

// Problem descriptor passed by value to kernels.  A[k] == nullptr means A_k = I.
struct ProblemDev {
  int n;
  int nterms;
  const double2* A[MAX_TERMS];
  int kind[MAX_TERMS];
  double param[MAX_TERMS];
  int real[MAX_TERMS];   // 1 if A_k has no imaginary part (set at plan time)
};

template <typename T>
hipError_t launch_assemble(const ProblemDev& pd, const double2* znode, c2<T>* W, long long mstride, int nbatch,
                           hipStream_t st);
hipError_t launch_rhs(const double2* F, int s, const double2* V, int L, int n, double2* X, long long xstride,
                      int nbatch, hipStream_t st);
hipError_t launch_sums(const double2* X, long long xstride, const double2* wts, const double2* zn, int N, int n,
                       int s, int L, double2* PfN, double2* PfN2, double2* C0, double2* C1, const int* disk_ids,
                       int ndisks, const long long* soff, int* nonfin, hipStream_t st);
hipError_t launch_profile(const double2* X, long long xstride, int N, int n, int s, int m, double* prof,
                          const int* disk_ids, int ndisks, hipStream_t st);
hipError_t launch_indicator(const double2* PfN, const double2* PfN2, const int* dn, const long long* soff, int s,
                            double tol, double* ind, unsigned char* flags, const int* sing, const int* nonfin,
                            int N, const double* prof, const double* rad, double floor, int ndisks, hipStream_t st);
// Rounding-noise floor of a quadrature sum relative to the size of its summands: a sum
// of N node solutions with normwise relative errors eps lies within (eps + gamma_N) S of
// the exact sum; a backward-stable LU gives eps <= c n u kappa, and with n <= 2^12,
// u = 2^-53 and kappa <= 2^10 (the floor only matters far from every eigenvalue, where
// the node matrices are well conditioned) that is 2^-31; the floor is twice that.
constexpr double INDICATOR_NOISE_FLOOR = 0x1p-30;
hipError_t launch_residual(const ProblemDev& pd, const double2* znode, const double2* X, const double2* F, int s,
                           const double2* V, int L, long long xstride, int m, int nbatch, double2* R,
                           const int* active, hipStream_t st);
hipError_t launch_is_real(const ProblemDev& pd, int* flags, hipStream_t st);
hipError_t launch_refine_check(const double2* D, const double2* X, long long xstride, int len, double tol,
                               double* dprev, int first, int* active, int* diverged, int nbatch, int* count,
                               hipStream_t st);
hipError_t launch_norms(const double2* R, const double2* X, long long xstride, int len, double* rn2, double* xn2,
                        int nbatch, hipStream_t st);
hipError_t launch_axpy(double2* X, const double2* D, long long xstride, int len, const int* active, int nbatch,
                       hipStream_t st);
hipError_t launch_fill_int(int* a, int v, int n, hipStream_t st);
hipError_t launch_mark_singular(const int* info, int nb, int* sing, hipStream_t st);
hipError_t launch_refine_init(const int* info, int nb, int* active, int* diverged, hipStream_t st);
hipError_t launch_or_flags(const int* a, const int* c, int nb, int* out, hipStream_t st);
hipError_t launch_elementwise_delay(const double2* A0, const double2* A1, const double* tau, int n, const double2* z,
                                    int nb, double2* W, long long mstride, hipStream_t st);
hipError_t launch_circle_double_layer(int P, const double2* k, int nb, double2* W, long long mstride, hipStream_t st);
hipError_t launch_rayleigh_terms(const ProblemDev& pd, const double2* U, const double2* V, long long xstride,
                                 int nb, double2* out, hipStream_t st);

}  // namespace nep
