// Beyn extraction and sigma_min helpers (see beyn.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace nep {

struct BeynArgs {
  const int* disk_ids;      // [ndisks] global disk ids (device)
  const int* dn;            // per global disk: n
  const long long* soff;    // per global disk: row offset of its sums
  const int* ix;            // per global disk: cell indices
  const int* iy;
  const double2* C0;        // sums buffers (rows soff[d]..soff[d]+n, L columns)
  const double2* C1;
  int L;
  int nmax;                 // scratch rows per disk
  double tol_svd;
  double x0, x1, y0, y1;    // region of the listed disks (one problem per launch)
  int nx, ny;
  double2* scratch;         // [ndisks][2][nmax][L]
  double2* eig_out;         // [ndisks][L]
  int* p_out;               // [ndisks]
  double* sv_out;           // [ndisks][L]
  unsigned char* keep_out;  // [ndisks][L] or null
  double2* eigvec_out;      // [ndisks][n][L] or null
  int* status;              // [ndisks] bit 0: eigenvalue iteration did not converge
};

hipError_t launch_beyn(const BeynArgs& a, int ndisks, hipStream_t st);
hipError_t launch_normalize(double2* X, long long xstride, int n, double* est, int record, int nb, hipStream_t st);
hipError_t launch_start(double2* X, long long xstride, int n, double* est, int nb, hipStream_t st);

}  // namespace nep
