// Quadrature sweep kernels around the batched LU:
//   assemble_kernel   T(z_t) = sum_k phi_k(z_t) A_k for a batch of nodes (eq (2.4)),
//                     written in the LU's arithmetic (complex128 or complex64)
//   rhs_kernel        copies [F | V] of each node's problem into its solution slot
//   sums_kernel       per disk: P f|_N, P f|_{N/2} (1-based even nodes, weight 2 w_j),
//                     C0 = sum w_j X_j^V, C1 = sum w_j z_j X_j^V (eqs (2.3), (3.2)-(3.3)),
//                     accumulated in complex128 in node order
//   profile_kernel    ||x_j[:, q]||_2 per node and probe column
//   indicator_kernel  I_q = || P f|_N ./ P f|_{N/2} ||_2 / sqrt(n)   (eq (3.1)), with the
//                     rounding-noise floor of the two rules' sums
//   residual_kernel   R_t = B_t - T(z_t) X_t in complex128 (mixed-precision refinement)
#include "common.h"
#include "sweep.h"

namespace nep {

NEP_DEV double2 phi_eval(int kind, double par, double2 z) {
  switch (kind) {
    case PHI_ONE: return cmk<double>(1.0, 0.0);
    case PHI_Z: return z;
    case PHI_Z2: return cmul<double>(z, z);
    case PHI_NEG_Z: return cmk<double>(-z.x, -z.y);
    case PHI_EXP_NEG_TAU_Z: {
      const double e = exp(-par * z.x), a = -par * z.y;
      double s, c;
      sincos(a, &s, &c);
      return cmk<double>(e * c, e * s);
    }
  }
  return cmk<double>(0.0, 0.0);
}

// grid: (ceil(n*n / 512), ceil(nbatch / NPB)).  Each thread loads 2 consecutive
// entries of every coefficient once and writes them for NPB nodes, so coefficient
// traffic is 1/NPB of the output traffic.
constexpr int ASM_NPB = 16;
template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(ProblemDev pd, const double2* __restrict__ znode,
                                                       c2<T>* __restrict__ W, long long mstride, int nbatch) {
  __shared__ double2 ph[ASM_NPB][MAX_TERMS];
  const int b0 = blockIdx.y * ASM_NPB;
  const int n = pd.n;
  const long long nn = (long long)n * n;
  if (threadIdx.x < ASM_NPB * MAX_TERMS) {
    const int nb = threadIdx.x / MAX_TERMS, k = threadIdx.x % MAX_TERMS;
    ph[nb][k] = (b0 + nb < nbatch && k < pd.nterms) ? phi_eval(pd.kind[k], pd.param[k], znode[b0 + nb])
                                                   : cmk<double>(0, 0);
  }
  __syncthreads();
  const long long e0 = ((long long)blockIdx.x * 256 + threadIdx.x) * 2;
  if (e0 >= nn) return;
  double2 a[MAX_TERMS][2];
  bool diag[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const long long e = e0 + u;
    diag[u] = (e < nn) && (e / n == e % n);
#pragma unroll
    for (int k = 0; k < MAX_TERMS; ++k) {
      if (k < pd.nterms && e < nn) a[k][u] = pd.A[k] ? pd.A[k][e] : (diag[u] ? cmk<double>(1, 0) : cmk<double>(0, 0));
      else a[k][u] = cmk<double>(0, 0);
    }
  }
  const int nbk = min(ASM_NPB, nbatch - b0);
  for (int nb = 0; nb < nbk; ++nb) {
    c2<T>* out = W + (long long)(b0 + nb) * mstride;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      double2 acc = cmk<double>(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < MAX_TERMS; ++k) acc = cfma<double>(acc, ph[nb][k], a[k][u]);
      if (e0 + u < nn) out[e0 + u] = ccast<T, double>(acc);
    }
  }
}

// X_t (n x m) = [F | V] of the node's problem; grid (ceil(n*m/256), nbatch)
__global__ __launch_bounds__(256) void rhs_kernel(const double2* __restrict__ F, int s, const double2* __restrict__ V,
                                                  int L, int n, double2* __restrict__ X, long long xstride,
                                                  int nbatch) {
  const int b = blockIdx.y;
  if (b >= nbatch) return;
  const int m = s + L;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * m) return;
  const int i = e / m, q = e % m;
  X[(long long)b * xstride + e] = (q < s) ? F[(long long)i * s + q] : V[(long long)i * L + (q - s)];
}

// grid (ceil(n*m/256), ndisks).  Node j of list entry dl has its solution at
// X + (dl*N + j)*xstride (n x m); dl maps to the global disk disk_ids[dl].  Sums run
// over j = 1..N in order (fixed rounding order).  A non-finite solution entry sets
// nonfin[dl*N + j] (every writer stores 1).
__global__ __launch_bounds__(256) void sums_kernel(const double2* __restrict__ X, long long xstride,
                                                   const double2* __restrict__ wts, const double2* __restrict__ zn,
                                                   int N, int n, int s, int L, double2* __restrict__ PfN,
                                                   double2* __restrict__ PfN2, double2* __restrict__ C0,
                                                   double2* __restrict__ C1, const int* __restrict__ disk_ids,
                                                   const long long* __restrict__ soff, int* __restrict__ nonfin) {
  const int dl = blockIdx.y;
  const int d = disk_ids ? disk_ids[dl] : dl;
  const int m = s + L;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * m) return;
  const int i = e / m, q = e % m;
  const double2* w = wts + (long long)d * N;
  const double2* z = zn + (long long)d * N;
  const long long t0 = (long long)dl * N;
  double2 a0 = cmk<double>(0, 0), a1 = cmk<double>(0, 0);
  for (int j = 0; j < N; ++j) {
    const double2 x = X[(t0 + j) * xstride + e];
    if (nonfin && !(fabs(x.x) <= 1.7976931348623157e308 && fabs(x.y) <= 1.7976931348623157e308)) nonfin[t0 + j] = 1;
    if (q < s) {
      a0 = cfma<double>(a0, w[j], x);
      if (j & 1) a1 = cfma<double>(a1, cscale<double>(w[j], 2.0), x);   // 1-based even node
    } else {
      a0 = cfma<double>(a0, w[j], x);
      a1 = cfma<double>(a1, cmul<double>(w[j], z[j]), x);
    }
  }
  const long long base = soff[d];
  if (q < s) {
    PfN[base * s + (long long)i * s + q] = a0;
    PfN2[base * s + (long long)i * s + q] = a1;
  } else if (L > 0) {
    C0[base * L + (long long)i * L + (q - s)] = a0;
    C1[base * L + (long long)i * L + (q - s)] = a1;
  }
}

// |a| without overflow or underflow of the squares
NEP_DEV double cabs_safe(double2 a) { return hypot(a.x, a.y); }

// Block-wide (256 threads) max and sum of three values; every thread gets the result.
NEP_DEV void block_max3(double* v, double (*red)[3]) {
  for (int k = 0; k < 3; ++k)
    for (int o = 32; o > 0; o >>= 1) {
      const double u = __shfl_xor(v[k], o, 64);
      v[k] = (u > v[k] || u != u) ? u : v[k];     // NaN wins
    }
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 3; ++k) red[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    double r = red[0][k];
    for (int w = 1; w < 4; ++w) r = (red[w][k] > r || red[w][k] != red[w][k]) ? red[w][k] : r;
    v[k] = r;
  }
}
NEP_DEV void block_sum3(double* v, double (*red)[3]) {
  for (int k = 0; k < 3; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 3; ++k) red[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
  for (int k = 0; k < 3; ++k) v[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
}

// 2-norm as max * sqrt(sum (|v_i| / max)^2): entries far outside 1e+-154 neither
// overflow nor underflow when squared
NEP_DEV double scaled_norm(double mx, double ssq) { return (mx > 0.0 && mx <= 1.7976931348623157e308) ? mx * sqrt(ssq) : mx; }

// grid (N, ndisks), 256 threads: profile[d][j][q] = ||x_j[:, q]||_2, q < s
__global__ __launch_bounds__(256) void profile_kernel(const double2* __restrict__ X, long long xstride, int N,
                                                      int n, int s, int m, double* __restrict__ prof,
                                                      const int* __restrict__ disk_ids) {
  const int j = blockIdx.x, dl = blockIdx.y, d = disk_ids[dl];
  const double2* x = X + ((long long)dl * N + j) * xstride;
  __shared__ double red[4][3];
  for (int q = 0; q < s; ++q) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += 256) {
      const double a = cabs_safe(x[(long long)i * m + q]);
      v[0] = (a > v[0] || a != a) ? a : v[0];
    }
    block_max3(v, red);
    const double mx = v[0];
    double t[3] = {0.0, 0.0, 0.0};
    if (mx > 0.0 && mx <= 1.7976931348623157e308)
      for (int i = threadIdx.x; i < n; i += 256) {
        const double a = cabs_safe(x[(long long)i * m + q]) / mx;
        t[0] += a * a;
      }
    block_sum3(t, red);
    if (threadIdx.x == 0) prof[((long long)d * N + j) * s + q] = scaled_norm(mx, t[0]);
  }
}

// one workgroup per disk, per probe column q:
//   I_q = ||P f|_N[:, q] ./ P f|_{N/2}[:, q]||_2 / sqrt(n), +inf if not finite;
//   I_q = 0 when ||P f|_N[:, q]|| <= floor * S_N and ||P f|_{N/2}[:, q]|| <= floor * S_half
//   (all four finite), S_N = (r/N) sum_j ||x_j[:, q]|| and S_half = (2r/N) sum over the
//   1-based even nodes, the summand sizes of the two rules: both sums are then rounding
//   noise and so is their ratio.
// The disk is flagged if some I_q > tol or one of its nodes is singular or non-finite.
__global__ __launch_bounds__(256) void indicator_kernel(const double2* __restrict__ PfN,
                                                        const double2* __restrict__ PfN2, const int* __restrict__ dn,
                                                        const long long* __restrict__ soff, int s, double tol,
                                                        double* __restrict__ ind, unsigned char* __restrict__ flags,
                                                        const int* __restrict__ sing, const int* __restrict__ nonfin,
                                                        int N, const double* __restrict__ prof,
                                                        const double* __restrict__ rad, double floor) {
  const int d = blockIdx.x;
  const int n = dn[d];
  const double2* A = PfN + soff[d] * s;
  const double2* B = PfN2 + soff[d] * s;
  __shared__ double red[4][3];
  bool flag = false;
  for (int q = 0; q < s; ++q) {
    // pass 1: largest |ratio|, |PfN|, |PfN2| (NaN propagates)
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += 256) {
      const double a = cabs_safe(A[(long long)i * s + q]), b = cabs_safe(B[(long long)i * s + q]);
      const double r = a / b;   // 0/0 -> NaN, x/0 -> inf
      const double c[3] = {r, a, b};
      for (int k = 0; k < 3; ++k) v[k] = (c[k] > v[k] || c[k] != c[k]) ? c[k] : v[k];
    }
    block_max3(v, red);
    // pass 2: sums of squares scaled by those maxima
    double t[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += 256) {
      const double a = cabs_safe(A[(long long)i * s + q]), b = cabs_safe(B[(long long)i * s + q]);
      const double c[3] = {a / b, a, b};
      for (int k = 0; k < 3; ++k)
        if (v[k] > 0.0 && v[k] <= 1.7976931348623157e308) {
          const double u = c[k] / v[k];
          t[k] += u * u;
        }
    }
    block_sum3(t, red);
    if (threadIdx.x == 0) {
      double I = scaled_norm(v[0], t[0]) / sqrt((double)n);
      if (!(I <= 1.7976931348623157e308)) I = __builtin_inf();
      if (prof) {
        double SN = 0.0, SH = 0.0;
        for (int j = 0; j < N; ++j) {
          const double p = prof[((long long)d * N + j) * s + q];
          SN += p;
          if (j & 1) SH += p;
        }
        SN *= rad[d] / N;
        SH *= 2.0 * rad[d] / N;
        const double na = scaled_norm(v[1], t[1]), nb = scaled_norm(v[2], t[2]);
        const double big = 1.7976931348623157e308;
        if (na <= big && nb <= big && SN <= big && SH <= big && na <= floor * SN && nb <= floor * SH) I = 0.0;
      }
      ind[(long long)d * s + q] = I;
      if (I > tol) flag = true;
    }
  }
  if (threadIdx.x == 0) {
    for (int j = 0; j < N; ++j) {
      if (sing) flag = flag || sing[(long long)d * N + j] != 0;
      if (nonfin) flag = flag || nonfin[(long long)d * N + j] != 0;
    }
    flags[d] = flag ? 1 : 0;
  }
}

// R_t = B_t - sum_k phi_k(z_t) A_k X_t over the batch; grid (row tiles of 64, column
// tiles of 64 over the concatenated columns of all tasks).  Column c of the product is
// column c % m of task c / m; columns of converged tasks (active[t] == 0) are skipped.
// Matrix cores, complex128; a real coefficient needs two of the four real products.
// Operands go through LDS in chunks of 16 along the inner dimension (a 64 x 16 block
// of A_k and the matching 16 x 64 block of X, each column scaled by its task's
// phi_k(z)); the next chunk is loaded into registers while the current one is used.
constexpr int RES_KC = 16;
__global__ __launch_bounds__(256, 3) void residual_kernel(ProblemDev pd, const double2* __restrict__ znode,
                                                       const double2* __restrict__ X, const double2* __restrict__ F,
                                                       int s, const double2* __restrict__ V, int L,
                                                       long long xstride, int m, int nbatch,
                                                       double2* __restrict__ R, const int* __restrict__ active) {
  const int n = pd.n;
  const int ncol = nbatch * m;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int R0 = blockIdx.x * 64, C0 = blockIdx.y * 64;
  const int rw = (wave >> 1) * 32, cw = (wave & 1) * 32;     // the wave's quarter of the tile
  const int rb = R0 + rw, cb = C0 + cw;
  // skip tiles whose tasks have all converged
  if (active) {
    __shared__ int s_any;
    if (t == 0) s_any = 0;
    __syncthreads();
    const int c = C0 + (t & 63);
    if (t < 64 && c < ncol && active[c / m]) s_any = 1;
    __syncthreads();
    if (!s_any) return;
  }
  // the column this thread stages into the X block (the same for every chunk)
  const int sc = C0 + (t & 63);
  const int stask = (sc < ncol && (!active || active[sc / m])) ? sc / m : -1;
  const int sq = sc < ncol ? sc % m : 0;
  __shared__ double2 As[64][RES_KC + 1];
  __shared__ double2 Bs[RES_KC][64 + 1];
  constexpr int QA = 64 * RES_KC / 256, QB = RES_KC * 64 / 256;
  d4 cre[2][2], cim[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) { cre[bi][bj] = acc_zero<double>(); cim[bi][bj] = acc_zero<double>(); }
#pragma unroll
  for (int k = 0; k < MAX_TERMS; ++k) {
    if (k >= pd.nterms) break;
    const double2* Ak = pd.A[k];
    if (!Ak) continue;
    const bool real = pd.real[k] != 0;
    const double2 sph = stask >= 0 ? phi_eval(pd.kind[k], pd.param[k], znode[stask]) : cmk<double>(0, 0);
    double2 pa[QA], pb[QB];
    auto fetch = [&](int kk) {
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int e = t + q * 256, row = R0 + e / RES_KC, col = kk + e % RES_KC;
        pa[q] = (row < n && col < n) ? Ak[(long long)row * n + col] : cmk<double>(0, 0);
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int xr = kk + (t >> 6) + 4 * q;
        pb[q] = (stask >= 0 && xr < n) ? X[(long long)stask * xstride + (long long)xr * m + sq] : cmk<double>(0, 0);
      }
    };
    fetch(0);
    for (int kk = 0; kk < n; kk += RES_KC) {
      __syncthreads();                       // the previous chunk has been read
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int e = t + q * 256;
        As[e / RES_KC][e % RES_KC] = pa[q];
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) Bs[(t >> 6) + 4 * q][t & 63] = cmul<double>(sph, pb[q]);
      __syncthreads();
      if (kk + RES_KC < n) fetch(kk + RES_KC);
#pragma unroll
      for (int k4 = 0; k4 < RES_KC; k4 += 4) {
        double2 af[2], bf[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) af[bi] = As[rw + bi * 16 + l16][k4 + kq];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) bf[bj] = Bs[k4 + kq][cw + bj * 16 + l16];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            cre[bi][bj] = mfma16(af[bi].x, bf[bj].x, cre[bi][bj]);
            cim[bi][bj] = mfma16(af[bi].x, bf[bj].y, cim[bi][bj]);
          }
        if (!real) {
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
              cre[bi][bj] = mfma16(-af[bi].y, bf[bj].y, cre[bi][bj]);
              cim[bi][bj] = mfma16(af[bi].y, bf[bj].x, cim[bi][bj]);
            }
        }
      }
    }
  }
  // epilogue: identity coefficients and R = B - T X for the wave's columns
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    const int c = cb + bj * 16 + l16;
    const int ctask = (c < ncol && (!active || active[c / m])) ? c / m : -1;
    if (ctask < 0) continue;
    const int q = c % m;
    double2 ph[MAX_TERMS];
#pragma unroll
    for (int k = 0; k < MAX_TERMS; ++k)
      ph[k] = (k < pd.nterms && !pd.A[k]) ? phi_eval(pd.kind[k], pd.param[k], znode[ctask]) : cmk<double>(0, 0);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb + bi * 16 + acc_row<double>(lane, r);
        if (row >= n) continue;
        const long long off = (long long)ctask * xstride + (long long)row * m + q;
        double2 tx = cmk<double>(cre[bi][bj][r], cim[bi][bj][r]);
        const double2 x = X[off];
#pragma unroll
        for (int k = 0; k < MAX_TERMS; ++k)
          if (k < pd.nterms && !pd.A[k]) tx = cfma<double>(tx, ph[k], x);   // identity coefficient
        const double2 bv = (q < s) ? F[(long long)row * s + q] : V[(long long)row * L + (q - s)];
        R[off] = csub<double>(bv, tx);
      }
    }
  }
}

// flags[k] = 1 if coefficient k has no nonzero imaginary part (identity: 1)
__global__ __launch_bounds__(256) void is_real_kernel(ProblemDev pd, int* __restrict__ flags) {
  const int k = blockIdx.x;
  __shared__ int s_nz;
  if (threadIdx.x == 0) s_nz = 0;
  __syncthreads();
  if (pd.A[k]) {
    const long long nn = (long long)pd.n * pd.n;
    int nz = 0;
    for (long long e = threadIdx.x; e < nn && !nz; e += 256) nz = pd.A[k][e].y != 0.0;
    if (nz) s_nz = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) flags[k] = s_nz ? 0 : 1;
}

hipError_t launch_is_real(const ProblemDev& pd, int* flags, hipStream_t st) {
  is_real_kernel<<<pd.nterms, 256, 0, st>>>(pd, flags);
  return hipGetLastError();
}

// After a correction D (= dX) of active task b: keep refining while
// ||D|| > tol ||X||; a correction that does not shrink to half of the previous one
// (from the second sweep on) or is not finite marks the task as diverged.
// One workgroup per task.
__global__ __launch_bounds__(256) void refine_check_kernel(const double2* __restrict__ D, const double2* __restrict__ X,
                                                           long long xstride, int len, double tol,
                                                           double* __restrict__ dprev, int first,
                                                           int* __restrict__ active, int* __restrict__ diverged,
                                                           int* __restrict__ count) {
  const int b = blockIdx.x;
  if (!active[b]) return;
  double a = 0, c = 0;
  for (int e = threadIdx.x; e < len; e += 256) {
    a += cabs2<double>(D[(long long)b * xstride + e]);
    c += cabs2<double>(X[(long long)b * xstride + e]);
  }
  __shared__ double ra[4], rc[4];
  a = wave_sum(a);
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) { ra[threadIdx.x >> 6] = a; rc[threadIdx.x >> 6] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double dn = sqrt(ra[0] + ra[1] + ra[2] + ra[3]);
    const double xn = sqrt(rc[0] + rc[1] + rc[2] + rc[3]);
    const bool finite = (dn == dn) && (xn == xn) && dn < 1e300 && xn < 1e300;
    const bool bad = !finite || (!first && dn > 0.5 * dprev[b]);
    dprev[b] = dn;
    if (bad) { diverged[b] = 1; active[b] = 0; }
    else if (dn <= tol * xn) active[b] = 0;
    else atomicAdd(count, 1);
  }
}

hipError_t launch_refine_check(const double2* D, const double2* X, long long xstride, int len, double tol,
                               double* dprev, int first, int* active, int* diverged, int nbatch, int* count,
                               hipStream_t st) {
  refine_check_kernel<<<nbatch, 256, 0, st>>>(D, X, xstride, len, tol, dprev, first, active, diverged, count);
  return hipGetLastError();
}

// per task: ||R_t||_F^2 and ||X_t||_F^2 (one workgroup per task)
__global__ __launch_bounds__(256) void norms_kernel(const double2* __restrict__ R, const double2* __restrict__ X,
                                                    long long xstride, int len, double* __restrict__ rn2,
                                                    double* __restrict__ xn2) {
  const int b = blockIdx.x;
  double a = 0, c = 0;
  for (int e = threadIdx.x; e < len; e += 256) {
    a += cabs2<double>(R[(long long)b * xstride + e]);
    c += cabs2<double>(X[(long long)b * xstride + e]);
  }
  __shared__ double ra[4], rc[4];
  a = wave_sum(a);
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) { ra[threadIdx.x >> 6] = a; rc[threadIdx.x >> 6] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    rn2[b] = ra[0] + ra[1] + ra[2] + ra[3];
    xn2[b] = rc[0] + rc[1] + rc[2] + rc[3];
  }
}

// X += D for active tasks
__global__ __launch_bounds__(256) void axpy_kernel(double2* __restrict__ X, const double2* __restrict__ D,
                                                   long long xstride, int len, const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= len) return;
  const long long o = (long long)b * xstride + e;
  X[o] = cadd<double>(X[o], D[o]);
}

// sing[t0 + b] = info[b] != 0 (exact zero pivot in the factorisation of node b)
__global__ void mark_singular_kernel(const int* __restrict__ info, int nb, int* __restrict__ sing) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) sing[b] = info[b] != 0 ? 1 : 0;
}

hipError_t launch_mark_singular(const int* info, int nb, int* sing, hipStream_t st) {
  mark_singular_kernel<<<(nb + 255) / 256, 256, 0, st>>>(info, nb, sing);
  return hipGetLastError();
}

// refinement state of a batch: active = 1 and diverged = 0, except for tasks whose
// LU met an exact zero pivot (info != 0), which are set diverged and inactive
__global__ void refine_init_kernel(const int* __restrict__ info, int nb, int* __restrict__ active,
                                   int* __restrict__ diverged) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) {
    const int z = info[b] != 0;
    active[b] = 1 - z;
    diverged[b] = z;
  }
}

hipError_t launch_refine_init(const int* info, int nb, int* active, int* diverged, hipStream_t st) {
  refine_init_kernel<<<(nb + 255) / 256, 256, 0, st>>>(info, nb, active, diverged);
  return hipGetLastError();
}

// out[b] = a[b] | c[b]: the tasks still unconverged or diverged after refinement
__global__ void or_flags_kernel(const int* __restrict__ a, const int* __restrict__ c, int nb, int* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) out[b] = (a[b] | c[b]) != 0 ? 1 : 0;
}

hipError_t launch_or_flags(const int* a, const int* c, int nb, int* out, hipStream_t st) {
  or_flags_kernel<<<(nb + 255) / 256, 256, 0, st>>>(a, c, nb, out);
  return hipGetLastError();
}

// a[b * MAX_TERMS + k] = u_b^H A_k v_b (u_b^H v_b for an identity coefficient): the
// scalars of the two-sided Rayleigh functional u^H T(rho) v = sum_k phi_k(rho) a_k.
// grid (nb, nterms); one wave per row of A_k, its lanes across the row (coalesced).
__global__ __launch_bounds__(256) void rayleigh_terms_kernel(ProblemDev pd, const double2* __restrict__ U,
                                                             const double2* __restrict__ Vv, long long xstride,
                                                             double2* __restrict__ out) {
  const int b = blockIdx.x, k = blockIdx.y, n = pd.n;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double2* u = U + (long long)b * xstride;
  const double2* v = Vv + (long long)b * xstride;
  const double2* A = pd.A[k];
  double2 acc = cmk<double>(0, 0);
  if (A) {
    for (int i = w; i < n; i += 4) {
      double2 r = cmk<double>(0, 0);
      for (int j = lane; j < n; j += 64) r = cfma<double>(r, A[(long long)i * n + j], v[j]);
      acc = cfma<double>(acc, cmk<double>(u[i].x, -u[i].y), r);
    }
  } else {
    for (int i = threadIdx.x; i < n; i += 256) acc = cfma<double>(acc, cmk<double>(u[i].x, -u[i].y), v[i]);
  }
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  __shared__ double2 part[4];
  if (lane == 0) part[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    out[(long long)b * MAX_TERMS + k] =
        cmk<double>(part[0].x + part[1].x + part[2].x + part[3].x, part[0].y + part[1].y + part[2].y + part[3].y);
}

hipError_t launch_rayleigh_terms(const ProblemDev& pd, const double2* U, const double2* V, long long xstride,
                                 int nb, double2* out, hipStream_t st) {
  if (pd.nterms < 1 || pd.nterms > MAX_TERMS || nb < 1) return hipErrorInvalidValue;
  rayleigh_terms_kernel<<<dim3(nb, pd.nterms), 256, 0, st>>>(pd, U, V, xstride, out);
  return hipGetLastError();
}

// W[b] = -z_b I + A0 + A1 .* exp(-tau .* z_b), one thread per entry (rows coalesced);
// grid (ceil(n^2 / 256), nb)
__global__ __launch_bounds__(256) void elementwise_delay_kernel(const double2* __restrict__ A0,
                                                                const double2* __restrict__ A1,
                                                                const double* __restrict__ tau, int n,
                                                                const double2* __restrict__ z, double2* __restrict__ W,
                                                                long long mstride) {
  const long long nn = (long long)n * n;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (e >= nn) return;
  const double2 zb = z[b];
  const double t = tau[e];
  const double m = exp(-t * zb.x);
  double sn, cs;
  sincos(-t * zb.y, &sn, &cs);
  const double2 a0 = A0[e], a1 = A1[e];
  double2 v = cmk<double>(a0.x + m * (a1.x * cs - a1.y * sn), a0.y + m * (a1.x * sn + a1.y * cs));
  const int i = (int)(e / n), j = (int)(e - (long long)i * n);
  if (i == j) { v.x -= zb.x; v.y -= zb.y; }
  W[(long long)b * mstride + e] = v;
}

hipError_t launch_elementwise_delay(const double2* A0, const double2* A1, const double* tau, int n, const double2* z,
                                    int nb, double2* W, long long mstride, hipStream_t st) {
  if (n < 1 || nb < 1 || nb > 65535) return hipErrorInvalidValue;
  const long long nn = (long long)n * n;
  elementwise_delay_kernel<<<dim3((unsigned)((nn + 255) / 256), (unsigned)nb), 256, 0, st>>>(A0, A1, tau, n, z, W,
                                                                                              mstride);
  return hipGetLastError();
}

// Scattering poles of the sound-soft unit disk: W[b] = (I + K_n(k_b)) / 2 on P
// equispaced points t_j = 2 pi j / P of the unit circle, K the double-layer operator
// (kernel 2 dPhi/dnu(y) = -(i k r / 4) H1(k r), r = 2 |sin((t_i - t_j)/2)|), split as
// L1 ln(4 sin^2) + L2 with L1 = (k r / 4 pi) J1(k r) and integrated by Kress's rule
// (log weights R_ij, trapezoid pi / (P/2) for L2).  J1 and the logarithm-free part of
// Y1 come from their power series in w = k r / 2 (|w| <= |k|: all terms decay after
// q ~ |w|, at most 60 of them); L2 = -1/(2 pi) on the diagonal.  One thread per entry,
// grid (ceil(P^2 / 256), nb).
// |k| up to which the power series are used: |w| <= |k|, the largest term is about
// |k|^(2q+1) / (q! (q+1)!) at q ~ |k| (~1e7 at |k| = 10, so ~1e-9 of the sums is lost to
// cancellation) and 60 terms reach the 1e-18 stopping level
constexpr double CDL_MAX_K = 10.0;
__global__ __launch_bounds__(256) void circle_double_layer_kernel(int P, const double2* __restrict__ kz,
                                                                  double2* __restrict__ W, long long mstride) {
  constexpr double PI = 3.141592653589793238, EULER = 0.5772156649015328606;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (e >= P * P) return;
  const int i = e / P, j = e - i * P;
  const int m = P / 2;
  const double2 k = kz[b];
  if (!(k.x * k.x + k.y * k.y <= CDL_MAX_K * CDL_MAX_K)) {
    // beyond the series' range (or a non-finite node): the node's matrix is NaN, which
    // the sweep reports as a non-finite node solution (warning, disk flagged)
    W[(long long)b * mstride + e] = cmk<double>(__builtin_nan(""), __builtin_nan(""));
    return;
  }
  const double d = 2.0 * PI * (double)(i - j) / (double)P;
  double R = 0.0;
  for (int l = 1; l < m; ++l) R += cos(l * d) / l;
  R = -(2.0 * PI / m) * R - (PI / ((double)m * m)) * cos(m * d);
  double2 L1 = cmk<double>(0.0, 0.0), L2 = cmk<double>(-1.0 / (2.0 * PI), 0.0);
  if (i != j) {
    const double r = 2.0 * fabs(sin(0.5 * d));
    const double2 z = cmk<double>(k.x * r, k.y * r);
    const double2 w = cmk<double>(0.5 * z.x, 0.5 * z.y);
    const double2 mw2 = cmk<double>(-(w.x * w.x - w.y * w.y), -2.0 * w.x * w.y);   // -w^2
    const double aw2 = w.x * w.x + w.y * w.y;
    double2 term = w;                                  // (-1)^q w^(2q+1) / (q! (q+1)!)
    double pa = -EULER, pb = 1.0 - EULER;              // psi(q+1), psi(q+2)
    double2 J1 = term, SY = cscale<double>(term, pa + pb);
    for (int q = 1; q < 60; ++q) {
      term = cscale<double>(cmul<double>(term, mw2), 1.0 / ((double)q * (q + 1)));
      pa += 1.0 / q;
      pb += 1.0 / (q + 1);
      J1 = cadd<double>(J1, term);
      SY = cfma<double>(SY, term, cmk<double>(pa + pb, 0.0));
      const double tm = sqrt(cabs2<double>(term)) * (pa + pb + 1.0);
      if ((double)q * (q + 1) > aw2 && tm < 1e-18 * (sqrt(cabs2<double>(J1)) + sqrt(cabs2<double>(SY))))
        break;
    }
    const double2 zJ1 = cmul<double>(z, J1);
    L1 = cscale<double>(zJ1, 1.0 / (4.0 * PI));
    const double2 lk = cmk<double>(log(0.5 * sqrt(k.x * k.x + k.y * k.y)), atan2(k.y, k.x));   // ln(k / 2)
    // L2 = -(i/4) z J1 - 1/(2 pi) + z J1 ln(k/2) / (2 pi) - z SY / (4 pi)
    const double2 a = cmul<double>(zJ1, lk), c = cmul<double>(z, SY);
    L2 = cmk<double>(0.25 * zJ1.y - 1.0 / (2.0 * PI) + a.x / (2.0 * PI) - c.x / (4.0 * PI),
                     -0.25 * zJ1.x + a.y / (2.0 * PI) - c.y / (4.0 * PI));
  }
  const double tw = PI / m;
  double2 v = cmk<double>(0.5 * (R * L1.x + tw * L2.x), 0.5 * (R * L1.y + tw * L2.y));
  if (i == j) v.x += 0.5;
  W[(long long)b * mstride + e] = v;
}

hipError_t launch_circle_double_layer(int P, const double2* k, int nb, double2* W, long long mstride, hipStream_t st) {
  if (P < 4 || (P & 1) || P > 4096 || nb < 1 || nb > 65535) return hipErrorInvalidValue;
  circle_double_layer_kernel<<<dim3((unsigned)((P * P + 255) / 256), (unsigned)nb), 256, 0, st>>>(P, k, W, mstride);
  return hipGetLastError();
}

// a[i] = v for i < n (a fill kernel instead of a memset node, so graph captures replay it)
__global__ void fill_int_kernel(int* a, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ----------------------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_assemble(const ProblemDev& pd, const double2* znode, c2<T>* W, long long mstride, int nbatch,
                           hipStream_t st) {
  const long long nn = (long long)pd.n * pd.n;
  dim3 grid((unsigned)((nn + 511) / 512), (unsigned)((nbatch + ASM_NPB - 1) / ASM_NPB));
  assemble_kernel<T><<<grid, 256, 0, st>>>(pd, znode, W, mstride, nbatch);
  return hipGetLastError();
}
template hipError_t launch_assemble<double>(const ProblemDev&, const double2*, c2<double>*, long long, int, hipStream_t);
template hipError_t launch_assemble<float>(const ProblemDev&, const double2*, c2<float>*, long long, int, hipStream_t);

hipError_t launch_rhs(const double2* F, int s, const double2* V, int L, int n, double2* X, long long xstride,
                      int nbatch, hipStream_t st) {
  dim3 grid((unsigned)((n * (s + L) + 255) / 256), (unsigned)nbatch);
  rhs_kernel<<<grid, 256, 0, st>>>(F, s, V, L, n, X, xstride, nbatch);
  return hipGetLastError();
}

hipError_t launch_sums(const double2* X, long long xstride, const double2* wts, const double2* zn, int N, int n,
                       int s, int L, double2* PfN, double2* PfN2, double2* C0, double2* C1, const int* disk_ids,
                       int ndisks, const long long* soff, int* nonfin, hipStream_t st) {
  dim3 grid((unsigned)((n * (s + L) + 255) / 256), (unsigned)ndisks);
  sums_kernel<<<grid, 256, 0, st>>>(X, xstride, wts, zn, N, n, s, L, PfN, PfN2, C0, C1, disk_ids, soff, nonfin);
  return hipGetLastError();
}

hipError_t launch_profile(const double2* X, long long xstride, int N, int n, int s, int m, double* prof,
                          const int* disk_ids, int ndisks, hipStream_t st) {
  profile_kernel<<<dim3((unsigned)N, (unsigned)ndisks), 256, 0, st>>>(X, xstride, N, n, s, m, prof, disk_ids);
  return hipGetLastError();
}

hipError_t launch_indicator(const double2* PfN, const double2* PfN2, const int* dn, const long long* soff, int s,
                            double tol, double* ind, unsigned char* flags, const int* sing, const int* nonfin,
                            int N, const double* prof, const double* rad, double floor, int ndisks, hipStream_t st) {
  indicator_kernel<<<ndisks, 256, 0, st>>>(PfN, PfN2, dn, soff, s, tol, ind, flags, sing, nonfin, N, prof, rad,
                                           floor);
  return hipGetLastError();
}

hipError_t launch_residual(const ProblemDev& pd, const double2* znode, const double2* X, const double2* F, int s,
                           const double2* V, int L, long long xstride, int m, int nbatch, double2* R,
                           const int* active, hipStream_t st) {
  dim3 grid((unsigned)((pd.n + 63) / 64), (unsigned)((nbatch * m + 63) / 64));
  residual_kernel<<<grid, 256, 0, st>>>(pd, znode, X, F, s, V, L, xstride, m, nbatch, R, active);
  return hipGetLastError();
}

hipError_t launch_norms(const double2* R, const double2* X, long long xstride, int len, double* rn2, double* xn2,
                        int nbatch, hipStream_t st) {
  norms_kernel<<<nbatch, 256, 0, st>>>(R, X, xstride, len, rn2, xn2);
  return hipGetLastError();
}

hipError_t launch_axpy(double2* X, const double2* D, long long xstride, int len, const int* active, int nbatch,
                       hipStream_t st) {
  axpy_kernel<<<dim3((unsigned)((len + 255) / 256), (unsigned)nbatch), 256, 0, st>>>(X, D, xstride, len, active);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* a, int v, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  fill_int_kernel<<<(n + 255) / 256, 256, 0, st>>>(a, v, n);
  return hipGetLastError();
}

}  // namespace nep
