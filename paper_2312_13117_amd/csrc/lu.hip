// Batched complex LU with partial pivoting (the node systems of eq (2.4)) and the
// matching triangular solves, for a batch of equal-order matrices.
//
// Storage: matrix b of the batch is row-major n x n at W + b*mstride (complex pairs).
// Right-looking blocked factorisation with panel width NB.  Step s (k0 = s*NB):
//   1. lu_panel_kernel   : factor the m x nbk panel (m = n - k0) with pivot search over
//                          the whole column, inner blocks of IB columns held in
//                          registers; record the step's row exchange as a compact
//                          permutation (new row pos[i] = old row src[i]) and the inverses
//                          of the diagonal blocks L11 (unit lower) and U11 (upper).
//   2. lu_gemm_kernel<TRSM>: apply the row exchange to the columns right of the panel and
//                          form U12 = inv(L11) * P A12 on the matrix cores.
//   3. lu_gemm_kernel<UPDATE>: A22 -= L21 * U12 on the matrix cores.
// Row exchanges are applied only right of each panel; the solve applies each step's
// exchange to the right-hand side before that step's block column of L, which is
// equivalent to LAPACK's fully swapped factor.
#include "common.h"
#include "lu.h"

namespace nep {

// ----------------------------------------------------------------------------- panel
// One workgroup of NT threads per matrix.  Row r >= k0 belongs to thread (r-k0) % NT,
// slot (r-k0) / NT, so n - k0 <= NT * RPT.
template <typename T, int NB, int IB, int NT, int RPT>
__global__ __launch_bounds__(NT) void lu_panel_kernel(c2<T>* __restrict__ W, long long mstride, int n,
                                                      int k0, int step, int* __restrict__ ipiv,
                                                      int* __restrict__ perm, long long perm_stride,
                                                      c2<T>* __restrict__ Linv, c2<T>* __restrict__ Uinv,
                                                      long long inv_stride, int* __restrict__ info) {
  constexpr int NW = NT / 64;
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  c2<T>* A = W + (long long)b * mstride;
  const int nbk = min(NB, n - k0);

  __shared__ c2<T> prow[IB];
  __shared__ c2<T> crow[IB];
  __shared__ T red_v[NW];
  __shared__ int red_r[NW];
  __shared__ int s_piv;
  __shared__ int s_ipiv[NB];
  __shared__ c2<T> Lb[IB][IB];
  __shared__ c2<T> Ub[IB][NB];
  __shared__ int s_pos[2 * NB], s_src[2 * NB];
  __shared__ int s_cnt;
  __shared__ c2<T> Mtri[NB][NB + 1];

  c2<T> a[RPT][IB];
  for (int c0 = k0; c0 < k0 + nbk; c0 += IB) {
    const int ib = min(IB, k0 + nbk - c0);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = k0 + t + q * NT;
#pragma unroll
      for (int jj = 0; jj < IB; ++jj)
        a[q][jj] = (r >= c0 && r < n && jj < ib) ? A[(long long)r * n + c0 + jj] : czero<T>();
    }
    for (int jj = 0; jj < ib; ++jj) {
      const int c = c0 + jj;
      // ---- pivot search: max |re|+|im| over rows r >= c, first index on ties
      T bv = T(-1);
      int br = 0x7fffffff;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = k0 + t + q * NT;
        if (r >= c && r < n) {
          // select the column jj without dynamic register indexing
          c2<T> v = a[q][0];
#pragma unroll
          for (int u = 1; u < IB; ++u)
            if (u == jj) v = a[q][u];
          const T m = cabs1<T>(v);
          if (m > bv) { bv = m; br = r; }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const T ov = __shfl_xor(bv, o, 64);
        const int orr = __shfl_xor(br, o, 64);
        if (ov > bv || (ov == bv && orr < br)) { bv = ov; br = orr; }
      }
      if (lane == 0) { red_v[wave] = bv; red_r[wave] = br; }
      __syncthreads();
      if (t == 0) {
        T v = red_v[0];
        int rr = red_r[0];
        for (int w = 1; w < NW; ++w)
          if (red_v[w] > v || (red_v[w] == v && red_r[w] < rr)) { v = red_v[w]; rr = red_r[w]; }
        if (!(v > T(0))) {        // exactly zero column (or NaN): keep the diagonal row
          rr = c;
          if (info[b] == 0) info[b] = c + 1;
        }
        s_piv = rr;
        s_ipiv[c - k0] = rr;
        ipiv[(long long)b * n + c] = rr;
      }
      __syncthreads();
      const int p = s_piv;
      const int tc = (c - k0) % NT, qc = (c - k0) / NT;
      const int tp = (p - k0) % NT, qp = (p - k0) / NT;
      // ---- exchange rows c and p inside the register block; prow = new row c
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (t == tp && q == qp)
#pragma unroll
          for (int u = 0; u < IB; ++u) prow[u] = a[q][u];
        if (p != c && t == tc && q == qc)
#pragma unroll
          for (int u = 0; u < IB; ++u) crow[u] = a[q][u];
      }
      __syncthreads();
      if (p != c) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (t == tp && q == qp)
#pragma unroll
            for (int u = 0; u < IB; ++u) a[q][u] = crow[u];
          if (t == tc && q == qc)
#pragma unroll
            for (int u = 0; u < IB; ++u) a[q][u] = prow[u];
        }
      }
      // ---- eliminate below the pivot
      c2<T> piv = prow[0];
#pragma unroll
      for (int u = 1; u < IB; ++u)
        if (u == jj) piv = prow[u];
      if (piv.x != T(0) || piv.y != T(0)) {
        const c2<T> rp = crcp<T>(piv);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = k0 + t + q * NT;
          if (r > c && r < n) {
            c2<T> l = a[q][0];
#pragma unroll
            for (int u = 1; u < IB; ++u)
              if (u == jj) l = a[q][u];
            l = cmul<T>(l, rp);
#pragma unroll
            for (int u = 0; u < IB; ++u) {
              if (u == jj) a[q][u] = l;
              else if (u > jj) a[q][u] = cfms<T>(a[q][u], l, prow[u]);
            }
          }
        }
      }
      __syncthreads();
    }
    // ---- write back the inner block
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = k0 + t + q * NT;
      if (r >= c0 && r < n)
#pragma unroll
        for (int u = 0; u < IB; ++u)
          if (u < ib) A[(long long)r * n + c0 + u] = a[q][u];
    }
    __syncthreads();
    // ---- the inner block's row exchanges on the other panel columns
    {
      const int nleft = c0 - k0, nother = nbk - ib;
      for (int e = t; e < nother; e += NT) {
        const int col = (e < nleft) ? k0 + e : c0 + ib + (e - nleft);
        for (int u = 0; u < ib; ++u) {
          const int c = c0 + u, p = s_ipiv[c - k0];
          if (p != c) {
            const c2<T> x = A[(long long)c * n + col];
            A[(long long)c * n + col] = A[(long long)p * n + col];
            A[(long long)p * n + col] = x;
          }
        }
      }
    }
    __syncthreads();
    // ---- right part of the panel: U rows of this block, then the rank-ib update
    const int cr0 = c0 + ib, nr = k0 + nbk - cr0;
    if (nr > 0) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = k0 + t + q * NT;
        if (r >= c0 && r < c0 + ib)
#pragma unroll
          for (int u = 0; u < IB; ++u) Lb[r - c0][u] = a[q][u];
      }
      __syncthreads();
      for (int e = t; e < nr; e += NT) {
        c2<T> x[IB];
#pragma unroll
        for (int i = 0; i < IB; ++i) x[i] = (i < ib) ? A[(long long)(c0 + i) * n + cr0 + e] : czero<T>();
#pragma unroll
        for (int i = 1; i < IB; ++i)
#pragma unroll
          for (int j = 0; j < IB; ++j)
            if (j < i) x[i] = cfms<T>(x[i], Lb[i][j], x[j]);
#pragma unroll
        for (int i = 0; i < IB; ++i)
          if (i < ib) { A[(long long)(c0 + i) * n + cr0 + e] = x[i]; Ub[i][e] = x[i]; }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = k0 + t + q * NT;
        if (r >= cr0 && r < n) {
          c2<T>* row = A + (long long)r * n + cr0;
          for (int e = 0; e < nr; ++e) {
            c2<T> acc = row[e];
#pragma unroll
            for (int i = 0; i < IB; ++i)
              if (i < ib) acc = cfms<T>(acc, a[q][i], Ub[i][e]);
            row[e] = acc;
          }
        }
      }
      __syncthreads();
    }
  }

  // ---- compact permutation of this step: new row s_pos[i] holds old row s_src[i]
  if (t == 0) {
    int cnt = nbk;
    for (int i = 0; i < nbk; ++i) { s_pos[i] = k0 + i; s_src[i] = k0 + i; }
    for (int i = 0; i < nbk; ++i) {
      const int p = s_ipiv[i];
      if (p == k0 + i) continue;
      int ip;
      if (p < k0 + nbk) {
        ip = p - k0;
      } else {
        ip = -1;
        for (int j = nbk; j < cnt; ++j)
          if (s_pos[j] == p) { ip = j; break; }
        if (ip < 0) { ip = cnt; s_pos[cnt] = p; s_src[cnt] = p; ++cnt; }
      }
      const int x = s_src[i]; s_src[i] = s_src[ip]; s_src[ip] = x;
    }
    s_cnt = cnt;
  }
  __syncthreads();
  {
    int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NB);
    for (int i = t; i < 2 * NB; i += NT) {
      P[1 + i] = (i < s_cnt) ? s_pos[i] : -1;
      P[1 + 2 * NB + i] = (i < s_cnt) ? s_src[i] : -1;
    }
    if (t == 0) P[0] = s_cnt;
  }

  // ---- inverse of the unit lower diagonal block L11 (column sweep from the right:
  //      column j of inv(L) = -inv(L)[j+1:, j+1:] * L[j+1:, j], one sync per column)
  c2<T>* Li = Linv + (long long)b * inv_stride + (long long)step * NB * NB;
  c2<T>* Ui = Uinv + (long long)b * inv_stride + (long long)step * NB * NB;
  for (int e = t; e < nbk * nbk; e += NT) {
    const int i = e / nbk, j = e % nbk;
    Mtri[i][j] = A[(long long)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  for (int j = nbk - 2; j >= 0; --j) {
    // rows i > j: new M[i][j] = -(L[i][j] + sum_{j<l<i} X[i][l] L[l][j]),  X = current inv
    c2<T> v = czero<T>();
    const int i = j + 1 + t;
    if (t < nbk - 1 - j) {
      v = Mtri[i][j];
      for (int l = j + 1; l < i; ++l) v = cfma<T>(v, Mtri[i][l], Mtri[l][j]);
      v = cmk<T>(-v.x, -v.y);
    }
    __syncthreads();
    if (t < nbk - 1 - j) Mtri[i][j] = v;
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += NT) {
    const int i = e / NB, j = e % NB;
    c2<T> v = czero<T>();
    if (i < nbk && j < nbk) v = (i == j) ? cmk<T>(T(1), T(0)) : (j < i ? Mtri[i][j] : czero<T>());
    Li[e] = v;
  }
  __syncthreads();
  // ---- inverse of the upper diagonal block U11 (row sweep from the bottom:
  //      row i of inv(U) = -inv(U_ii) * U[i, i+1:] * inv(U)[i+1:, i+1:])
  for (int e = t; e < nbk * nbk; e += NT) {
    const int i = e / nbk, j = e % nbk;
    Mtri[i][j] = A[(long long)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  for (int i = nbk - 1; i >= 0; --i) {
    const c2<T> d = Mtri[i][i];
    const c2<T> rd = (d.x != T(0) || d.y != T(0)) ? crcp<T>(d) : cmk<T>(T(0), T(0));
    c2<T> v = czero<T>();
    const int j = i + 1 + t;
    if (t < nbk - 1 - i) {
      for (int l = i + 1; l <= j; ++l) v = cfma<T>(v, Mtri[i][l], Mtri[l][j]);
      v = cmul<T>(cmk<T>(-v.x, -v.y), rd);
    }
    __syncthreads();
    if (t < nbk - 1 - i) Mtri[i][j] = v;
    if (t == 0) Mtri[i][i] = rd;
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += NT) {
    const int i = e / NB, j = e % NB;
    c2<T> v = czero<T>();
    if (i < nbk && j < nbk && j >= i) v = Mtri[i][j];
    Ui[e] = v;
  }
}

// ----------------------------------------------------------------------------- matrix-core steps
// 256 threads = 4 waves; a workgroup owns a 64 x 64 tile, a wave a 32 x 32 quarter
// (2 x 2 blocks of 16 x 16, real and imaginary accumulators).  Workgroup ids are
// spread round-robin over the 8 XCDs; all tiles of one matrix are mapped to one XCD
// so the panels L21 / U12 it re-reads stay in that XCD's L2.
enum { GEMM_UPDATE = 0, GEMM_TRSM = 1 };

template <typename T, int MODE>
__global__ __launch_bounds__(256) void lu_gemm_kernel(c2<T>* __restrict__ W, long long mstride, int n, int k0,
                                                      int nbk, int step, int nbatch, int tiles_r, int tiles_c,
                                                      const int* __restrict__ perm, long long perm_stride,
                                                      const c2<T>* __restrict__ Linv, long long inv_stride) {
  constexpr int NBMAX = 64;
  const int wg = blockIdx.x;
  const int xcd = wg & 7, slot = wg >> 3;
  const int ntile = tiles_r * tiles_c;
  const int b = (slot / ntile) * 8 + xcd;
  if (b >= nbatch) return;
  const int tile = slot % ntile;
  const int tr = tile / tiles_c, tcn = tile % tiles_c;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  c2<T>* A = W + (long long)b * mstride;
  const int kend = k0 + nbk;
  const int R0 = (MODE == GEMM_UPDATE ? kend : k0) + tr * 64;
  const int C0 = kend + tcn * 64;
  const int rlim = (MODE == GEMM_UPDATE) ? n : kend;
  const int rb = R0 + (wave >> 1) * 32, cb = C0 + (wave & 1) * 32;
  const int l16 = lane & 15, kq = lane >> 4;

  __shared__ int s_src[2 * NBMAX], s_pos[2 * NBMAX];
  __shared__ int s_cnt;
  const c2<T>* Li = nullptr;
  if (MODE == GEMM_TRSM) {
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NBMAX);
    if (t == 0) s_cnt = P[0];
    for (int i = t; i < 2 * NBMAX; i += 256) { s_pos[i] = P[1 + i]; s_src[i] = P[1 + 2 * NBMAX + i]; }
    __syncthreads();
    Li = Linv + (long long)b * inv_stride + (long long)step * NBMAX * NBMAX;
  }

  acc4<T> cre[2][2], cim[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      cre[bi][bj] = acc_zero<T>();
      cim[bi][bj] = acc_zero<T>();
      if (MODE == GEMM_UPDATE) {
        const int col = cb + bj * 16 + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb + bi * 16 + acc_row<T>(lane, r);
          if (row < n && col < n) {
            const c2<T> v = A[(long long)row * n + col];
            cre[bi][bj][r] = v.x;
            cim[bi][bj][r] = v.y;
          }
        }
      }
    }

  // displaced rows of the row exchange (TRSM mode): old values, read before any write
  constexpr int DMAX = (NBMAX * 64) / 256;
  c2<T> dval[DMAX];
  int ndisp = 0;
  if (MODE == GEMM_TRSM) {
    ndisp = s_cnt - nbk;
#pragma unroll
    for (int q = 0; q < DMAX; ++q) {
      const int e = t + q * 256;
      const int i = nbk + e / 64, col = C0 + (e & 63);
      dval[q] = (e < ndisp * 64 && col < n) ? A[(long long)s_src[i] * n + col] : czero<T>();
    }
  }

  for (int kk = 0; kk < nbk; kk += 4) {
    const int k = kk + kq;
    c2<T> af[2], bf[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int row = rb + bi * 16 + l16;
      if (MODE == GEMM_UPDATE)
        af[bi] = (row < n && k < nbk) ? A[(long long)row * n + k0 + k] : czero<T>();
      else
        af[bi] = (row < kend && k < nbk) ? Li[(row - k0) * NBMAX + k] : czero<T>();
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = cb + bj * 16 + l16;
      if (k < nbk && col < n) {
        const int srow = (MODE == GEMM_UPDATE) ? (k0 + k) : s_src[k];
        bf[bj] = A[(long long)srow * n + col];
      } else {
        bf[bj] = czero<T>();
      }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        if (MODE == GEMM_UPDATE) {   // C -= A B
          cre[bi][bj] = mfma16(-af[bi].x, bf[bj].x, cre[bi][bj]);
          cim[bi][bj] = mfma16(-af[bi].x, bf[bj].y, cim[bi][bj]);
          cre[bi][bj] = mfma16(af[bi].y, bf[bj].y, cre[bi][bj]);
          cim[bi][bj] = mfma16(-af[bi].y, bf[bj].x, cim[bi][bj]);
        } else {                     // C = A B
          cre[bi][bj] = mfma16(af[bi].x, bf[bj].x, cre[bi][bj]);
          cim[bi][bj] = mfma16(af[bi].x, bf[bj].y, cim[bi][bj]);
          cre[bi][bj] = mfma16(-af[bi].y, bf[bj].y, cre[bi][bj]);
          cim[bi][bj] = mfma16(af[bi].y, bf[bj].x, cim[bi][bj]);
        }
      }
  }
  if (MODE == GEMM_TRSM) __syncthreads();   // every wave has read its operands

#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = cb + bj * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb + bi * 16 + acc_row<T>(lane, r);
        if (row < rlim && col < n) A[(long long)row * n + col] = cmk<T>(cre[bi][bj][r], cim[bi][bj][r]);
      }
    }
  if (MODE == GEMM_TRSM) {
#pragma unroll
    for (int q = 0; q < DMAX; ++q) {
      const int e = t + q * 256;
      const int i = nbk + e / 64, col = C0 + (e & 63);
      if (e < ndisp * 64 && col < n) A[(long long)s_pos[i] * n + col] = dval[q];
    }
  }
}

// ----------------------------------------------------------------------------- solves
// One workgroup per matrix; the right-hand side block X (n x m, complex128, row-major)
// is solved in place in the factor's arithmetic T.  TRANS = false: A x = b;
// TRANS = true: A^H x = b.
template <typename T, int NB, bool TRANS>
__global__ __launch_bounds__(256) void lu_solve_kernel(const c2<T>* __restrict__ W, long long mstride, int n,
                                                       const int* __restrict__ perm, long long perm_stride,
                                                       const c2<T>* __restrict__ Linv, const c2<T>* __restrict__ Uinv,
                                                       long long inv_stride, double2* __restrict__ X,
                                                       long long xstride, int m, const int* __restrict__ active) {
  constexpr int MMAX = 32;
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const int t = threadIdx.x;
  const c2<T>* A = W + (long long)b * mstride;
  double2* Xb = X + (long long)b * xstride;
  const int nsteps = (n + NB - 1) / NB;
  __shared__ c2<T> Y[NB][MMAX];
  __shared__ c2<T> Z[NB][MMAX];
  __shared__ int s_pos[2 * NB], s_src[2 * NB];
  __shared__ int s_cnt;
  constexpr int GMAX = (2 * NB * MMAX + 255) / 256;

  auto load_perm = [&](int s) {
    const int* P = perm + (long long)b * perm_stride + (long long)s * (1 + 4 * NB);
    __syncthreads();
    if (t == 0) s_cnt = P[0];
    for (int i = t; i < 2 * NB; i += 256) { s_pos[i] = P[1 + i]; s_src[i] = P[1 + 2 * NB + i]; }
    __syncthreads();
  };
  // new[pos[i]] = old[src[i]] (forward) or new[src[i]] = old[pos[i]] (inverse)
  auto permute = [&](bool inverse) {
    const int cnt = s_cnt;
    c2<T> g[GMAX];
#pragma unroll
    for (int q = 0; q < GMAX; ++q) {
      const int e = t + q * 256;
      const int i = e / m, c = e % m;
      g[q] = (e < cnt * m) ? ccast<T, double>(Xb[(long long)(inverse ? s_pos[i] : s_src[i]) * m + c]) : czero<T>();
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GMAX; ++q) {
      const int e = t + q * 256;
      const int i = e / m, c = e % m;
      if (e < cnt * m) Xb[(long long)(inverse ? s_src[i] : s_pos[i]) * m + c] = ccast<double, T>(g[q]);
    }
    __syncthreads();
  };

  if (!TRANS) {
    // forward: for each step, exchange rows, y = inv(L11) x_top, x_rest -= L21 y
    for (int s = 0; s < nsteps; ++s) {
      const int k0 = s * NB, nbk = min(NB, n - k0), kend = k0 + nbk;
      load_perm(s);
      permute(false);
      for (int e = t; e < nbk * m; e += 256) Z[e / m][e % m] = ccast<T, double>(Xb[(long long)(k0 + e / m) * m + e % m]);
      __syncthreads();
      const c2<T>* Li = Linv + (long long)b * inv_stride + (long long)s * NB * NB;
      for (int e = t; e < nbk * m; e += 256) {
        const int i = e / m, c = e % m;
        c2<T> acc = czero<T>();
        for (int j = 0; j <= i; ++j) acc = cfma<T>(acc, Li[i * NB + j], Z[j][c]);
        Y[i][c] = acc;
        Xb[(long long)(k0 + i) * m + c] = ccast<double, T>(acc);
      }
      __syncthreads();
      for (int e = t; e < (n - kend) * m; e += 256) {
        const int r = kend + e / m, c = e % m;
        const c2<T>* Lr = A + (long long)r * n + k0;
        c2<T> acc = ccast<T, double>(Xb[(long long)r * m + c]);
        for (int j = 0; j < nbk; ++j) acc = cfms<T>(acc, Lr[j], Y[j][c]);
        Xb[(long long)r * m + c] = ccast<double, T>(acc);
      }
      __syncthreads();
    }
    // backward: x_top = inv(U11) (x_top - U12 x_rest)
    for (int s = nsteps - 1; s >= 0; --s) {
      const int k0 = s * NB, nbk = min(NB, n - k0), kend = k0 + nbk;
      for (int e = t; e < nbk * m; e += 256) {
        const int i = e / m, c = e % m;
        const c2<T>* Ur = A + (long long)(k0 + i) * n;
        c2<T> acc = ccast<T, double>(Xb[(long long)(k0 + i) * m + c]);
        for (int j = kend; j < n; ++j) acc = cfms<T>(acc, Ur[j], ccast<T, double>(Xb[(long long)j * m + c]));
        Z[i][c] = acc;
      }
      __syncthreads();
      const c2<T>* Ui = Uinv + (long long)b * inv_stride + (long long)s * NB * NB;
      for (int e = t; e < nbk * m; e += 256) {
        const int i = e / m, c = e % m;
        c2<T> acc = czero<T>();
        for (int j = i; j < nbk; ++j) acc = cfma<T>(acc, Ui[i * NB + j], Z[j][c]);
        Xb[(long long)(k0 + i) * m + c] = ccast<double, T>(acc);
      }
      __syncthreads();
    }
  } else {
    // A = P_0^T L_0 ... P_{S-1}^T L_{S-1} U  =>  A^H x = b:  w = U^{-H} b, then for
    // s = S-1..0: w_blk = inv(L11)^H (w_blk - L21^H w_rest), w = P_s^T w.
    for (int s = 0; s < nsteps; ++s) {   // U^H is lower triangular: forward over steps
      const int k0 = s * NB, nbk = min(NB, n - k0);
      // z_blk = b_blk - sum_{j < k0} U[j, blk]^H w_j
      for (int e = t; e < nbk * m; e += 256) {
        const int i = e / m, c = e % m;
        c2<T> acc = ccast<T, double>(Xb[(long long)(k0 + i) * m + c]);
        for (int j = 0; j < k0; ++j) {
          const c2<T> u = A[(long long)j * n + k0 + i];
          acc = csub<T>(acc, cconjmul<T>(u, ccast<T, double>(Xb[(long long)j * m + c])));
        }
        Z[i][c] = acc;
      }
      __syncthreads();
      const c2<T>* Ui = Uinv + (long long)b * inv_stride + (long long)s * NB * NB;
      for (int e = t; e < nbk * m; e += 256) {
        const int i = e / m, c = e % m;
        c2<T> acc = czero<T>();
        for (int j = 0; j <= i; ++j) acc = cadd<T>(acc, cconjmul<T>(Ui[j * NB + i], Z[j][c]));
        Xb[(long long)(k0 + i) * m + c] = ccast<double, T>(acc);
      }
      __syncthreads();
    }
    for (int s = nsteps - 1; s >= 0; --s) {
      const int k0 = s * NB, nbk = min(NB, n - k0), kend = k0 + nbk;
      for (int e = t; e < nbk * m; e += 256) {
        const int i = e / m, c = e % m;
        c2<T> acc = ccast<T, double>(Xb[(long long)(k0 + i) * m + c]);
        for (int r = kend; r < n; ++r) {
          const c2<T> l = A[(long long)r * n + k0 + i];
          acc = csub<T>(acc, cconjmul<T>(l, ccast<T, double>(Xb[(long long)r * m + c])));
        }
        Z[i][c] = acc;
      }
      __syncthreads();
      const c2<T>* Li = Linv + (long long)b * inv_stride + (long long)s * NB * NB;
      for (int e = t; e < nbk * m; e += 256) {
        const int i = e / m, c = e % m;
        c2<T> acc = czero<T>();
        for (int j = i; j < nbk; ++j) acc = cadd<T>(acc, cconjmul<T>(Li[j * NB + i], Z[j][c]));
        Xb[(long long)(k0 + i) * m + c] = ccast<double, T>(acc);
      }
      load_perm(s);
      permute(true);
    }
  }
}

// ----------------------------------------------------------------------------- launchers
template <typename T>
static int panel_threads(int n) { return n <= 1024 ? 256 : (n <= 2048 ? 512 : 1024); }

template <typename T>
hipError_t lu_factor_batch(c2<T>* W, long long mstride, int n, int nbatch, int* ipiv, int* perm,
                           long long perm_stride, c2<T>* Linv, c2<T>* Uinv, long long inv_stride, int* info,
                           hipStream_t st, LuTimers* tm) {
  constexpr int NB = LU_NB, IB = 8, RPT = 4;
  if (n > 4096 || n < 1) return hipErrorInvalidValue;
  const int nsteps = (n + NB - 1) / NB;
  for (int s = 0; s < nsteps; ++s) {
    const int k0 = s * NB, nbk = min(NB, n - k0), m = n - k0 - nbk;
    const int nt = panel_threads<T>(n);
    if (nt == 256)
      lu_panel_kernel<T, NB, IB, 256, RPT><<<nbatch, 256, 0, st>>>(W, mstride, n, k0, s, ipiv, perm, perm_stride, Linv, Uinv, inv_stride, info);
    else if (nt == 512)
      lu_panel_kernel<T, NB, IB, 512, RPT><<<nbatch, 512, 0, st>>>(W, mstride, n, k0, s, ipiv, perm, perm_stride, Linv, Uinv, inv_stride, info);
    else
      lu_panel_kernel<T, NB, IB, 1024, RPT><<<nbatch, 1024, 0, st>>>(W, mstride, n, k0, s, ipiv, perm, perm_stride, Linv, Uinv, inv_stride, info);
    if (m <= 0) continue;
    const int tc = (m + 63) / 64;
    const long long groups = (nbatch + 7) / 8;
    lu_gemm_kernel<T, GEMM_TRSM><<<dim3((unsigned)(groups * 8 * tc)), 256, 0, st>>>(
        W, mstride, n, k0, nbk, s, nbatch, 1, tc, perm, perm_stride, Linv, inv_stride);
    const bool timed = tm && tm->ev_enabled && tm->npairs < LuTimers::MAXP;
    if (timed) hipEventRecord(tm->ev[2 * tm->npairs], st);
    lu_gemm_kernel<T, GEMM_UPDATE><<<dim3((unsigned)(groups * 8 * tc * tc)), 256, 0, st>>>(
        W, mstride, n, k0, nbk, s, nbatch, tc, tc, perm, perm_stride, Linv, inv_stride);
    if (timed) { hipEventRecord(tm->ev[2 * tm->npairs + 1], st); tm->npairs++; }
    if (tm) {
      tm->gemm_launches += 1;
      tm->gemm_flops += 8.0 * (double)m * (double)m * (double)nbk * (double)nbatch;
    }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t lu_solve_batch(const c2<T>* W, long long mstride, int n, int nbatch, const int* perm, long long perm_stride,
                          const c2<T>* Linv, const c2<T>* Uinv, long long inv_stride, double2* X, long long xstride,
                          int m, bool trans, const int* active, hipStream_t st) {
  if (m > 32 || m < 1) return hipErrorInvalidValue;
  if (trans)
    lu_solve_kernel<T, LU_NB, true><<<nbatch, 256, 0, st>>>(W, mstride, n, perm, perm_stride, Linv, Uinv, inv_stride, X, xstride, m, active);
  else
    lu_solve_kernel<T, LU_NB, false><<<nbatch, 256, 0, st>>>(W, mstride, n, perm, perm_stride, Linv, Uinv, inv_stride, X, xstride, m, active);
  return hipGetLastError();
}

template hipError_t lu_factor_batch<double>(c2<double>*, long long, int, int, int*, int*, long long, c2<double>*,
                                            c2<double>*, long long, int*, hipStream_t, LuTimers*);
template hipError_t lu_factor_batch<float>(c2<float>*, long long, int, int, int*, int*, long long, c2<float>*,
                                           c2<float>*, long long, int*, hipStream_t, LuTimers*);
template hipError_t lu_solve_batch<double>(const c2<double>*, long long, int, int, const int*, long long,
                                           const c2<double>*, const c2<double>*, long long, double2*, long long, int,
                                           bool, const int*, hipStream_t);
template hipError_t lu_solve_batch<float>(const c2<float>*, long long, int, int, const int*, long long,
                                          const c2<float>*, const c2<float>*, long long, double2*, long long, int,
                                          bool, const int*, hipStream_t);

}  // namespace nep
