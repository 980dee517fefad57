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


// ----------------------------------------------------------------------------- small inverses
// In-place inverses of the nbk x nbk diagonal blocks held in LDS (M[i][j]), blocked in
// 8 x 8 tiles: the diagonal tiles are inverted by substitution (one thread per column),
// then each block row is formed from the rows above it (two small products, two
// barriers per block row).
constexpr int TB = 8;

// unit lower: strict lower part of M holds L on entry and inv(L) on exit
template <typename T, int NB, int NT>
__device__ void inv_unit_lower(c2<T> (*M)[NB + 1], c2<T> (*S)[NB], int nbk) {
  const int t = threadIdx.x;
  const int nblk = (nbk + TB - 1) / TB;
  c2<T> x[TB];
  const int col = t;            // one thread per column for the diagonal tiles
  const bool act = col < nbk;
  const int b0 = (col / TB) * TB, b1 = min(b0 + TB, nbk);
  if (act) {
#pragma unroll
    for (int u = 0; u < TB; ++u) x[u] = czero<T>();
    for (int i = col + 1; i < b1; ++i) {
      c2<T> v = M[i][col];
      for (int l = col + 1; l < i; ++l) v = cfma<T>(v, M[i][l], x[l - b0]);
      x[i - b0] = cmk<T>(-v.x, -v.y);
    }
  }
  __syncthreads();
  if (act)
    for (int i = col + 1; i < b1; ++i) M[i][col] = x[i - b0];
  __syncthreads();
  for (int I = 1; I < nblk; ++I) {
    const int r0 = I * TB, r1 = min(r0 + TB, nbk), nr = r1 - r0, nc = r0;
    // S[i][j] = sum_{l = j..r0-1} L[i][l] X[l][j]   (X unit lower, already inverted)
    for (int e = t; e < nr * nc; e += NT) {
      const int i = r0 + e / nc, j = e % nc;
      c2<T> v = M[i][j];                       // l = j term (X[j][j] = 1)
      for (int l = j + 1; l < r0; ++l) v = cfma<T>(v, M[i][l], M[l][j]);
      S[i - r0][j] = v;
    }
    __syncthreads();
    // X[i][j] = -(S[i][j] + sum_{r0 <= l < i} X_II[i][l] S[l][j])
    c2<T> out[(TB * NB + NT - 1) / NT];
    int q = 0;
    for (int e = t; e < nr * nc; e += NT, ++q) {
      const int i = r0 + e / nc, j = e % nc;
      c2<T> v = S[i - r0][j];
      for (int l = r0; l < i; ++l) v = cfma<T>(v, M[i][l], S[l - r0][j]);
      out[q] = cmk<T>(-v.x, -v.y);
    }
    __syncthreads();
    q = 0;
    for (int e = t; e < nr * nc; e += NT, ++q) M[r0 + e / nc][e % nc] = out[q];
    __syncthreads();
  }
}

// upper (non-unit): upper part of M holds U on entry and inv(U) on exit
template <typename T, int NB, int NT>
__device__ void inv_upper(c2<T> (*M)[NB + 1], c2<T> (*S)[NB], int nbk) {
  const int t = threadIdx.x;
  const int nblk = (nbk + TB - 1) / TB;
  c2<T> x[TB];
  const int col = t;
  const bool act = col < nbk;
  const int b0 = (col / TB) * TB;
  if (act) {
#pragma unroll
    for (int u = 0; u < TB; ++u) x[u] = czero<T>();
    const c2<T> d = M[col][col];
    x[col - b0] = (d.x != T(0) || d.y != T(0)) ? crcp<T>(d) : czero<T>();
    for (int i = col - 1; i >= b0; --i) {
      c2<T> v = czero<T>();
      for (int l = i + 1; l <= col; ++l) v = cfma<T>(v, M[i][l], x[l - b0]);
      const c2<T> di = M[i][i];
      const c2<T> rd = (di.x != T(0) || di.y != T(0)) ? crcp<T>(di) : czero<T>();
      x[i - b0] = cmul<T>(cmk<T>(-v.x, -v.y), rd);
    }
  }
  __syncthreads();
  if (act)
    for (int i = b0; i <= col; ++i) M[i][col] = x[i - b0];
  __syncthreads();
  for (int I = nblk - 2; I >= 0; --I) {
    const int r0 = I * TB, r1 = r0 + TB, c0 = r1, nc = nbk - c0;
    // S[i][j] = sum_{l = r1..j} U[i][l] X[l][j]   (j >= r1, X upper already inverted)
    for (int e = t; e < TB * nc; e += NT) {
      const int i = r0 + e / nc, j = c0 + e % nc;
      c2<T> v = czero<T>();
      for (int l = r1; l <= j; ++l) v = cfma<T>(v, M[i][l], M[l][j]);
      S[i - r0][j] = v;
    }
    __syncthreads();
    // X[i][j] = -sum_{i <= l < r1} X_II[i][l] S[l][j]
    c2<T> out[(TB * NB + NT - 1) / NT];
    int q = 0;
    for (int e = t; e < TB * nc; e += NT, ++q) {
      const int i = r0 + e / nc, j = c0 + e % nc;
      c2<T> v = czero<T>();
      for (int l = i; l < r1; ++l) v = cfma<T>(v, M[i][l], S[l - r0][j]);
      out[q] = cmk<T>(-v.x, -v.y);
    }
    __syncthreads();
    q = 0;
    for (int e = t; e < TB * nc; e += NT, ++q) M[r0 + e / nc][c0 + e % nc] = out[q];
    __syncthreads();
  }
}

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
  __shared__ c2<T> Stmp[TB][NB];
  __shared__ int s_ipos[2 * IB], s_isrc[2 * IB];
  __shared__ int s_icnt;

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
#pragma unroll
    for (int jj = 0; jj < IB; ++jj) {
      if (jj >= ib) break;
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
    // ---- the inner block's row exchanges on the other panel columns, as one compact
    //      permutation (new row s_ipos[i] = old row s_isrc[i]): one gather and one
    //      scatter per column instead of a chain of dependent swaps
    if (t == 0) {
      int cnt = ib;
      for (int i = 0; i < ib; ++i) { s_ipos[i] = c0 + i; s_isrc[i] = c0 + i; }
      for (int i = 0; i < ib; ++i) {
        const int p = s_ipiv[c0 + i - k0];
        if (p == c0 + i) continue;
        int ip = -1;
        if (p < c0 + ib) ip = p - c0;
        else {
          for (int j = ib; j < cnt; ++j)
            if (s_ipos[j] == p) { ip = j; break; }
          if (ip < 0) { ip = cnt; s_ipos[cnt] = p; s_isrc[cnt] = p; ++cnt; }
        }
        const int x = s_isrc[i]; s_isrc[i] = s_isrc[ip]; s_isrc[ip] = x;
      }
      s_icnt = cnt;
    }
    __syncthreads();
    {
      const int nleft = c0 - k0, nother = nbk - ib, cnt = s_icnt;
      constexpr int GQ = (2 * IB * NB + NT - 1) / NT;
      c2<T> g[GQ];
#pragma unroll
      for (int q = 0; q < GQ; ++q) {
        const int e = t + q * NT;
        g[q] = czero<T>();
        if (e < nother * cnt) {
          const int ee = e % nother, i = e / nother;
          const int col = (ee < nleft) ? k0 + ee : c0 + ib + (ee - nleft);
          g[q] = A[(long long)s_isrc[i] * n + col];
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < GQ; ++q) {
        const int e = t + q * NT;
        if (e < nother * cnt) {
          const int ee = e % nother, i = e / nother;
          const int col = (ee < nleft) ? k0 + ee : c0 + ib + (ee - nleft);
          A[(long long)s_ipos[i] * n + col] = g[q];
        }
      }
    }
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
      // U rows of this block: unit-lower substitution with Lb, in halves of 8 rows so
      // that every register array stays statically indexed
      for (int e = t; e < nr; e += NT) {
        constexpr int H = (IB > 8) ? 8 : IB;
        c2<T> x[H], y[H];
#pragma unroll
        for (int i = 0; i < H; ++i) x[i] = (i < ib) ? A[(long long)(c0 + i) * n + cr0 + e] : czero<T>();
#pragma unroll
        for (int i = 0; i < H; ++i) y[i] = (H + i < ib && IB > H) ? A[(long long)(c0 + H + i) * n + cr0 + e] : czero<T>();
#pragma unroll
        for (int i = 1; i < H; ++i)
#pragma unroll
          for (int j = 0; j < H; ++j)
            if (j < i) x[i] = cfms<T>(x[i], Lb[i][j], x[j]);
        if (IB > H) {
#pragma unroll
          for (int i = 0; i < H; ++i)
#pragma unroll
            for (int j = 0; j < H; ++j) y[i] = cfms<T>(y[i], Lb[(H + i) & (IB - 1)][j], x[j]);
#pragma unroll
          for (int i = 1; i < H; ++i)
#pragma unroll
            for (int j = 0; j < H; ++j)
              if (j < i) y[i] = cfms<T>(y[i], Lb[(H + i) & (IB - 1)][(H + j) & (IB - 1)], y[j]);
        }
#pragma unroll
        for (int i = 0; i < H; ++i)
          if (i < ib) { A[(long long)(c0 + i) * n + cr0 + e] = x[i]; Ub[i][e] = x[i]; }
#pragma unroll
        for (int i = 0; i < H; ++i)
          if (IB > H && H + i < ib) {
            A[(long long)(c0 + H + i) * n + cr0 + e] = y[i];
            Ub[(H + i) & (IB - 1)][e] = y[i];
          }
      }
      __syncthreads();
      // chunks of 8 columns; all of a thread's rows load together before any store
      for (int e0 = 0; e0 < nr; e0 += 8) {
        c2<T> acc[RPT][8];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = k0 + t + q * NT;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            acc[q][u] = (r >= cr0 && r < n && e0 + u < nr) ? A[(long long)r * n + cr0 + e0 + u] : czero<T>();
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q)
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int i = 0; i < IB; ++i)
              if (i < ib) acc[q][u] = cfms<T>(acc[q][u], a[q][i], Ub[i][(e0 + u) & (NB - 1)]);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = k0 + t + q * NT;
          if (r >= cr0 && r < n)
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (e0 + u < nr) A[(long long)r * n + cr0 + e0 + u] = acc[q][u];
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

  // ---- inverses of the diagonal blocks L11 (unit lower) and U11 (upper)
  c2<T>* Li = Linv + (long long)b * inv_stride + (long long)step * NB * NB;
  c2<T>* Ui = Uinv + (long long)b * inv_stride + (long long)step * NB * NB;
  for (int e = t; e < nbk * nbk; e += NT) {
    const int i = e / nbk, j = e % nbk;
    Mtri[i][j] = A[(long long)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  inv_unit_lower<T, NB, NT>(Mtri, Stmp, nbk);
  for (int e = t; e < NB * NB; e += NT) {
    const int i = e / NB, j = e % NB;
    c2<T> v = czero<T>();
    if (i < nbk && j < nbk) v = (i == j) ? cmk<T>(T(1), T(0)) : (j < i ? Mtri[i][j] : czero<T>());
    Li[e] = v;
  }
  __syncthreads();
  for (int e = t; e < nbk * nbk; e += NT) {
    const int i = e / nbk, j = e % nbk;
    Mtri[i][j] = A[(long long)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  inv_upper<T, NB, NT>(Mtri, Stmp, nbk);
  for (int e = t; e < NB * NB; e += NT) {
    const int i = e / NB, j = e % NB;
    c2<T> v = czero<T>();
    if (i < nbk && j < nbk && j >= i) v = Mtri[i][j];
    Ui[e] = v;
  }
}


// ----------------------------------------------------------------------------- tournament panel
// Panel factorisation with tournament pivoting (communication-avoiding LU: partial
// pivoting inside row chunks, winners merged pairwise, the final 64 rows factored).
// The pivot rows differ from plain partial pivoting; the result is still P A = L U
// with |multipliers| bounded in practice, and every pass over the panel is parallel.
//
// gepp_chunk: partial pivoting on up to R (128 or 256) rows x nbk <= 64 panel columns
// held in registers: 4R threads, thread t owns chunk row i = t/4 and the 16 columns
// 16*(t&3) .. +15, so the four threads of a row form a quad of lanes.  Rows are never
// moved; a row is marked when chosen.  Produces the pivot rows in order (win) and
// leaves every row factored in place: a chosen row holds its multipliers left of its
// pivot column and its U row from there on, a row never chosen holds its multipliers
// (its row of L21).  Every value read is an original panel value.
//
// One workgroup barrier per column: each wave reduces its best row for column j to a
// packed key (magnitude bits | row), and the lanes holding that row publish it (and
// the reciprocal of its column-j entry) to LDS; after the barrier every thread picks
// the best of the wave keys and reads the pivot row from that wave's slot.  Slots are
// double-buffered by column parity.
//
// Key: the IEEE bits of |Re| + |Im| (bits of a non-negative value order like unsigned
// integers) with the low bits replaced by (2R - 1 - i), so that equal keys go to the
// lowest row and 0 means no candidate.  32-bit keys keep 12 (double) / 15 (float)
// mantissa bits: the pivot is the largest row up to a relative 2^-12 (the tournament's
// selection passes).  64-bit keys keep 43 (double) / all 23 (float) mantissa bits: the
// choice of partial pivoting, up to ties within 2^-43 relative.
constexpr int GEPP_Q = 4, GEPP_H = 64 / GEPP_Q;

template <typename T>
struct Gepp {
  c2<T> a[GEPP_H];
  int row;       // global row id of this thread's candidate row (-1: none)
  bool chosen;
};

template <typename T, int R, typename K>
struct GeppShared {
  static constexpr int NW = 4 * R / 64;
  c2<T> rowbuf[2][NW][64];
  c2<T> rinv[2][NW];               // 1 / (the wave candidate's column-j entry)
  K keys[2][NW];
  int win[64];
  int singular;
};

template <int R> __device__ inline unsigned gepp_key32(double m, int i) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(m) >> 32);
  return (hi & ~(unsigned)(2 * R - 1)) | (unsigned)(2 * R - 1 - i);
}
template <int R> __device__ inline unsigned gepp_key32(float m, int i) {
  return ((unsigned)__float_as_uint(m) & ~(unsigned)(2 * R - 1)) | (unsigned)(2 * R - 1 - i);
}
template <int R> __device__ inline unsigned long long gepp_key64(double m, int i) {
  return ((unsigned long long)__double_as_longlong(m) & ~(unsigned long long)(2 * R - 1)) |
         (unsigned long long)(2 * R - 1 - i);
}
template <int R> __device__ inline unsigned long long gepp_key64(float m, int i) {
  return ((unsigned long long)__float_as_uint(m) << 16) | (unsigned long long)(2 * R - 1 - i);
}
template <int R, typename K, typename T> __device__ inline K gepp_key(T m, int i) {
  if constexpr (sizeof(K) == 4) return gepp_key32<R>(m, i);
  else return gepp_key64<R>(m, i);
}

// DPP move of lane data; ctrl_sel picks a constant control: quad xor 1, quad xor 2,
// half-row mirror, row mirror
__device__ inline unsigned dpp_mov(unsigned v, int ctrl_sel) {
  switch (ctrl_sel) {
    case 0: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);
    case 1: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);
    case 2: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);
    default: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false);
  }
}
__device__ inline unsigned long long dpp_mov(unsigned long long v, int ctrl_sel) {
  const unsigned lo = dpp_mov((unsigned)v, ctrl_sel), hi = dpp_mov((unsigned)(v >> 32), ctrl_sel);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ inline unsigned readlane_k(unsigned v, int l) { return (unsigned)__builtin_amdgcn_readlane((int)v, l); }
__device__ inline unsigned long long readlane_k(unsigned long long v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// maximum over the 64 lanes, returned to every lane (all lanes must be active)
template <typename K>
__device__ inline K wave_max_key(K v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const K o = dpp_mov(v, c);
    v = v > o ? v : o;
  }
  const K a = readlane_k(v, 0), b = readlane_k(v, 16), c = readlane_k(v, 32), d = readlane_k(v, 48);
  const K x = a > b ? a : b, y = c > d ? c : d;
  return x > y ? x : y;
}

// value of lane `src` (0..3, uniform) of each quad, to all four lanes of the quad
__device__ inline int quad_bcast(int v, int src) {
  switch (src) {
    case 0: return __builtin_amdgcn_update_dpp(0, v, 0x00, 0xf, 0xf, false);
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0x55, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0xAA, 0xf, 0xf, false);
    default: return __builtin_amdgcn_update_dpp(0, v, 0xFF, 0xf, 0xf, false);
  }
}
__device__ inline double quad_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = quad_bcast((int)(b & 0xffffffffll), src), hi = quad_bcast((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline float quad_bcast(float v, int src) { return __int_as_float(quad_bcast(__float_as_int(v), src)); }

template <typename T, int R, typename K>
__device__ __forceinline__ void gepp_chunk(Gepp<T>& g, int nbk, GeppShared<T, R, K>& sh) {
  constexpr int H = GEPP_H, NW = GeppShared<T, R, K>::NW;
  constexpr K MASK = (K)(2 * R - 1);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int h = t & (GEPP_Q - 1), i = t / GEPP_Q;
  g.chosen = false;
  bool done = false;
  for (int jb = 0; jb < GEPP_Q && !done; ++jb) {        // column quarter, owned by lanes h == jb
#pragma clang loop unroll(full)
    for (int ju = 0; ju < H; ++ju) {                    // static register index of column j
      const int j = jb * H + ju;
      if (done || j >= nbk) continue;                   // uniform
      const int buf = j & 1;
      const bool live = g.row >= 0 && !g.chosen;
      const c2<T> ajj = g.a[ju];
      K key = 0;
      if (h == jb && live) key = gepp_key<R, K>(cabs1<T>(ajj), i);
      // the reciprocal is formed by every owner lane while the reduction runs, so
      // that no division sits between the barrier and the update
      const bool nzj = ajj.x != T(0) || ajj.y != T(0);
      const c2<T> r = nzj ? crcp<T>(ajj) : czero<T>();
      const K wk = wave_max_key<K>(key);
      if (wk != 0 && i == (int)(MASK - (wk & MASK))) {
#pragma unroll
        for (int u = 0; u < H; ++u) sh.rowbuf[buf][wave][h * H + u] = g.a[u];
        if (h == jb) sh.rinv[buf][wave] = r;
      }
      if (lane == 0) sh.keys[buf][wave] = wk;
      __syncthreads();
      // the best of the wave keys, reduced once more across a wave; the winning row's
      // index names its wave (16 rows per wave)
      const K best = wave_max_key<K>(lane < NW ? sh.keys[buf][lane] : K(0));
      if (best == 0) { done = true; continue; }         // no candidate rows left (uniform)
      const int pi = (int)(MASK - (best & MASK));
      const int bw = pi / (64 / GEPP_Q);
      if ((best & ~MASK) == 0 && t == 0) sh.singular = 1;
      if (i == pi) {
        g.chosen = true;
        if (h == 0) sh.win[j] = g.row;
      }
      const c2<T>* prow = sh.rowbuf[buf][bw];
      const c2<T> rp = sh.rinv[buf][bw];
      const bool upd = g.row >= 0 && !g.chosen;
      // multiplier of this row (zero for rows not updated and for a zero pivot)
      c2<T> l = (h == jb && upd) ? cmul<T>(ajj, rp) : czero<T>();
      l.x = quad_bcast(l.x, jb);
      l.y = quad_bcast(l.y, jb);
      // rank-1 correction of the columns right of j (u > ju in the owner's quarter,
      // every column of the quarters after it); column j takes the multiplier
      if (upd) {
#pragma unroll
        for (int u = 0; u < H; ++u) {
          if (u == ju && h == jb) {
            g.a[u] = l;
          } else if ((u > ju ? h >= jb : h > jb) && h * H + u < nbk) {
            const c2<T> p = prow[h * H + u];
            g.a[u].x = fma(-l.x, p.x, fma(l.y, p.y, g.a[u].x));
            g.a[u].y = fma(-l.x, p.y, fma(-l.y, p.x, g.a[u].y));
          }
        }
      }
    }
  }
  __syncthreads();                                      // win / singular complete
}

template <typename T>
__device__ __forceinline__ void gepp_load(Gepp<T>& g, const c2<T>* A, int n, int k0, int nbk, int row) {
  const int h = threadIdx.x % GEPP_Q;
  g.row = row;
#pragma unroll
  for (int u = 0; u < GEPP_H; ++u) {
    const int c = h * GEPP_H + u;
    g.a[u] = (row >= 0 && c < nbk) ? A[(long long)row * n + k0 + c] : czero<T>();
  }
}

template <typename T, int R, typename K>
__device__ void gepp_init(GeppShared<T, R, K>& sh) {
  const int t = threadIdx.x;
  if (t < 64) sh.win[t] = -1;
  if (t == 0) sh.singular = 0;
}

// Tournament selection passes use 128-row chunks and 32-bit keys.
constexpr int TSLU_ROWS = 128, TSLU_NT = 4 * TSLU_ROWS;

// T1: grid nbatch x nch, chunk c of matrix b: rows k0 + 128c .. +127 -> 64 nominations
template <typename T>
__global__ __launch_bounds__(TSLU_NT) void tslu_local_kernel(const c2<T>* __restrict__ W, long long mstride,
                                                             int n, int k0, int nbk, int nch,
                                                             int* __restrict__ cand) {
  const int b = blockIdx.x / nch, c = blockIdx.x % nch;
  const c2<T>* A = W + (long long)b * mstride;
  __shared__ GeppShared<T, TSLU_ROWS, unsigned> sh;
  const int t = threadIdx.x;
  gepp_init(sh);
  Gepp<T> g;
  const int r = k0 + c * TSLU_ROWS + t / GEPP_Q;
  gepp_load<T>(g, A, n, k0, nbk, r < n ? r : -1);
  __syncthreads();
  gepp_chunk(g, nbk, sh);
  if (t < 64) cand[((long long)b * 64 + c) * 64 + t] = sh.win[t];
}

// T2: grid nbatch x npair, merge candidate sets 2p and 2p+1 (of nin) -> set p
template <typename T>
__global__ __launch_bounds__(TSLU_NT) void tslu_merge_kernel(const c2<T>* __restrict__ W, long long mstride,
                                                             int n, int k0, int nbk, int nin,
                                                             const int* __restrict__ cin, int* __restrict__ cout) {
  const int npair = (nin + 1) / 2;
  const int b = blockIdx.x / npair, p = blockIdx.x % npair;
  const c2<T>* A = W + (long long)b * mstride;
  __shared__ GeppShared<T, TSLU_ROWS, unsigned> sh;
  const int t = threadIdx.x;
  gepp_init(sh);
  const int i = t / GEPP_Q;
  const int set = 2 * p + (i >> 6);
  const int row = (set < nin) ? cin[((long long)b * 64 + set) * 64 + (i & 63)] : -1;
  Gepp<T> g;
  gepp_load<T>(g, A, n, k0, nbk, row);
  __syncthreads();
  gepp_chunk(g, nbk, sh);
  if (t < 64) cout[((long long)b * 64 + p) * 64 + t] = sh.win[t];
}

// Final panel pass, one workgroup of 4R threads per matrix, partial pivoting with
// 64-bit keys on
//   DIRECT:  every row of the panel (n - k0 <= R), or
//   !DIRECT: the union of <= 2 tournament candidate sets (R = 128),
// then
//   - the step's row exchange as a compact permutation (top rows k0+k <- winner k;
//     the displaced top rows fill the positions the winners vacate below kend),
//   - the winners' factored rows (L11 \ U11) written to the top rows,
//   - DIRECT: every other row's multipliers (its row of L21) written at its new
//     position; !DIRECT: the displaced top rows' panel values saved for the L21 pass,
//   - inv(L11) and inv(U11).
template <typename T, int NB, int R, bool DIRECT>
__global__ __launch_bounds__(4 * R) void tslu_root_kernel(c2<T>* __restrict__ W, long long mstride, int n, int k0,
                                                          int nbk, int step, int nin, const int* __restrict__ cin,
                                                          int* __restrict__ perm, long long perm_stride,
                                                          c2<T>* __restrict__ saved, c2<T>* __restrict__ Linv,
                                                          c2<T>* __restrict__ Uinv, long long inv_stride,
                                                          int* __restrict__ info) {
  constexpr int NT = 4 * R;
  using K = unsigned long long;
  const int b = blockIdx.x;
  c2<T>* A = W + (long long)b * mstride;
  // the GEPP state and the triangle workspace are used one after the other
  union RootShared {
    GeppShared<T, R, K> g;
    struct { c2<T> M[NB][NB + 1]; c2<T> S[TB][NB]; } tri;
  };
  __shared__ RootShared shu;
  __shared__ int win[64];
  __shared__ int s_pos[2 * NB], s_src[2 * NB], s_cnt, s_sing;
  __shared__ int s_dest[NB];         // DIRECT: new position of each top row not chosen
  __shared__ unsigned char s_top[NB];
  auto Mtri = shu.tri.M;
  auto Stmp = shu.tri.S;
  const int t = threadIdx.x;
  gepp_init(shu.g);
  const int i = t / GEPP_Q;
  int row;
  if (DIRECT) {
    row = (k0 + i < n) ? k0 + i : -1;
  } else {
    const int set = i >> 6;
    row = (set < nin) ? cin[((long long)b * 64 + set) * 64 + (i & 63)] : -1;
  }
  Gepp<T> g;
  gepp_load<T>(g, A, n, k0, nbk, row);
  __syncthreads();
  gepp_chunk(g, nbk, shu.g);
  if (t < 64) win[t] = shu.g.win[t];
  if (t == 0) s_sing = shu.g.singular;
  __syncthreads();
  // ---- compact permutation
  const int kend = k0 + nbk;
  if (t == 0) {
    for (int k = 0; k < nbk; ++k) { s_top[k] = 0; s_dest[k] = -1; }
    for (int k = 0; k < nbk; ++k)
      if (win[k] >= k0 && win[k] < kend) s_top[win[k] - k0] = 1;
    int cnt = nbk, d = 0;
    for (int k = 0; k < nbk; ++k) { s_pos[k] = k0 + k; s_src[k] = win[k]; }
    for (int k = 0; k < nbk; ++k) {
      if (win[k] >= kend) {
        while (d < nbk - 1 && s_top[d]) ++d;   // next top row that was not chosen
        s_pos[cnt] = win[k];
        s_src[cnt] = k0 + d;
        s_dest[d] = win[k];
        ++d;
        ++cnt;
      }
    }
    s_cnt = cnt;
    if (s_sing && info[b] == 0) info[b] = k0 + 1;
  }
  __syncthreads();
  {
    int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NB);
    for (int e = t; e < 2 * NB; e += NT) {
      P[1 + e] = (e < s_cnt) ? s_pos[e] : -1;
      P[1 + 2 * NB + e] = (e < s_cnt) ? s_src[e] : -1;
    }
    if (t == 0) P[0] = s_cnt;
  }
  if (!DIRECT) {
    // ---- save the displaced top rows (original panel values), slot e - nbk
    c2<T>* sv = saved + (long long)b * NB * NB;
    for (int e = t; e < (s_cnt - nbk) * nbk; e += NT) {
      const int q = e / nbk, c = e % nbk;
      sv[q * NB + c] = A[(long long)s_src[nbk + q] * n + k0 + c];
    }
    __syncthreads();
  }
  // ---- factored rows to their positions; every value comes from the registers
  int k = -1;
  if (g.chosen)
    for (int q = 0; q < nbk; ++q)
      if (win[q] == g.row) k = q;
  const int h = t % GEPP_Q;
  int dest = -1;
  if (k >= 0) dest = k0 + k;
  else if (DIRECT && g.row >= 0) dest = (g.row < kend) ? s_dest[g.row - k0] : g.row;
  if (dest >= 0) {
#pragma unroll
    for (int u = 0; u < GEPP_H; ++u) {
      const int c = h * GEPP_H + u;
      if (c < nbk) A[(long long)dest * n + k0 + c] = g.a[u];
    }
  }
  auto fill = [&]() {
    if (k >= 0) {
#pragma unroll
      for (int u = 0; u < GEPP_H; ++u) {
        const int c = h * GEPP_H + u;
        if (c < nbk) Mtri[k][c] = g.a[u];
      }
    }
  };
  fill();
  __syncthreads();
  c2<T>* Li = Linv + (long long)b * inv_stride + (long long)step * NB * NB;
  c2<T>* Ui = Uinv + (long long)b * inv_stride + (long long)step * NB * NB;
  inv_unit_lower<T, NB, NT>(Mtri, Stmp, nbk);
  for (int e = t; e < NB * NB; e += NT) {
    const int r = e / NB, c = e % NB;
    c2<T> v = czero<T>();
    if (r < nbk && c < nbk) v = (r == c) ? cmk<T>(T(1), T(0)) : (c < r ? Mtri[r][c] : czero<T>());
    Li[e] = v;
  }
  __syncthreads();
  fill();
  __syncthreads();
  inv_upper<T, NB, NT>(Mtri, Stmp, nbk);
  for (int e = t; e < NB * NB; e += NT) {
    const int r = e / NB, c = e % NB;
    Ui[e] = (r < nbk && c < nbk && c >= r) ? Mtri[r][c] : czero<T>();
  }
}

// ----------------------------------------------------------------------------- recursive panel
// Panels of more than 128 rows under partial pivoting, as leaves of W columns.  A
// leaf holds rows r0 .. n-1 of its W columns in registers (RPT rows per thread, NT
// threads), runs partial pivoting on them (one barrier per column; 64-bit keys hold
// the magnitude's top bits and the row), writes the factored columns at their
// exchanged rows, applies its exchange to the panel's other 64 - W columns and forms
// the W rows of U to its right inside the panel.  A rank-W update of the rows below
// follows as a launch of its own (many workgroups per matrix).  A finishing kernel
// composes the leaves' exchanges into the step's one and forms inv(L11) and inv(U11).
// Leaf shapes: panels of up to 1024 rows use 8-column leaves of 256 threads (four rows
// each; fewer waves per barrier) in pairs, in both precisions; complex64 panels of
// 1025 to 2048 rows use 16-column leaves of 1024 threads (two rows each).
constexpr int RP_NTMAX = 1024, RP_WMAX = 16;
constexpr int rp_ex(int w) { return 1 + 4 * w; }   // leaf exchange record: cnt, pos[2W], src[2W]
constexpr int RP_EXMAX = rp_ex(8) * 8;             // ints per matrix for the records of one step

__device__ inline unsigned long long rp_key(double m, int i) {
  return ((unsigned long long)__double_as_longlong(m) & ~4095ull) | (unsigned long long)(4095 - i);
}
__device__ inline unsigned long long rp_key(float m, int i) {
  return ((unsigned long long)__float_as_uint(m) << 16) | (unsigned long long)(4095 - i);
}

// PREV: the rank-W update of the previous leaf (q - 1) has not been applied to this
// leaf's columns nor to the panel's top rows right of it; the leaf applies it to its own
// rows on load and to its top rows before forming U (leaves then run in pairs with one
// rank-2W update per pair for the columns right of both).
template <typename T, int RP_W, int RP_NT, int RPT, bool PREV>
__global__ __launch_bounds__(RP_NT) void rpanel_leaf_kernel(c2<T>* __restrict__ W, long long mstride, int n,
                                                            int k0, int q, int* __restrict__ sub,
                                                            int* __restrict__ info) {
  using K = unsigned long long;
  constexpr K MASK = 4095;
  constexpr int RP_NW = RP_NT / 64, NL = 64 / RP_W, OC = 64 - RP_W, RP_EX = rp_ex(RP_W);
  const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  c2<T>* A = W + (long long)b * mstride;
  const int c0 = k0 + RP_W * q, r0 = c0;           // the leaf's first column and first row
  const int cr = c0 + RP_W, wr = k0 + 64 - cr;     // panel columns right of the leaf
  __shared__ c2<T> rowbuf[2][RP_NW][RP_W];
  __shared__ c2<T> rinv[2][RP_NW];
  __shared__ K keys[2][RP_NW];
  __shared__ int win[RP_W];
  __shared__ int s_pos[2 * RP_W], s_src[2 * RP_W], s_cnt, s_sing;
  __shared__ int s_dest[RP_W];
  __shared__ unsigned char s_top[RP_W];
  __shared__ c2<T> xbuf[2 * RP_W][OC];             // exchanged rows of the other panel columns
  __shared__ c2<T> Lqq[RP_W][RP_W + 1];
  __shared__ c2<T> Up[PREV ? RP_W : 1][RP_W];      // U of the previous leaf in this leaf's columns

  c2<T> a[RPT][RP_W];
  int row[RPT];
  bool chosen[RPT];
#pragma unroll
  for (int p = 0; p < RPT; ++p) {
    const int r = r0 + t + p * RP_NT;
    row[p] = r < n ? r : -1;
    chosen[p] = false;
#pragma unroll
    for (int u = 0; u < RP_W; ++u) a[p][u] = (r < n) ? A[(long long)r * n + c0 + u] : czero<T>();
  }
  if constexpr (PREV) {
    // a -= L[r, c0-W : c0] U[r0-W : r0, c0 : c0+W] (the previous leaf's multipliers and U rows)
    for (int e = t; e < RP_W * RP_W; e += RP_NT)
      Up[e / RP_W][e % RP_W] = A[(long long)(r0 - RP_W + e / RP_W) * n + c0 + e % RP_W];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      if (row[p] < 0) continue;
      const c2<T>* Lr = A + (long long)row[p] * n + c0 - RP_W;
#pragma unroll
      for (int kk = 0; kk < RP_W; ++kk) {
        const c2<T> l = Lr[kk];
#pragma unroll
        for (int u = 0; u < RP_W; ++u) a[p][u] = cfms<T>(a[p][u], l, Up[kk][u]);
      }
    }
  }
  if (t == 0) s_sing = 0;
  if (t < RP_W) win[t] = -1;
  __syncthreads();
#pragma clang loop unroll(full)
  for (int j = 0; j < RP_W; ++j) {
    const int buf = j & 1;
    K key = 0;
    c2<T> ajj = czero<T>();
    int bp = 0;
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      if (row[p] >= 0 && !chosen[p]) {
        const K kk = rp_key(cabs1<T>(a[p][j]), row[p] - r0);
        if (kk > key) { key = kk; ajj = a[p][j]; bp = p; }
      }
    }
    const bool nzj = ajj.x != T(0) || ajj.y != T(0);
    const c2<T> r = nzj ? crcp<T>(ajj) : czero<T>();
    const K wk = wave_max_key<K>(key);
    if (wk != 0 && key == wk) {                     // this thread holds the wave's best row
#pragma unroll
      for (int p = 0; p < RPT; ++p)
        if (p == bp) {
#pragma unroll
          for (int u = 0; u < RP_W; ++u) rowbuf[buf][wave][u] = a[p][u];
        }
      rinv[buf][wave] = r;
    }
    if (lane == 0) keys[buf][wave] = wk;
    __syncthreads();
    // the best of the wave keys, reduced once more across a wave; the winning row's
    // index names the thread (row r0 + t + p * RP_NT) and so its wave
    const K best = wave_max_key<K>(lane < RP_NW ? keys[buf][lane] : K(0));
    const int bi = (int)(MASK - (best & MASK));          // rows > 16 remain, so best != 0
    const int pi = r0 + bi;
    const int bw = (bi % RP_NT) / 64;
    if ((best & ~MASK) == 0 && t == 0) s_sing = 1;
#pragma unroll
    for (int p = 0; p < RPT; ++p)
      if (row[p] == pi) { chosen[p] = true; win[j] = pi; }
    const c2<T>* prow = rowbuf[buf][bw];
    const c2<T> rp = rinv[buf][bw];
#pragma unroll
    for (int p = 0; p < RPT; ++p) {
      if (row[p] >= 0 && !chosen[p]) {
        const c2<T> l = cmul<T>(a[p][j], rp);
        a[p][j] = l;
#pragma unroll
        for (int u = j + 1; u < RP_W; ++u) {
          const c2<T> pv = prow[u];
          a[p][u].x = fma(-l.x, pv.x, fma(l.y, pv.y, a[p][u].x));
          a[p][u].y = fma(-l.x, pv.y, fma(-l.y, pv.x, a[p][u].y));
          // keep at most four pivot-row entries in flight (the row itself fills half
          // of the registers a 1024-thread workgroup may use)
          if ((u - j) % 4 == 0) __asm__ volatile("" ::: "memory");
        }
      }
    }
  }
  __syncthreads();
  // ---- the leaf's exchange: top rows r0 + k <- winner k; the top rows not chosen fill
  // the positions the winners below vacate
  if (t == 0) {
    const int tend = r0 + RP_W;
    for (int k = 0; k < RP_W; ++k) { s_top[k] = 0; s_dest[k] = -1; }
    for (int k = 0; k < RP_W; ++k)
      if (win[k] >= r0 && win[k] < tend) s_top[win[k] - r0] = 1;
    int cnt = RP_W, d = 0;
    for (int k = 0; k < RP_W; ++k) { s_pos[k] = r0 + k; s_src[k] = win[k]; }
    for (int k = 0; k < RP_W; ++k) {
      if (win[k] >= tend) {
        while (d < RP_W - 1 && s_top[d]) ++d;
        s_pos[cnt] = win[k];
        s_src[cnt] = r0 + d;
        s_dest[d] = win[k];
        ++d;
        ++cnt;
      }
    }
    s_cnt = cnt;
    if (s_sing && info[b] == 0) info[b] = c0 + 1;
    int* R = sub + ((long long)b * NL + q) * RP_EX;
    R[0] = cnt;
    for (int i = 0; i < 2 * RP_W; ++i) {
      R[1 + i] = i < cnt ? s_pos[i] : -1;
      R[1 + 2 * RP_W + i] = i < cnt ? s_src[i] : -1;
    }
  }
  __syncthreads();
  const int cnt = s_cnt;
  // ---- factored leaf columns at their new rows; the chosen rows also into Lqq
#pragma unroll
  for (int p = 0; p < RPT; ++p) {
    if (row[p] < 0) continue;
    int dest = row[p];
    if (chosen[p]) {
      for (int k = 0; k < RP_W; ++k)
        if (win[k] == row[p]) dest = r0 + k;
#pragma unroll
      for (int u = 0; u < RP_W; ++u) Lqq[dest - r0][u] = a[p][u];
    } else if (row[p] < r0 + RP_W) {
      dest = s_dest[row[p] - r0];
    }
    if (dest >= 0) {
#pragma unroll
      for (int u = 0; u < RP_W; ++u) A[(long long)dest * n + c0 + u] = a[p][u];
    }
  }
  // ---- the exchange on the other panel columns (gathered before any is written)
  auto ocol = [&](int cc) { return cc < RP_W * q ? k0 + cc : k0 + RP_W + cc; };
  for (int e = t; e < cnt * OC; e += RP_NT) {
    const int i = e / OC, cc = e % OC;
    xbuf[i][cc] = A[(long long)s_src[i] * n + ocol(cc)];
  }
  __syncthreads();
  const int cright = RP_W * q;                      // xbuf columns >= cright lie right of the leaf
  for (int e = t; e < cnt * OC; e += RP_NT) {
    const int i = e / OC, cc = e % OC;
    if (i < RP_W && cc >= cright) continue;         // the top rows' right part: U, written below
    A[(long long)s_pos[i] * n + ocol(cc)] = xbuf[i][cc];
  }
  // ---- U rows right of the leaf: inv(L_qq) times the exchanged top rows (one column
  // per thread, forward substitution out of LDS)
  if (t < wr) {
    const int cc = cright + t;                      // each thread owns one column of xbuf
    if constexpr (PREV) {
      // the previous leaf's update on the top rows: xbuf columns cright - W .. cright - 1
      // hold their multipliers, its U rows sit at rows r0 - W .. r0 - 1
      c2<T> up[RP_W];
#pragma unroll
      for (int kk = 0; kk < RP_W; ++kk) up[kk] = A[(long long)(r0 - RP_W + kk) * n + cr + t];
      for (int i = 0; i < RP_W; ++i) {
        c2<T> v = xbuf[i][cc];
#pragma unroll
        for (int kk = 0; kk < RP_W; ++kk) v = cfms<T>(v, xbuf[i][cright - RP_W + kk], up[kk]);
        xbuf[i][cc] = v;
      }
    }
    for (int i = 0; i < RP_W; ++i) {
      c2<T> v = xbuf[i][cc];
      for (int l = 0; l < i; ++l) v = cfms<T>(v, Lqq[i][l], xbuf[l][cc]);
      xbuf[i][cc] = v;
      A[(long long)(r0 + i) * n + cr + t] = v;
    }
  }
}

// rank-16 update of the panel columns right of leaf q, rows below the leaf's top rows:
// A[r, cr:k0+64] -= L[r, c0:c0+16] U[r0:r0+16, cr:k0+64]; 64 rows per workgroup
template <typename T, int RP_W>
__global__ __launch_bounds__(256) void rpanel_update_kernel(c2<T>* __restrict__ W, long long mstride, int n, int k0,
                                                            int q, int tiles) {
  const int b = blockIdx.x / tiles, tile = blockIdx.x % tiles, t = threadIdx.x;
  c2<T>* A = W + (long long)b * mstride;
  const int c0 = k0 + RP_W * q, r0 = c0, cr = c0 + RP_W, wr = k0 + 64 - cr;
  const int R0 = r0 + RP_W + tile * 64;
  __shared__ c2<T> U[RP_W][64 - RP_W];
  __shared__ c2<T> Lt[64][RP_W + 1];
  for (int e = t; e < RP_W * wr; e += 256) U[e / wr][e % wr] = A[(long long)(r0 + e / wr) * n + cr + e % wr];
  for (int e = t; e < 64 * RP_W; e += 256) {
    const int i = e / RP_W, u = e % RP_W, r = R0 + i;
    Lt[i][u] = r < n ? A[(long long)r * n + c0 + u] : czero<T>();
  }
  __syncthreads();
  for (int e = t; e < 64 * wr; e += 256) {
    const int i = e / wr, c = e % wr, r = R0 + i;
    if (r >= n) continue;
    c2<T> v = A[(long long)r * n + cr + c];
#pragma unroll
    for (int u = 0; u < RP_W; ++u) v = cfms<T>(v, Lt[i][u], U[u][c]);
    A[(long long)r * n + cr + c] = v;
  }
}

// the step's exchange (the leaf exchanges composed, top rows first) and the inverses
// of the factored 64 x 64 diagonal block.  The leaves' exchange records are staged in
// LDS before one thread composes the step's record from them; the row map of that
// phase shares its LDS with the diagonal block of the next (at most RP_ROWS rows: the
// launcher sends only panels that fit the leaves), so two workgroups fit on a CU.
constexpr int RP_ROWS = 2 * RP_NTMAX;
template <typename T, int NB, int RP_W>
__global__ __launch_bounds__(256) void rpanel_finish_kernel(const c2<T>* __restrict__ W, long long mstride, int n,
                                                            int k0, int step, const int* __restrict__ sub,
                                                            int* __restrict__ perm, long long perm_stride,
                                                            c2<T>* __restrict__ Linv, c2<T>* __restrict__ Uinv,
                                                            long long inv_stride) {
  constexpr int NL = NB / RP_W, RP_EX = rp_ex(RP_W);
  constexpr size_t TRI_BYTES = sizeof(c2<T>) * NB * (NB + 1), MAP_BYTES = (sizeof(int) + 1) * RP_ROWS;
  const int b = blockIdx.x, t = threadIdx.x;
  const c2<T>* A = W + (long long)b * mstride;
  __shared__ __align__(16) unsigned char shared_buf[TRI_BYTES > MAP_BYTES ? TRI_BYTES : MAP_BYTES];
  __shared__ c2<T> Stmp[TB][NB];
  __shared__ int rec[NL * RP_EX];
  __shared__ int nv[2 * RP_W];
  auto Mtri = reinterpret_cast<c2<T> (*)[NB + 1]>(shared_buf);
  // srcmap[r - k0] = original row now at position r (rows k0 .. n-1)
  int* srcmap = reinterpret_cast<int*>(shared_buf);
  unsigned char* emitted = shared_buf + sizeof(int) * RP_ROWS;
  for (int i = t; i < n - k0; i += 256) { srcmap[i] = k0 + i; emitted[i] = 0; }
  for (int e = t; e < NL * RP_EX; e += 256) rec[e] = sub[(long long)b * NL * RP_EX + e];
  __syncthreads();
  for (int q = 0; q < NL; ++q) {
    const int* R = rec + q * RP_EX;
    const int cnt = R[0];
    if (t < cnt) nv[t] = srcmap[R[1 + 2 * RP_W + t] - k0];   // sources before this leaf
    __syncthreads();
    if (t < cnt) srcmap[R[1 + t] - k0] = nv[t];
    __syncthreads();
  }
  if (t == 0) {
    // record: the top rows k0 .. k0+63 in order, then every other position that moved
    int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NB);
    int cnt = 0;
    for (int k = 0; k < NB; ++k) { P[1 + cnt] = k0 + k; P[1 + 2 * NB + cnt] = srcmap[k]; ++cnt; }
    for (int q = 0; q < NL; ++q) {
      const int* R = rec + q * RP_EX;
      for (int i = 0; i < R[0]; ++i) {
        const int pos = R[1 + i];
        if (pos >= k0 + NB && !emitted[pos - k0] && srcmap[pos - k0] != pos && cnt < 2 * NB) {
          emitted[pos - k0] = 1;
          P[1 + cnt] = pos;
          P[1 + 2 * NB + cnt] = srcmap[pos - k0];
          ++cnt;
        }
      }
    }
    for (int e = cnt; e < 2 * NB; ++e) { P[1 + e] = -1; P[1 + 2 * NB + e] = -1; }
    P[0] = cnt;
  }
  __syncthreads();                                   // the row map's LDS becomes the diagonal block
  for (int e = t; e < NB * NB; e += 256) Mtri[e / NB][e % NB] = A[(long long)(k0 + e / NB) * n + k0 + e % NB];
  __syncthreads();
  c2<T>* Li = Linv + (long long)b * inv_stride + (long long)step * NB * NB;
  c2<T>* Ui = Uinv + (long long)b * inv_stride + (long long)step * NB * NB;
  inv_unit_lower<T, NB, 256>(Mtri, Stmp, NB);
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    Li[e] = (r == c) ? cmk<T>(T(1), T(0)) : (c < r ? Mtri[r][c] : czero<T>());
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += 256) Mtri[e / NB][e % NB] = A[(long long)(k0 + e / NB) * n + k0 + e % NB];
  __syncthreads();
  inv_upper<T, NB, 256>(Mtri, Stmp, NB);
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    Ui[e] = (c >= r) ? Mtri[r][c] : czero<T>();
  }
}

// A workgroup barrier that orders LDS accesses only: the caller first waits for what
// must be complete (s_waitcnt), and the asm's memory clobber keeps the compiler from
// moving any memory access across it.  __syncthreads() would also be a release/acquire
// fence, which waits for every load in flight, including loads meant to stay in flight
// across the barrier (and LDS loads issued by the memory units).
__device__ __forceinline__ void barrier_only() { asm volatile("s_barrier" ::: "memory"); }

// ----------------------------------------------------------------------------- matrix-core steps
// 256 threads = 4 waves; a workgroup owns a 64 x 64 tile, a wave a 32 x 32 quarter
// (2 x 2 blocks of 16 x 16, real and imaginary accumulators).  Workgroup ids are
// spread round-robin over the 8 XCDs; all tiles of one matrix are mapped to one XCD
// so the panels L21 / U12 it re-reads stay in that XCD's L2.
// GEMM_PANEL (tournament panel): rows below the diagonal block, L21 = A21 inv(U11),
// A21 read from the row's source under the step's row exchange.
// Delayed updates: panels are taken in pairs (s, s+1).  After panel s and its U12,
// GEMM_UPDATE with one column tile makes panel s+1 current; after panel s+1,
//   GEMM_PREUPD    the top rows of block s+1 under its exchange with step s's update
//                  applied, C = A[src] - L_s[src] U_s (and the exchange's displaced rows
//                  moved unchanged),
//   GEMM_TRSM_ID   U12 of block s+1 = inv(L11) C in place,
//   GEMM_UPDATE2   the trailing matrix once for both steps, K = 128:
//                  C -= [L_s[src'] | L_{s+1}] [U_s; U_{s+1}], src' the row a position
//                  holds after step s+1's exchange.
// The trailing matrix is then read and written once per two panels.
enum { GEMM_UPDATE = 0, GEMM_TRSM = 1, GEMM_PANEL = 2, GEMM_PREUPD = 3, GEMM_TRSM_ID = 4, GEMM_UPDATE2 = 5 };

// three workgroups per CU, except the modes that keep a panel's displaced rows in
// registers (two: three would spill them)
template <int MODE>
constexpr int gemm_min_blocks() { return (MODE == GEMM_TRSM || MODE == GEMM_PREUPD) ? 2 : 3; }

template <typename T, int MODE>
__global__ __launch_bounds__(256, gemm_min_blocks<MODE>()) void lu_gemm_kernel(c2<T>* __restrict__ W, long long mstride, int n, int k0,
                                                      int nbk, int step, int nbatch, int tiles_r, int tiles_c,
                                                      const int* __restrict__ perm, long long perm_stride,
                                                      const c2<T>* __restrict__ Linv, long long inv_stride,
                                                      const c2<T>* __restrict__ saved = nullptr) {
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
  const int k0p = k0 - NBMAX;                       // paired modes: the previous block
  constexpr bool TOP = MODE == GEMM_TRSM || MODE == GEMM_TRSM_ID || MODE == GEMM_PREUPD;
  constexpr bool SUB = MODE == GEMM_UPDATE || MODE == GEMM_UPDATE2 || MODE == GEMM_PREUPD;   // C - A B
  const int R0 = (TOP ? k0 : kend) + tr * 64;
  const int C0 = (MODE == GEMM_PANEL ? k0 : kend) + tcn * 64;
  const int rlim = TOP ? kend : n;
  const int clim = (MODE == GEMM_PANEL) ? kend : n;
  const int ktot = MODE == GEMM_PREUPD ? NBMAX : (MODE == GEMM_UPDATE2 ? NBMAX + nbk : nbk);
  const int rb = R0 + (wave >> 1) * 32, cb = C0 + (wave & 1) * 32;
  const int l16 = lane & 15, kq = lane >> 4;

  __shared__ int s_src[2 * NBMAX], s_pos[2 * NBMAX];
  __shared__ int s_cnt;
  const c2<T>* Li = nullptr;
  if (MODE == GEMM_TRSM || MODE == GEMM_PREUPD) {
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NBMAX);
    if (t == 0) s_cnt = P[0];
    for (int i = t; i < 2 * NBMAX; i += 256) { s_pos[i] = P[1 + i]; s_src[i] = P[1 + 2 * NBMAX + i]; }
    __syncthreads();
  }
  if (MODE == GEMM_TRSM || MODE == GEMM_TRSM_ID)
    Li = Linv + (long long)b * inv_stride + (long long)step * NBMAX * NBMAX;
  // GEMM_UPDATE2: s_from[i] = the row whose step-s multipliers position R0 + i uses
  __shared__ int s_from[64];
  if (MODE == GEMM_UPDATE2) {
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NBMAX);
    if (t < 64) s_from[t] = R0 + t;
    __syncthreads();
    const int cnt = P[0];
    if (t < cnt - nbk) {
      const int pos = P[1 + nbk + t];
      if (pos >= R0 && pos < R0 + 64) s_from[pos - R0] = P[1 + 2 * NBMAX + nbk + t];
    }
    __syncthreads();
  }
  // GEMM_PANEL: Linv carries inv(U11); s_slot[i] = saved-row slot of tile row i, or -1
  __shared__ int s_slot[64];
  const c2<T>* sv = nullptr;
  if (MODE == GEMM_PANEL) {
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NBMAX);
    if (t < 64) s_slot[t] = -1;
    __syncthreads();
    const int cnt = P[0];
    if (t < cnt - nbk) {
      const int pos = P[1 + nbk + t];
      if (pos >= R0 && pos < R0 + 64) s_slot[pos - R0] = t;
    }
    __syncthreads();
    Li = Linv + (long long)b * inv_stride + (long long)step * NBMAX * NBMAX;
    sv = saved + (long long)b * NBMAX * NBMAX;
  }

  // accumulators start from C (update: C - A B) or zero (TRSM: A B); the C loads are in
  // flight together with the first operand chunks
  // The complex128 UPDATE forms its complex products by three real products per
  // block (Gauss / 3M): with the negated operand a' = -a and b,
  //   A1 += a'.x b.x,  A2 += (-a'.y) b.y,  A3 += (a'.x + a'.y)(b.x + b.y),
  // starting from A1 = Re C, A2 = 0, A3 = Im C + Re C; at the end re = A1 + A2 and
  // im = A3 - A1 + A2.  Everything else uses four real products into (c1, c3) =
  // (re, im): in the other modes a third accumulator would cost occupancy, and in
  // complex64 the larger rounding error of 3M more than doubled the nodes whose
  // refinement fails (delay workload: 230 instead of 96 of 49152).
  constexpr bool G3 = (MODE == GEMM_UPDATE || MODE == GEMM_UPDATE2) && sizeof(T) == 8;
  acc4<T> c1[2][2], c2a[2][2], c3[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      c1[bi][bj] = acc_zero<T>();
      c2a[bi][bj] = acc_zero<T>();
      c3[bi][bj] = acc_zero<T>();
      if (SUB) {
        const int col = cb + bj * 16 + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb + bi * 16 + acc_row<T>(lane, r);
          if (row < rlim && col < n) {
            const int srow = MODE == GEMM_PREUPD ? s_src[row - k0] : row;
            const c2<T> v = A[(long long)srow * n + col];
            c1[bi][bj][r] = v.x;
            c3[bi][bj][r] = G3 ? v.y + v.x : v.y;
          }
        }
      }
    }

  // displaced rows of the row exchange (TRSM mode): old values, read before any write
  constexpr int DMAX = (NBMAX * 64) / 256;
  c2<T> dval[DMAX];
  int ndisp = 0;
  if (MODE == GEMM_TRSM || MODE == GEMM_PREUPD) {
    ndisp = s_cnt - nbk;
#pragma unroll
    for (int q = 0; q < DMAX; ++q) {
      const int e = t + q * 256;
      const int i = nbk + e / 64, col = C0 + (e & 63);
      dval[q] = (e < ndisp * 64 && col < n) ? A[(long long)s_src[i] * n + col] : czero<T>();
    }
  }

  // Operand chunks of KC columns of A (64 x KC) and rows of B (KC x 64) are loaded
  // cooperatively (EPT entries per thread each), double-buffered in LDS, one chunk
  // ahead.  complex128 takes KC = 8: 35 KB of LDS and at most 168 VGPRs leave room for
  // three workgroups per CU (3 waves per SIMD; 16-deep chunks allowed two and ran the
  // paired update at 36 instead of 48 TFLOP/s); complex64 keeps 16-deep chunks.
  constexpr int KC = sizeof(T) == 8 ? 8 : 16, AP = KC + 1;
  constexpr int EPT = KC * 64 / 256;
  __shared__ c2<T> As[2][64][AP];
  __shared__ c2<T> Bs[2][KC][64];
  const int wr = wave >> 1, wc = wave & 1;
  const int arow = t / (KC / EPT), akq = (t % (KC / EPT)) * EPT;   // A chunk: row, first k
  const int bk = t / (64 / EPT), bcq = (t % (64 / EPT)) * EPT;     // B chunk: k row, first column
  c2<T> ra[EPT], rbv[EPT];
  long long a_lo = 0, a_hi = 0;                   // GEMM_UPDATE2: A-operand row bases
  if (MODE == GEMM_UPDATE2) {
    a_lo = (long long)s_from[arow] * n + k0p;
    a_hi = (long long)(R0 + arow) * n + k0 - NBMAX;
  }
  auto load_chunk = [&](int kc) {
    const int row = R0 + arow;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int k = kc + akq + u;
      if (MODE == GEMM_UPDATE)
        ra[u] = (row < n && k < nbk) ? A[(long long)row * n + k0 + k] : czero<T>();
      else if (MODE == GEMM_TRSM || MODE == GEMM_TRSM_ID)
        ra[u] = (row < kend && k < nbk) ? Li[(row - k0) * NBMAX + k] : czero<T>();
      else if (MODE == GEMM_PREUPD)
        ra[u] = (row < kend && k < NBMAX) ? A[(long long)s_src[row - k0] * n + k0p + k] : czero<T>();
      else if (MODE == GEMM_UPDATE2)   // a chunk lies wholly in one of the two blocks
        ra[u] = (row < n && k < ktot) ? A[(kc < NBMAX ? a_lo : a_hi) + k] : czero<T>();
      else if (row < n && k < nbk)
        ra[u] = s_slot[arow] >= 0 ? sv[s_slot[arow] * NBMAX + k] : A[(long long)row * n + k0 + k];
      else
        ra[u] = czero<T>();
    }
    const int k = kc + bk;
    if (MODE == GEMM_PANEL) {
#pragma unroll
      for (int u = 0; u < EPT; ++u) rbv[u] = (k < nbk) ? Li[k * NBMAX + bcq + u] : czero<T>();
      return;
    }
    int srow = 0;
    if (k < ktot) {
      if (MODE == GEMM_TRSM) srow = s_src[k];
      else if (MODE == GEMM_PREUPD || MODE == GEMM_UPDATE2) srow = k0p + k;
      else srow = k0 + k;
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int col = C0 + bcq + u;
      rbv[u] = (k < ktot && col < n) ? A[(long long)srow * n + col] : czero<T>();
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      As[buf][arow][akq + u] = ra[u];
      Bs[buf][bk][bcq + u] = rbv[u];
    }
  };
  const int nch = (ktot + KC - 1) / KC;
  load_chunk(0);
  store_chunk(0);
  if (nch > 1) load_chunk(KC);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int k = ks * 4 + kq;
      c2<T> af[2], bf[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) af[bi] = As[buf][wr * 32 + bi * 16 + l16][k];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) bf[bj] = Bs[buf][k][wc * 32 + bj * 16 + l16];
      if (SUB) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) af[bi] = cmk<T>(-af[bi].x, -af[bi].y);   // C - A B
      }
      if (G3) {
        T as[2], bs[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          as[q] = af[q].x + af[q].y;
          bs[q] = bf[q].x + bf[q].y;
        }
        // the three products of a block are 4 apart in issue order
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) c1[bi][bj] = mfma16(af[bi].x, bf[bj].x, c1[bi][bj]);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) c2a[bi][bj] = mfma16(-af[bi].y, bf[bj].y, c2a[bi][bj]);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) c3[bi][bj] = mfma16(as[bi], bs[bj], c3[bi][bj]);
      } else {
        // real parts of A first, then imaginary parts: dependent products 8 apart
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            c1[bi][bj] = mfma16(af[bi].x, bf[bj].x, c1[bi][bj]);
            c3[bi][bj] = mfma16(af[bi].x, bf[bj].y, c3[bi][bj]);
          }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            c1[bi][bj] = mfma16(-af[bi].y, bf[bj].y, c1[bi][bj]);
            c3[bi][bj] = mfma16(af[bi].y, bf[bj].x, c3[bi][bj]);
          }
      }
    }
    if (c + 1 < nch) {
      store_chunk(buf ^ 1);                  // chunk c+1 (its readers finished at the last barrier)
      if (c + 2 < nch) load_chunk((c + 2) * KC);
    }
    __syncthreads();
  }
  if (TOP) __syncthreads();   // every wave has read its operands (and C's source rows)

#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = cb + bj * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb + bi * 16 + acc_row<T>(lane, r);
        if (row < rlim && col < clim) {
          const T a1 = c1[bi][bj][r], a3 = c3[bi][bj][r];
          if (G3) {
            const T a2 = c2a[bi][bj][r];
            A[(long long)row * n + col] = cmk<T>(a1 + a2, a3 - a1 + a2);
          } else {
            A[(long long)row * n + col] = cmk<T>(a1, a3);
          }
        }
      }
    }
  if (MODE == GEMM_TRSM || MODE == GEMM_PREUPD) {
#pragma unroll
    for (int q = 0; q < DMAX; ++q) {
      const int e = t + q * 256;
      const int i = nbk + e / 64, col = C0 + (e & 63);
      if (e < ndisp * 64 && col < n) A[(long long)s_pos[i] * n + col] = dval[q];
    }
  }
}

// the products of one operand chunk of lu_gemm_dma_kernel (its swizzled A layout)
template <typename T, int KC, int EPS, bool SUB>
__device__ __forceinline__ void upd2_compute(acc4<T> (&c1)[2][2], acc4<T> (&c2a)[2][2], acc4<T> (&c3)[2][2],
                                             const c2<T>* __restrict__ as, const c2<T>* __restrict__ bs, int wave,
                                             int l16, int kq) {
  constexpr bool G3 = SUB && sizeof(T) == 8;
#pragma unroll
  for (int ks = 0; ks < KC / 4; ++ks) {
    const int k = ks * 4 + kq;
    c2<T> af[2], bf[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int i = (wave >> 1) * 32 + bi * 16 + l16;
      const c2<T> v = as[i * KC + (((k / EPS) ^ ((i >> 1) & 7)) * EPS) + k % EPS];
      af[bi] = SUB ? cmk<T>(-v.x, -v.y) : v;     // C - A B, or A B
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) bf[bj] = bs[k * 64 + (wave & 1) * 32 + bj * 16 + l16];
    if (G3) {
      T as_[2], bs_[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        as_[q] = af[q].x + af[q].y;
        bs_[q] = bf[q].x + bf[q].y;
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) c1[bi][bj] = mfma16(af[bi].x, bf[bj].x, c1[bi][bj]);
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) c2a[bi][bj] = mfma16(-af[bi].y, bf[bj].y, c2a[bi][bj]);
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) c3[bi][bj] = mfma16(as_[bi], bs_[bj], c3[bi][bj]);
    } else {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          c1[bi][bj] = mfma16(af[bi].x, bf[bj].x, c1[bi][bj]);
          c3[bi][bj] = mfma16(af[bi].x, bf[bj].y, c3[bi][bj]);
        }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          c1[bi][bj] = mfma16(-af[bi].y, bf[bj].y, c1[bi][bj]);
          c3[bi][bj] = mfma16(af[bi].y, bf[bj].x, c3[bi][bj]);
        }
    }
  }
}

// lu_gemm_kernel's UPDATE2 (the paired trailing update), UPDATE, PREUPD, TRSM and
// TRSM_ID steps for full 64-column panels (same tiles and operands; PREUPD in complex128
// also takes 3M products; PREUPD and TRSM run at two workgroups per CU for the
// exchange's displaced rows they hold in registers, and TRSM reads its B rows through
// the exchange, each lane's rows of every chunk taken from the record once), with the
// operand chunks
// loaded by the memory units straight into LDS (global_load_lds_dwordx4: a lane's 16
// bytes land at the instruction's LDS base + 16 lane) three chunks deep, so that a
// chunk's loads are issued two chunks of products before they are read; the
// register-staged kernel waits for each chunk one chunk after issuing it.  A chunk is 64 rows x KC entries of A (8 slots of 16 bytes per row) and
// KC rows x 64 columns of B, 8 KB each.  The A slots of row i are stored XOR-swizzled
// (slot s holds entries (s ^ ((i >> 1) & 7)) EPS ..) so that the 16 rows a quarter-wave
// reads for one k fall on 16 different bank groups; B rows are read along columns and
// need none.  Rows and columns past the matrix are read at clamped addresses (they only
// feed outputs that are not stored).  The launcher sends full panels only (K = 128 for
// UPDATE2: 16 chunks in complex128, 8 in complex64; K = 64 for the others; a narrower
// last panel takes lu_gemm_kernel) and, in complex64, even orders (16-byte aligned
// rows).
template <typename T, int MODE>
__global__ __launch_bounds__(256, ((MODE == GEMM_PREUPD || MODE == GEMM_TRSM) ? 2 : 3)) void lu_gemm_dma_kernel(c2<T>* __restrict__ W, long long mstride, int n, int k0,
                                                             int nbk, int step, int nbatch, int tiles_r, int tiles_c,
                                                             const int* __restrict__ perm, long long perm_stride,
                                                             const c2<T>* __restrict__ Linv, long long inv_stride) {
  typedef __attribute__((address_space(3))) void* lds_ptr;
  static_assert(MODE == GEMM_UPDATE2 || MODE == GEMM_UPDATE || MODE == GEMM_TRSM_ID || MODE == GEMM_PREUPD ||
                    MODE == GEMM_TRSM, "mode");
  constexpr int NBMAX = 64;
  constexpr int EPS = 16 / (int)sizeof(c2<T>);     // complex entries per 16-byte slot
  constexpr int KC = 8 * EPS;                      // chunk depth: 8 (complex128), 16 (complex64)
  constexpr bool TOP = MODE == GEMM_TRSM_ID || MODE == GEMM_PREUPD || MODE == GEMM_TRSM;
  constexpr bool SUB = MODE != GEMM_TRSM_ID && MODE != GEMM_TRSM;   // C - A B (TRSM, TRSM_ID: A B)
  constexpr bool EXCH = MODE == GEMM_PREUPD || MODE == GEMM_TRSM;    // applies the step's row exchange
  constexpr bool G3 = SUB && sizeof(T) == 8;
  constexpr int NCH = (MODE == GEMM_UPDATE2 ? 2 * NBMAX : NBMAX) / KC;   // full panels only
  const int wg = blockIdx.x, xcd = wg & 7, slot = wg >> 3;
  const int ntile = tiles_r * tiles_c;
  const int b = (slot / ntile) * 8 + xcd;
  if (b >= nbatch) return;
  const int tile = slot % ntile, tr = tile / tiles_c, tcn = tile % tiles_c;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, l16 = lane & 15, kq = lane >> 4;
  c2<T>* A = W + (long long)b * mstride;
  const int kend = k0 + nbk, k0p = k0 - NBMAX;
  const int R0 = (TOP ? k0 : kend) + tr * 64, C0 = kend + tcn * 64;
  const int rlim = TOP ? kend : n;
  const int rb = R0 + (wave >> 1) * 32, cb = C0 + (wave & 1) * 32;

  // UPDATE2: s_from[i] = the row whose step-s multipliers position R0 + i uses
  // (positions past the matrix: its last row)
  __shared__ int s_from[64];
  if (MODE == GEMM_UPDATE2) {
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NBMAX);
    if (t < 64) s_from[t] = min(R0 + t, n - 1);
    __syncthreads();
    const int cnt = P[0];
    if (t < cnt - nbk) {
      const int pos = P[1 + nbk + t];
      if (pos >= R0 && pos < R0 + 64) s_from[pos - R0] = P[1 + 2 * NBMAX + nbk + t];
    }
    __syncthreads();
  }
  // PREUPD, TRSM: the step's exchange record (position, source of every moved row)
  __shared__ int s_src[EXCH ? 2 * NBMAX : 1], s_pos[EXCH ? 2 * NBMAX : 1];
  __shared__ int s_cnt;
  if (EXCH) {
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NBMAX);
    if (t == 0) s_cnt = P[0];
    for (int i = t; i < 2 * NBMAX; i += 256) { s_pos[i] = P[1 + i]; s_src[i] = P[1 + 2 * NBMAX + i]; }
    __syncthreads();
  }

  // the C tile's loads first: they complete with chunk 0's
  c2<T> cv[2][2][4];
  if (SUB) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int col = min(cb + bj * 16 + l16, n - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(rb + bi * 16 + acc_row<T>(lane, r), n - 1);
          const int srow = MODE == GEMM_PREUPD ? s_src[row - k0] : row;   // PREUPD: rows k0 .. kend-1
          cv[bi][bj][r] = A[(long long)srow * n + col];
        }
      }
  }

  // this wave's two A and two B load instructions per chunk: instruction j = 2 wave + q
  // covers A rows 8 j .. 8 j + 7 (lane: row 8 j + lane / 8, slot lane % 8) and B's
  // 1 KB row block j (complex128: row j, column lane; complex64: row 2 j + lane / 32,
  // columns 2 (lane % 32) + 0, 1).  A rows: UPDATE2 the step-s multipliers of row
  // s_from[i] for k < 64 and the step-s+1 multipliers of row R0 + i after; UPDATE the
  // step's multipliers of row R0 + i; PREUPD the previous step's multipliers of row
  // s_src[i] (the row the exchange brings to k0 + i); TRSM and TRSM_ID row i of the
  // step's inv(L11).  B rows: the U rows of the pair (UPDATE2), of the previous step
  // (PREUPD) or of the step (UPDATE, TRSM_ID); TRSM row s_src[k] for k.
  // PREUPD, TRSM: the rows the exchange displaces from the top block, read before any
  // write (they move unchanged to the positions their replacements left)
  constexpr int DMAX = EXCH ? (NBMAX * 64) / 256 : 1;
  c2<T> dval[DMAX];
  int ndisp = 0;
  if (EXCH) {
    ndisp = s_cnt - nbk;
#pragma unroll
    for (int q = 0; q < DMAX; ++q) {
      const int e = t + q * 256;
      const int i = nbk + e / 64, col = C0 + (e & 63);
      dval[q] = (e < ndisp * 64 && col < n) ? A[(long long)s_src[i] * n + col] : czero<T>();
    }
  }
  const c2<T>* a_lo[2];
  const c2<T>* a_hi[2];
  const c2<T>* b_at[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int j = 2 * wave + q, i = 8 * j + (lane >> 3);
    const int sw = ((lane & 7) ^ ((i >> 1) & 7)) * EPS;
    if (MODE == GEMM_UPDATE2) {
      a_lo[q] = A + (long long)s_from[i] * n + k0p + sw;
      a_hi[q] = A + (long long)min(R0 + i, n - 1) * n + k0 - NBMAX + sw;
    } else if (MODE == GEMM_UPDATE) {
      a_lo[q] = a_hi[q] = A + (long long)min(R0 + i, n - 1) * n + k0 + sw;
    } else if (MODE == GEMM_PREUPD) {
      a_lo[q] = a_hi[q] = A + (long long)s_src[i] * n + k0p + sw;
    } else {
      a_lo[q] = a_hi[q] = Linv + (long long)b * inv_stride + (long long)step * NBMAX * NBMAX + i * NBMAX + sw;
    }
    const int brow0 = (MODE == GEMM_UPDATE2 || MODE == GEMM_PREUPD) ? k0p : k0;
    if (MODE == GEMM_TRSM)   // the column part only: the row comes from the exchange record
      b_at[q] = A + (EPS == 1 ? min(C0 + lane, n - 1) : min(C0 + 2 * (lane & 31), n - 2));
    else if (EPS == 1)
      b_at[q] = A + (long long)(brow0 + j) * n + min(C0 + lane, n - 1);
    else
      b_at[q] = A + (long long)(brow0 + 2 * j + (lane >> 5)) * n + min(C0 + 2 * (lane & 31), n - 2);
  }
  // TRSM: B row k of the step is the row its exchange brings to k0 + k, s_src[k]; this
  // lane's rows of every chunk, read once (the pipeline's addresses then wait on no LDS)
  int bsrc[MODE == GEMM_TRSM ? NCH : 1][2];
  if (MODE == GEMM_TRSM) {
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int j = 2 * wave + q;
        bsrc[c][q] = s_src[c * KC + (EPS == 1 ? j : 2 * j + (lane >> 5))];
      }
  }
  __shared__ __align__(16) c2<T> As0[64 * KC], As1[64 * KC], As2[64 * KC];
  __shared__ __align__(16) c2<T> Bs0[KC * 64], Bs1[KC * 64], Bs2[KC * 64];
  auto issue = [&](c2<T>* as, c2<T>* bs, int c) {
    const int kc = c * KC;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int j = 2 * wave + q;
      const c2<T>* ga = (kc < NBMAX ? a_lo[q] : a_hi[q]) + kc;
      __builtin_amdgcn_global_load_lds((const void*)ga, (lds_ptr)(as + j * 64 * EPS), 16, 0, 0);
      const c2<T>* gb;
      if constexpr (MODE == GEMM_TRSM) gb = b_at[q] + (long long)bsrc[c][q] * n;
      else gb = b_at[q] + (long long)kc * n;
      __builtin_amdgcn_global_load_lds((const void*)gb, (lds_ptr)(bs + j * 64 * EPS), 16, 0, 0);
    }
  };

  // Chunk c: issue chunk c + 2 into the buffer chunk c - 1 used (free since the last
  // barrier), multiply chunk c, wait for this wave's loads of chunk c + 1 (its four
  // loads of chunk c + 2 may stay in flight) and for its LDS traffic (lgkmcnt(0): with
  // the vector-memory count alone, orders from 1600 on gave wrong sums now and then),
  // and meet the other waves, whose loads of chunk c + 1 are then complete too.  The loop is unrolled, so every buffer is a
  // distinct array at every use and the compiler's own waits never cover the loads
  // still in flight.
  issue(As0, Bs0, 0);
  issue(As1, Bs1, 1);
  __builtin_amdgcn_sched_barrier(0);    // nothing that reads C moves above
  __builtin_amdgcn_s_waitcnt(0x0074);   // vmcnt(4) lgkmcnt(0): chunk 0 and the C loads before it
  barrier_only();
  // accumulators from C (3M: A1 = Re C, A2 = 0, A3 = Im C + Re C) or zero (TRSM_ID)
  acc4<T> c1[2][2], c2a[2][2], c3[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      c1[bi][bj] = acc_zero<T>();
      c2a[bi][bj] = acc_zero<T>();
      c3[bi][bj] = acc_zero<T>();
      if (SUB) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          c1[bi][bj][r] = cv[bi][bj][r].x;
          c3[bi][bj][r] = G3 ? cv[bi][bj][r].y + cv[bi][bj][r].x : cv[bi][bj][r].y;
        }
      }
    }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    c2<T>* as = c % 3 == 0 ? As0 : (c % 3 == 1 ? As1 : As2);
    c2<T>* bs = c % 3 == 0 ? Bs0 : (c % 3 == 1 ? Bs1 : Bs2);
    c2<T>* an = c % 3 == 0 ? As2 : (c % 3 == 1 ? As0 : As1);
    c2<T>* bn = c % 3 == 0 ? Bs2 : (c % 3 == 1 ? Bs0 : Bs1);
    if (c + 2 < NCH) issue(an, bn, c + 2);
    upd2_compute<T, KC, EPS, SUB>(c1, c2a, c3, as, bs, wave, l16, kq);
    if (c + 1 < NCH) {
      if (c + 2 < NCH) __builtin_amdgcn_s_waitcnt(0x0074);   // vmcnt(4) lgkmcnt(0)
      else __builtin_amdgcn_s_waitcnt(0x0070);               // vmcnt(0) lgkmcnt(0)
      barrier_only();
    }
  }

#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = cb + bj * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb + bi * 16 + acc_row<T>(lane, r);
        if (row < rlim && col < n) {
          const T a1 = c1[bi][bj][r], a3 = c3[bi][bj][r];
          A[(long long)row * n + col] = G3 ? cmk<T>(a1 + c2a[bi][bj][r], a3 - a1 + c2a[bi][bj][r]) : cmk<T>(a1, a3);
        }
      }
    }
  // PREUPD, TRSM: every read of the exchange's rows (the C tile, the B rows, the
  // displaced rows) completed before the last barrier, so the moved rows are written now
  if (EXCH) {
#pragma unroll
    for (int q = 0; q < DMAX; ++q) {
      const int e = t + q * 256;
      const int i = nbk + e / 64, col = C0 + (e & 63);
      if (e < ndisp * 64 && col < n) A[(long long)s_pos[i] * n + col] = dval[q];
    }
  }
}

// ----------------------------------------------------------------------------- solves
// One workgroup of 256 threads per matrix; the right-hand sides X (n x m, m <= 32,
// complex128, row-major) are solved in place in the factor's arithmetic T.
// Every block product runs as a 64 x 8 JN tile (thread t owns rows 2(t/8)+{0,1} and
// columns t%8 + 8{0..JN-1}; JN = ceil(m / 8), so no column group is all padding) over
// operand chunks staged in LDS.
template <typename T, int JN>
struct SolveTile {
  static constexpr int MMAX = 32, KC = 32;
  c2<T> acc[2][JN];
  int r0, cb;
  __device__ SolveTile() {
    r0 = 2 * (threadIdx.x >> 3);
    cb = threadIdx.x & 7;
  }
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < JN; ++j) acc[i][j] = czero<T>();
  }
  // acc (+|-)= Ash[r][0:kc] * Bsh[kbase + 0:kc][c]
  template <bool SUB>
  __device__ void mma(const c2<T> (*Ash)[KC + 1], const c2<T> (*Bsh)[MMAX], int kbase, int kc) {
    for (int k = 0; k < kc; ++k) {
      const c2<T> a0 = Ash[r0][k], a1 = Ash[r0 + 1][k];
#pragma unroll
      for (int j = 0; j < JN; ++j) {
        const c2<T> bv = Bsh[kbase + k][cb + 8 * j];
        if (SUB) {
          acc[0][j] = cfms<T>(acc[0][j], a0, bv);
          acc[1][j] = cfms<T>(acc[1][j], a1, bv);
        } else {
          acc[0][j] = cfma<T>(acc[0][j], a0, bv);
          acc[1][j] = cfma<T>(acc[1][j], a1, bv);
        }
      }
    }
  }
};

template <typename T, int NB, bool TRANS, int JN>
__global__ __launch_bounds__(256) void lu_solve_kernel(const c2<T>* __restrict__ W, long long mstride, int n,
                                                       const int* __restrict__ perm, long long perm_stride,
                                                       const c2<T>* __restrict__ Linv, const c2<T>* __restrict__ Uinv,
                                                       long long inv_stride, double2* __restrict__ X,
                                                       long long xstride, int m, const int* __restrict__ active) {
  constexpr int MMAX = 32, KC = SolveTile<T, JN>::KC;
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const int t = threadIdx.x;
  const c2<T>* A = W + (long long)b * mstride;
  double2* Xb = X + (long long)b * xstride;
  const int nsteps = (n + NB - 1) / NB;
  // Ash and Bsh form one contiguous block (the row exchange uses it as a flat buffer)
  __shared__ c2<T> tiles[NB * (KC + 1) + NB * MMAX];
  c2<T> (*Ash)[KC + 1] = reinterpret_cast<c2<T>(*)[KC + 1]>(tiles);
  c2<T> (*Bsh)[MMAX] = reinterpret_cast<c2<T>(*)[MMAX]>(tiles + NB * (KC + 1));
  __shared__ int s_pos[2 * NB], s_src[2 * NB];
  __shared__ int s_cnt;
  SolveTile<T, JN> tile;

  auto load_perm = [&](int s) {
    const int* P = perm + (long long)b * perm_stride + (long long)s * (1 + 4 * NB);
    __syncthreads();
    if (t == 0) s_cnt = P[0];
    for (int i = t; i < 2 * NB; i += 256) { s_pos[i] = P[1 + i]; s_src[i] = P[1 + 2 * NB + i]; }
    __syncthreads();
  };
  // new[pos[i]] = old[src[i]] (forward) or new[src[i]] = old[pos[i]] (inverse); the old
  // rows are gathered into the LDS tiles (as one flat buffer) before any row is written
  auto permute = [&](bool inverse) {
    const int cnt = s_cnt;
    c2<T>* buf = &Ash[0][0];
    constexpr int CAP = NB * (KC + 1) + NB * MMAX;   // Ash and Bsh are contiguous
    static_assert(2 * NB * MMAX <= CAP, "permutation buffer");
    for (int e = t; e < cnt * m; e += 256) {
      const int i = e / m, c = e % m;
      buf[e] = ccast<T, double>(Xb[(long long)(inverse ? s_pos[i] : s_src[i]) * m + c]);
    }
    __syncthreads();
    for (int e = t; e < cnt * m; e += 256) {
      const int i = e / m, c = e % m;
      Xb[(long long)(inverse ? s_src[i] : s_pos[i]) * m + c] = ccast<double, T>(buf[e]);
    }
    __syncthreads();
  };
  // stage rows [r0, r0+nr) x cols [c0, c0+kc) of a row-major matrix (leading dim ld) into Ash
  auto stage_A = [&](const c2<T>* src, long long ld, int nr, int kc) {
    for (int e = t; e < NB * KC; e += 256) {
      const int i = e / KC, k = e % KC;
      Ash[i][k] = (i < nr && k < kc) ? src[(long long)i * ld + k] : czero<T>();
    }
  };
  // stage rows of X (complex128) into Bsh rows [dst0, dst0+nr)
  auto stage_X = [&](int xrow0, int nr, int dst0) {
    for (int e = t; e < nr * MMAX; e += 256) {
      const int i = e / MMAX, c = e % MMAX;
      Bsh[dst0 + i][c] = (c < m) ? ccast<T, double>(Xb[(long long)(xrow0 + i) * m + c]) : czero<T>();
    }
  };
  auto load_acc_X = [&](int xrow0, int nr) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < JN; ++j) {
        const int r = tile.r0 + i, c = tile.cb + 8 * j;
        tile.acc[i][j] = (r < nr && c < m) ? ccast<T, double>(Xb[(long long)(xrow0 + r) * m + c]) : czero<T>();
      }
  };
  auto store_acc_X = [&](int xrow0, int nr) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < JN; ++j) {
        const int r = tile.r0 + i, c = tile.cb + 8 * j;
        if (r < nr && c < m) Xb[(long long)(xrow0 + r) * m + c] = ccast<double, T>(tile.acc[i][j]);
      }
  };
  auto store_acc_B = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < JN; ++j) Bsh[tile.r0 + i][tile.cb + 8 * j] = tile.acc[i][j];
  };

  if (!TRANS) {
    // forward: exchange rows, y = inv(L11) x_top, x_rest -= L21 y
    for (int s = 0; s < nsteps; ++s) {
      const int k0 = s * NB, nbk = min(NB, n - k0), kend = k0 + nbk;
      load_perm(s);
      permute(false);
      stage_X(k0, nbk, 0);
      for (int i = nbk + t / MMAX; i < NB; i += 256 / MMAX) Bsh[i][t % MMAX] = czero<T>();
      const c2<T>* Li = Linv + (long long)b * inv_stride + (long long)s * NB * NB;
      tile.zero();
      for (int kc = 0; kc < nbk; kc += KC) {
        __syncthreads();
        stage_A(Li + kc, NB, nbk, min(KC, nbk - kc));
        __syncthreads();
        tile.template mma<false>(Ash, Bsh, kc, min(KC, nbk - kc));
      }
      __syncthreads();
      store_acc_B();                       // y for the trailing rows
      store_acc_X(k0, nbk);
      __syncthreads();
      // rest rows in blocks of 64, operand chunks of 64 x KC; the next chunk is loaded
      // into registers while the current one is multiplied out of LDS
      {
        const int nkc = (nbk + KC - 1) / KC;
        const int nrb = (n - kend + NB - 1) / NB;
        const int nch = nrb * nkc;
        c2<T> pre[NB * KC / 256];
        auto fetch = [&](int c) {
          const int r = kend + (c / nkc) * NB, kc = (c % nkc) * KC;
          const int nr = min(NB, n - r), kk = min(KC, nbk - kc);
#pragma unroll
          for (int q = 0; q < NB * KC / 256; ++q) {
            const int e = t + q * 256, i = e / KC, k = e % KC;
            pre[q] = (i < nr && k < kk) ? A[(long long)(r + i) * n + k0 + kc + k] : czero<T>();
          }
        };
        if (nch > 0) fetch(0);
        for (int c = 0; c < nch; ++c) {
          const int r = kend + (c / nkc) * NB, kc = (c % nkc) * KC;
          const int nr = min(NB, n - r), kk = min(KC, nbk - kc);
          if (kc == 0) load_acc_X(r, nr);
          __syncthreads();
#pragma unroll
          for (int q = 0; q < NB * KC / 256; ++q) {
            const int e = t + q * 256;
            Ash[e / KC][e % KC] = pre[q];
          }
          if (c + 1 < nch) fetch(c + 1);
          __syncthreads();
          tile.template mma<true>(Ash, Bsh, kc, kk);
          if (kc + KC >= nbk) store_acc_X(r, nr);
        }
      }
      __syncthreads();
    }
    // backward: x_top = inv(U11) (x_top - U12 x_rest)
    for (int s = nsteps - 1; s >= 0; --s) {
      const int k0 = s * NB, nbk = min(NB, n - k0), kend = k0 + nbk;
      load_acc_X(k0, nbk);
      {
        // K chunks of U12 (64 x KC) and X (KC x m), next chunk prefetched into registers
        c2<T> pa[NB * KC / 256], pb[KC * MMAX / 256];
        auto fetch = [&](int kc) {
          const int kk = min(KC, n - kc);
#pragma unroll
          for (int q = 0; q < NB * KC / 256; ++q) {
            const int e = t + q * 256, i = e / KC, k = e % KC;
            pa[q] = (i < nbk && k < kk) ? A[(long long)(k0 + i) * n + kc + k] : czero<T>();
          }
#pragma unroll
          for (int q = 0; q < KC * MMAX / 256; ++q) {
            const int e = t + q * 256, i = e / MMAX, c = e % MMAX;
            pb[q] = (i < kk && c < m) ? ccast<T, double>(Xb[(long long)(kc + i) * m + c]) : czero<T>();
          }
        };
        if (kend < n) fetch(kend);
        for (int kc = kend; kc < n; kc += KC) {
          const int kk = min(KC, n - kc);
          __syncthreads();
#pragma unroll
          for (int q = 0; q < NB * KC / 256; ++q) {
            const int e = t + q * 256;
            Ash[e / KC][e % KC] = pa[q];
          }
#pragma unroll
          for (int q = 0; q < KC * MMAX / 256; ++q) {
            const int e = t + q * 256;
            Bsh[e / MMAX][e % MMAX] = pb[q];
          }
          if (kc + KC < n) fetch(kc + KC);
          __syncthreads();
          tile.template mma<true>(Ash, Bsh, 0, kk);
        }
      }
      __syncthreads();
      store_acc_B();                       // z
      for (int i = nbk + t / MMAX; i < NB; i += 256 / MMAX) Bsh[i][t % MMAX] = czero<T>();
      const c2<T>* Ui = Uinv + (long long)b * inv_stride + (long long)s * NB * NB;
      tile.zero();
      for (int kc = 0; kc < nbk; kc += KC) {
        __syncthreads();
        stage_A(Ui + kc, NB, nbk, min(KC, nbk - kc));
        __syncthreads();
        tile.template mma<false>(Ash, Bsh, kc, min(KC, nbk - kc));
      }
      store_acc_X(k0, nbk);
      __syncthreads();
    }
  } else {
    // A = P_0^T L_0 ... P_{S-1}^T L_{S-1} U  =>  A^H x = b:  w = U^{-H} b, then for
    // s = S-1..0: w_blk = inv(L11)^H (w_blk - L21^H w_rest), w = P_s^T w.  The
    // operands are staged conjugate-transposed into the same LDS tiles.
    auto stage_AH = [&](const c2<T>* src, long long ld, int nr, int kc) {
      // Ash[i][k] = conj(src[k * ld + i]) for i < nr, k < kc
      for (int e = t; e < NB * KC; e += 256) {
        const int k = e / NB, i = e % NB;
        const c2<T> v = (i < nr && k < kc) ? src[(long long)k * ld + i] : czero<T>();
        Ash[i][k] = cmk<T>(v.x, -v.y);
      }
    };
    for (int s = 0; s < nsteps; ++s) {   // U^H is lower triangular: forward over steps
      const int k0 = s * NB, nbk = min(NB, n - k0);
      // z_blk = b_blk - sum_{j < k0} U[j, blk]^H w_j
      load_acc_X(k0, nbk);
      for (int kc = 0; kc < k0; kc += KC) {
        const int kk = min(KC, k0 - kc);
        __syncthreads();
        stage_AH(A + (long long)kc * n + k0, n, nbk, kk);
        stage_X(kc, kk, 0);
        __syncthreads();
        tile.template mma<true>(Ash, Bsh, 0, kk);
      }
      __syncthreads();
      store_acc_B();
      for (int i = nbk + t / MMAX; i < NB; i += 256 / MMAX) Bsh[i][t % MMAX] = czero<T>();
      const c2<T>* Ui = Uinv + (long long)b * inv_stride + (long long)s * NB * NB;
      tile.zero();
      for (int kc = 0; kc < nbk; kc += KC) {
        __syncthreads();
        stage_AH(Ui + (long long)kc * NB, NB, nbk, min(KC, nbk - kc));   // (inv U11)^H
        __syncthreads();
        tile.template mma<false>(Ash, Bsh, kc, min(KC, nbk - kc));
      }
      store_acc_X(k0, nbk);
      __syncthreads();
    }
    for (int s = nsteps - 1; s >= 0; --s) {
      const int k0 = s * NB, nbk = min(NB, n - k0), kend = k0 + nbk;
      // z = w_blk - L21^H w_rest
      load_acc_X(k0, nbk);
      for (int kc = kend; kc < n; kc += KC) {
        const int kk = min(KC, n - kc);
        __syncthreads();
        stage_AH(A + (long long)kc * n + k0, n, nbk, kk);
        stage_X(kc, kk, 0);
        __syncthreads();
        tile.template mma<true>(Ash, Bsh, 0, kk);
      }
      __syncthreads();
      store_acc_B();
      for (int i = nbk + t / MMAX; i < NB; i += 256 / MMAX) Bsh[i][t % MMAX] = czero<T>();
      const c2<T>* Li = Linv + (long long)b * inv_stride + (long long)s * NB * NB;
      tile.zero();
      for (int kc = 0; kc < nbk; kc += KC) {
        __syncthreads();
        stage_AH(Li + (long long)kc * NB, NB, nbk, min(KC, nbk - kc));   // (inv L11)^H
        __syncthreads();
        tile.template mma<false>(Ash, Bsh, kc, min(KC, nbk - kc));
      }
      store_acc_X(k0, nbk);
      load_perm(s);
      permute(true);
    }
  }
}

// ----------------------------------------------------------------------------- step-parallel solve
// The forward and backward substitutions of lu_solve_kernel, spread over many
// workgroups per matrix: per step one launch of one workgroup per matrix forms the
// step's block of the solution (forward: exchange the rows, then inv(L11) times the top
// rows; backward: inv(U11) times the top rows), and one launch over 64-row tiles
// subtracts the step's block column times that block from the rows below (forward) or
// above (backward).  Same arithmetic as lu_solve_kernel (products in T, X in
// complex128), many more loads in flight.
template <typename T, int NB, bool FWD, int JN>
__global__ __launch_bounds__(256) void solve_top_kernel(const c2<T>* __restrict__ W, long long mstride, int n,
                                                        int step, const int* __restrict__ perm,
                                                        long long perm_stride, const c2<T>* __restrict__ Inv,
                                                        long long inv_stride, double2* __restrict__ X,
                                                        long long xstride, int m, const int* __restrict__ active) {
  constexpr int MMAX = SolveTile<T, JN>::MMAX, KC = SolveTile<T, JN>::KC;
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const int t = threadIdx.x;
  double2* Xb = X + (long long)b * xstride;
  const int k0 = step * NB, nbk = min(NB, n - k0);
  __shared__ c2<T> Ash[NB][KC + 1];
  __shared__ c2<T> Bsh[NB][MMAX];
  __shared__ int s_pos[2 * NB], s_src[2 * NB], s_cnt;
  // rows of the top block (after the exchange) into Bsh; displaced rows into registers
  constexpr int DV = NB * MMAX / 256;
  double2 dv[DV];
  int cnt = nbk;
  if (FWD) {
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NB);
    if (t == 0) s_cnt = P[0];
    for (int i = t; i < 2 * NB; i += 256) { s_pos[i] = P[1 + i]; s_src[i] = P[1 + 2 * NB + i]; }
    __syncthreads();
    cnt = s_cnt;
  }
  for (int e = t; e < NB * MMAX; e += 256) {
    const int i = e / MMAX, c = e % MMAX;
    const int r = FWD ? s_src[min(i, nbk - 1)] : k0 + i;
    Bsh[i][c] = (i < nbk && c < m) ? ccast<T, double>(Xb[(long long)r * m + c]) : czero<T>();
  }
  const int nd = cnt - nbk;
#pragma unroll
  for (int q = 0; q < DV; ++q) {
    const int e = t + q * 256, i = e / MMAX, c = e % MMAX;
    dv[q] = (FWD && i < nd && c < m) ? Xb[(long long)s_src[nbk + i] * m + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (FWD) {
#pragma unroll
    for (int q = 0; q < DV; ++q) {
      const int e = t + q * 256, i = e / MMAX, c = e % MMAX;
      if (i < nd && c < m) Xb[(long long)s_pos[nbk + i] * m + c] = dv[q];
    }
  }
  const c2<T>* Ib = Inv + (long long)b * inv_stride + (long long)step * NB * NB;
  SolveTile<T, JN> tile;
  tile.zero();
  for (int kc = 0; kc < nbk; kc += KC) {
    const int kk = min(KC, nbk - kc);
    __syncthreads();
    for (int e = t; e < NB * KC; e += 256) {
      const int i = e / KC, k = e % KC;
      Ash[i][k] = (i < nbk && k < kk) ? Ib[(long long)i * NB + kc + k] : czero<T>();
    }
    __syncthreads();
    tile.template mma<false>(Ash, Bsh, kc, kk);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const int r = tile.r0 + i, c = tile.cb + 8 * j;
      if (r < nbk && c < m) Xb[(long long)(k0 + r) * m + c] = ccast<double, T>(tile.acc[i][j]);
    }
}

// X[r, :] -= F[r, k0:k0+nbk] X[k0:k0+nbk, :] for the 64 rows of tile `tile` of the
// range [r_lo, r_hi) (forward: rows below the block, backward: rows above it)
template <typename T, int NB, int JN>
__global__ __launch_bounds__(256) void solve_rows_kernel(const c2<T>* __restrict__ W, long long mstride, int n,
                                                         int step, int r_lo, int r_hi, int tiles,
                                                         double2* __restrict__ X, long long xstride, int m,
                                                         const int* __restrict__ active) {
  constexpr int MMAX = SolveTile<T, JN>::MMAX, KC = SolveTile<T, JN>::KC;
  const int b = blockIdx.x / tiles, tl = blockIdx.x % tiles;
  if (active && !active[b]) return;
  const int t = threadIdx.x;
  const c2<T>* A = W + (long long)b * mstride;
  double2* Xb = X + (long long)b * xstride;
  const int k0 = step * NB, nbk = min(NB, n - k0);
  const int R0 = r_lo + tl * 64, nr = min(64, r_hi - R0);
  __shared__ c2<T> Ash[NB][KC + 1];
  __shared__ c2<T> Bsh[NB][MMAX];
  for (int e = t; e < NB * MMAX; e += 256) {
    const int i = e / MMAX, c = e % MMAX;
    Bsh[i][c] = (i < nbk && c < m) ? ccast<T, double>(Xb[(long long)(k0 + i) * m + c]) : czero<T>();
  }
  SolveTile<T, JN> tile;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const int r = tile.r0 + i, c = tile.cb + 8 * j;
      tile.acc[i][j] = (r < nr && c < m) ? ccast<T, double>(Xb[(long long)(R0 + r) * m + c]) : czero<T>();
    }
  for (int kc = 0; kc < nbk; kc += KC) {
    const int kk = min(KC, nbk - kc);
    __syncthreads();
    for (int e = t; e < NB * KC; e += 256) {
      const int i = e / KC, k = e % KC;
      Ash[i][k] = (i < nr && k < kk) ? A[(long long)(R0 + i) * n + k0 + kc + k] : czero<T>();
    }
    __syncthreads();
    tile.template mma<true>(Ash, Bsh, kc, kk);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const int r = tile.r0 + i, c = tile.cb + 8 * j;
      if (r < nr && c < m) Xb[(long long)(R0 + r) * m + c] = ccast<double, T>(tile.acc[i][j]);
    }
}

// solve_top_kernel for a single right-hand side: the step's row exchange (forward), then
// the block of the solution as a 64 x 64 matrix-vector product with inv(L11) (forward)
// or inv(U11) (backward), 16 lanes per row, partial sums added by lane shuffles.
template <typename T, int NB, bool FWD>
__global__ __launch_bounds__(256) void solve_top1_kernel(const c2<T>* __restrict__ W, long long mstride, int n,
                                                         int step, const int* __restrict__ perm,
                                                         long long perm_stride, const c2<T>* __restrict__ Inv,
                                                         long long inv_stride, double2* __restrict__ X,
                                                         long long xstride, const int* __restrict__ active) {
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const int t = threadIdx.x, kl = t & 15, rl = t >> 4;
  double2* Xb = X + (long long)b * xstride;
  const int k0 = step * NB, nbk = min(NB, n - k0);
  __shared__ c2<T> xs[NB];
  if (FWD) {
    // new[pos[i]] = old[src[i]], pos[i] = k0 + i for i < nbk: the new top rows go to
    // LDS, the displaced ones are written after every old value has been read
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NB);
    const int cnt = P[0];
    double2 dv = make_double2(0.0, 0.0);
    int dpos = -1;
    if (t < nbk) xs[t] = ccast<T, double>(Xb[P[1 + 2 * NB + t]]);
    else if (t < NB) xs[t] = czero<T>();
    if (t >= nbk && t < cnt) {
      dv = Xb[P[1 + 2 * NB + t]];
      dpos = P[1 + t];
    }
    __syncthreads();
    if (dpos >= 0) Xb[dpos] = dv;
  } else {
    if (t < NB) xs[t] = (t < nbk) ? ccast<T, double>(Xb[k0 + t]) : czero<T>();
    __syncthreads();
  }
  const c2<T>* Ib = Inv + (long long)b * inv_stride + (long long)step * NB * NB;
#pragma unroll
  for (int pass = 0; pass < NB / 16; ++pass) {
    const int r = pass * 16 + rl;
    c2<T> acc = czero<T>();
    if (r < nbk) {
#pragma unroll
      for (int j = 0; j < NB / 16; ++j) {
        const int k = kl + 16 * j;
        if (k < nbk) acc = cfma<T>(acc, Ib[(long long)r * NB + k], xs[k]);
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, 16);
      acc.y += __shfl_xor(acc.y, o, 16);
    }
    if (kl == 0 && r < nbk) Xb[k0 + r] = ccast<double, T>(acc);
  }
}

// solve_rows_kernel for a single right-hand side: the tile product is a matrix-vector
// product, so the factor's rows are streamed straight from global memory with no LDS
// staging and no barrier.  A workgroup owns 16 rows, 16 lanes per row read 16
// consecutive entries (one 128-byte line per row per load in complex64, two in
// complex128) and the 16 partial sums of a row are added by lane shuffles.
template <typename T, int NB>
__global__ __launch_bounds__(256) void solve_rows1_kernel(const c2<T>* __restrict__ W, long long mstride, int n,
                                                          int step, int r_lo, int r_hi, int tiles,
                                                          double2* __restrict__ X, long long xstride,
                                                          const int* __restrict__ active) {
  const int b = blockIdx.x / tiles, tl = blockIdx.x % tiles;
  if (active && !active[b]) return;
  const int t = threadIdx.x, kl = t & 15, rl = t >> 4;
  const int k0 = step * NB, nbk = min(NB, n - k0);
  const int row = r_lo + tl * 16 + rl;
  const c2<T>* A = W + (long long)b * mstride;
  double2* Xb = X + (long long)b * xstride;
  c2<T> acc = czero<T>();
  if (row < r_hi) {
    const c2<T>* Ar = A + (long long)row * n + k0;
#pragma unroll
    for (int j = 0; j < NB / 16; ++j) {
      const int k = kl + 16 * j;
      if (k < nbk) acc = cfma<T>(acc, Ar[k], ccast<T, double>(Xb[k0 + k]));
    }
  }
  // the 16 lanes of a row are consecutive: reduce within each group of 16
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    acc.x += __shfl_xor(acc.x, o, 16);
    acc.y += __shfl_xor(acc.y, o, 16);
  }
  if (kl == 0 && row < r_hi) {
    const double2 x = Xb[row];
    Xb[row] = make_double2(x.x - (double)acc.x, x.y - (double)acc.y);
  }
}

// solve_rows_kernel on the matrix cores for 9 to 32 right-hand sides.  A workgroup
// takes up to SOLVE_TPW consecutive 64-row tiles of one matrix, a wave 16 rows of each
// and all 16 JB columns (16 x 16 blocks of the 16x16x4 MFMA).  The factor goes from
// global memory straight into the A operands: for each group of 16 entries of a row a
// lane reads the 4 consecutive ones its 4 products take (the sum over k is regrouped
// to match: in product u of group g the lanes of quarter kq take k = 16 g + 4 kq + u),
// so a wave's load covers 64 contiguous bytes of each of its 16 rows.  Each group's
// registers are refilled with the same group of the next tile as soon as they are
// used, one tile ahead of the products.  The step's block of X is staged once per
// workgroup in LDS as the B operands; the tiles of a matrix share one XCD, so the block
// stays in its L2.  The products start from zero and are subtracted from the tile's
// rows of X at its end.  complex128 forms each
// complex product from three real ones (as the paired update), complex64 from four.
constexpr int SOLVE_TPW = 4;
// two workgroups per CU for complex128 (a tile of operands in flight, the tile's rows
// of X and three accumulator sets need up to 256 registers), three for complex64
template <typename T, int JB>
constexpr int solve_rowsm_min_blocks() { return sizeof(T) == 8 ? 2 : 3; }
template <typename T, int NB, int JB>
__global__ __launch_bounds__(256, (solve_rowsm_min_blocks<T, JB>())) void solve_rowsm_kernel(const c2<T>* __restrict__ W, long long mstride, int n,
                                                             int step, int r_lo, int r_hi, int tiles, int nbatch,
                                                             double2* __restrict__ X, long long xstride, int m,
                                                             const int* __restrict__ active) {
  constexpr int NC = 16 * JB, G = NB / 16;
  constexpr bool G3 = sizeof(T) == 8;
  const int wpm = (tiles + SOLVE_TPW - 1) / SOLVE_TPW;   // workgroups per matrix
  const int wg = blockIdx.x, xcd = wg & 7, slot = wg >> 3;
  const int b = (slot / wpm) * 8 + xcd, w = slot % wpm;
  if (b >= nbatch || (active && !active[b])) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, l16 = lane & 15, kq = lane >> 4;
  const int k0 = step * NB, nbk = min(NB, n - k0);
  const int tfirst = w * SOLVE_TPW, tcount = min(SOLVE_TPW, tiles - tfirst);
  const c2<T>* A = W + (long long)b * mstride;
  double2* Xb = X + (long long)b * xstride;
  // Every load below is issued unconditionally at a clamped in-range address: with no
  // branches or selects next to them the compiler can wait for each group of operands
  // alone instead of for every load in flight.
  // the step's block of X into LDS (its loads first, so that waiting for them does not
  // wait for the operands issued next)
  __shared__ c2<T> Xs[NB][NC];
  constexpr int XE = NB * NC / 256;
  double2 xs[XE];
#pragma unroll
  for (int q = 0; q < XE; ++q) {
    const int e = t + q * 256, k = e / NC, c = e % NC;
    xs[q] = Xb[(long long)(k0 + min(k, nbk - 1)) * m + min(c, m - 1)];
  }
  __builtin_amdgcn_sched_barrier(0);   // these loads stay ahead of the operands'
  // A operands of group g of tile i: row r_lo + 64 (tfirst + i) + 16 wave + l16,
  // entries 16 g + 4 kq + 0..3
  c2<T> af[G][4];
  // Out-of-range operands are read at clamped addresses and not masked: a row past the
  // range only feeds outputs that are not stored, and an entry k >= nbk (the last step
  // of an order that is not a multiple of 64) meets a zero row of the X block, being a
  // copy of the row's entry nbk - 1 (finite wherever that one is).  Past the last tile
  // (i == tcount) the last tile is read again (from L2; values unused).
  auto load_a = [&](int g, int i) {
    const int row = min(r_lo + (tfirst + min(i, tcount - 1)) * 64 + wave * 16 + l16, r_hi - 1);
    const c2<T>* Ar = A + (long long)row * n + k0;
#pragma unroll
    for (int u = 0; u < 4; ++u) af[g][u] = Ar[min(16 * g + 4 * kq + u, nbk - 1)];
  };
#pragma unroll
  for (int g = 0; g < G; ++g) load_a(g, 0);
#pragma unroll
  for (int q = 0; q < XE; ++q) {
    const int e = t + q * 256, k = e / NC, c = e % NC;
    Xs[k][c] = (k < nbk && c < m) ? ccast<T, double>(xs[q]) : czero<T>();
  }
  // the LDS writes done, then the barrier alone (the operand loads stay in flight)
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
  barrier_only();
  // the tile loop is unrolled (no loop-carried copies of the prefetched operands)
#pragma unroll
  for (int i = 0; i < SOLVE_TPW; ++i) {
    if (i >= tcount) break;
    const int R0 = r_lo + (tfirst + i) * 64 + wave * 16;
    // the tile's rows of X, loaded before the next tile's operands so that waiting for
    // them does not wait for those
    double2 xv[JB][4];
#pragma unroll
    for (int bj = 0; bj < JB; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = R0 + acc_row<T>(lane, r), col = bj * 16 + l16;
        xv[bj][r] = Xb[(long long)min(row, r_hi - 1) * m + min(col, m - 1)];
      }
    __builtin_amdgcn_sched_barrier(0);   // these loads stay ahead of the next tile's
    acc4<T> p1[JB], p2[JB], p3[JB];
#pragma unroll
    for (int bj = 0; bj < JB; ++bj) {
      p1[bj] = acc_zero<T>();
      p2[bj] = acc_zero<T>();
      p3[bj] = acc_zero<T>();
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 16 * g + 4 * kq + u;
        const c2<T> a = af[g][u];
        c2<T> bf[JB];
#pragma unroll
        for (int bj = 0; bj < JB; ++bj) bf[bj] = Xs[k][bj * 16 + l16];
        if (G3) {
          // p1 = sum a.x b.x, p2 = -sum a.y b.y, p3 = sum (a.x + a.y)(b.x + b.y)
          const T as = a.x + a.y;
#pragma unroll
          for (int bj = 0; bj < JB; ++bj) p1[bj] = mfma16(a.x, bf[bj].x, p1[bj]);
#pragma unroll
          for (int bj = 0; bj < JB; ++bj) p2[bj] = mfma16(-a.y, bf[bj].y, p2[bj]);
#pragma unroll
          for (int bj = 0; bj < JB; ++bj) p3[bj] = mfma16(as, bf[bj].x + bf[bj].y, p3[bj]);
        } else {
          // p1 = Re, p3 = Im of the product
#pragma unroll
          for (int bj = 0; bj < JB; ++bj) {
            p1[bj] = mfma16(a.x, bf[bj].x, p1[bj]);
            p3[bj] = mfma16(a.x, bf[bj].y, p3[bj]);
          }
#pragma unroll
          for (int bj = 0; bj < JB; ++bj) {
            p1[bj] = mfma16(-a.y, bf[bj].y, p1[bj]);
            p3[bj] = mfma16(a.y, bf[bj].x, p3[bj]);
          }
        }
      }
      load_a(g, i + 1);
      // keep the B-fragment reads of later groups from being hoisted here (they would
      // hold a whole tile's fragments in registers)
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int bj = 0; bj < JB; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = R0 + acc_row<T>(lane, r), col = bj * 16 + l16;
        const T re = G3 ? p1[bj][r] + p2[bj][r] : p1[bj][r];
        const T im = G3 ? p3[bj][r] - p1[bj][r] + p2[bj][r] : p3[bj][r];
        const double2 v = make_double2(xv[bj][r].x - (double)re, xv[bj][r].y - (double)im);
        if (row < r_hi && col < m) Xb[(long long)row * m + col] = v;
      }
  }
}

// solve_top_kernel on the matrix cores for 9 to 32 right-hand sides (one workgroup per
// matrix): the step's block of the solution, inv(L11) (forward, after the step's row
// exchange) or inv(U11) (backward) times the block's rows, as one 64-row tile of
// solve_rowsm_kernel's products with the inverse as the A operands.  Forward, the rows
// the exchange displaces from the block are moved unchanged; every read of X precedes
// the barrier, every write follows it.
template <typename T, int NB, bool FWD, int JB>
__global__ __launch_bounds__(256, (solve_rowsm_min_blocks<T, JB>())) void solve_topm_kernel(
    int n, int step, const int* __restrict__ perm, long long perm_stride, const c2<T>* __restrict__ Inv,
    long long inv_stride, double2* __restrict__ X, long long xstride, int m, const int* __restrict__ active) {
  constexpr int NC = 16 * JB, G = NB / 16, XE = NB * NC / 256;
  constexpr bool G3 = sizeof(T) == 8;
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, l16 = lane & 15, kq = lane >> 4;
  const int k0 = step * NB, nbk = min(NB, n - k0);
  double2* Xb = X + (long long)b * xstride;
  const c2<T>* Ib = Inv + (long long)b * inv_stride + (long long)step * NB * NB;
  __shared__ c2<T> Xs[NB][NC];
  __shared__ int s_pos[2 * NB], s_src[2 * NB], s_cnt;
  int cnt = nbk;
  if (FWD) {
    const int* P = perm + (long long)b * perm_stride + (long long)step * (1 + 4 * NB);
    if (t == 0) s_cnt = P[0];
    for (int i = t; i < 2 * NB; i += 256) { s_pos[i] = P[1 + i]; s_src[i] = P[1 + 2 * NB + i]; }
    __syncthreads();
    cnt = s_cnt;
  }
  // inverse rows 16 wave + l16 (clamped to the block: rows past it are not stored),
  // entries 16 g + 4 kq + 0..3 (clamped: entries past the block meet zero rows of Xs)
  c2<T> af[G][4];
  const c2<T>* Ar = Ib + (long long)min(wave * 16 + l16, nbk - 1) * NB;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int u = 0; u < 4; ++u) af[g][u] = Ar[min(16 * g + 4 * kq + u, nbk - 1)];
  // the block's rows (forward: the rows the exchange brings in) into LDS
#pragma unroll
  for (int q = 0; q < XE; ++q) {
    const int e = t + q * 256, k = e / NC, c = e % NC;
    const int kk = min(k, nbk - 1);
    const int r = FWD ? s_src[kk] : k0 + kk;
    const double2 v = Xb[(long long)r * m + min(c, m - 1)];
    Xs[k][c] = (k < nbk && c < m) ? ccast<T, double>(v) : czero<T>();
  }
  __syncthreads();
  // forward: the rows the exchange displaces from the block (old block rows, intact
  // until the block is written after the second barrier) move below it
  if constexpr (FWD) {
    const int nd = cnt - nbk;
    for (int e = t; e < nd * m; e += 256) {
      const int i = e / m, c = e % m;
      Xb[(long long)s_pos[nbk + i] * m + c] = Xb[(long long)s_src[nbk + i] * m + c];
    }
  }
  acc4<T> p1[JB], p2[JB], p3[JB];
#pragma unroll
  for (int bj = 0; bj < JB; ++bj) {
    p1[bj] = acc_zero<T>();
    p2[bj] = acc_zero<T>();
    p3[bj] = acc_zero<T>();
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 16 * g + 4 * kq + u;
      const c2<T> a = af[g][u];
      c2<T> bf[JB];
#pragma unroll
      for (int bj = 0; bj < JB; ++bj) bf[bj] = Xs[k][bj * 16 + l16];
      if (G3) {
        const T as = a.x + a.y;
#pragma unroll
        for (int bj = 0; bj < JB; ++bj) p1[bj] = mfma16(a.x, bf[bj].x, p1[bj]);
#pragma unroll
        for (int bj = 0; bj < JB; ++bj) p2[bj] = mfma16(-a.y, bf[bj].y, p2[bj]);
#pragma unroll
        for (int bj = 0; bj < JB; ++bj) p3[bj] = mfma16(as, bf[bj].x + bf[bj].y, p3[bj]);
      } else {
#pragma unroll
        for (int bj = 0; bj < JB; ++bj) {
          p1[bj] = mfma16(a.x, bf[bj].x, p1[bj]);
          p3[bj] = mfma16(a.x, bf[bj].y, p3[bj]);
        }
#pragma unroll
        for (int bj = 0; bj < JB; ++bj) {
          p1[bj] = mfma16(-a.y, bf[bj].y, p1[bj]);
          p3[bj] = mfma16(a.y, bf[bj].x, p3[bj]);
        }
      }
    }
  if constexpr (FWD) __syncthreads();   // every displaced row has been read
#pragma unroll
  for (int bj = 0; bj < JB; ++bj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = wave * 16 + acc_row<T>(lane, r), col = bj * 16 + l16;
      const T re = G3 ? p1[bj][r] + p2[bj][r] : p1[bj][r];
      const T im = G3 ? p3[bj][r] - p1[bj][r] + p2[bj][r] : p3[bj][r];
      if (row < nbk && col < m) Xb[(long long)(k0 + row) * m + col] = make_double2((double)re, (double)im);
    }
}

// ----------------------------------------------------------------------------- launchers
size_t lu_factor_scratch_bytes(int n, size_t elem_bytes) {
  const size_t partial = sizeof(int) * ((size_t)n + RP_EXMAX);
  const size_t tournament = 2 * sizeof(int) * 64 * 64 + elem_bytes * (size_t)LU_NB * LU_NB;
  return partial > tournament ? partial : tournament;
}

template <typename T>
hipError_t lu_factor_batch(c2<T>* W, long long mstride, int n, int nbatch, void* scratch, int* perm,
                           long long perm_stride, c2<T>* Linv, c2<T>* Uinv, long long inv_stride, int* info,
                           int pivot, hipStream_t st, LuTimers* tm) {
  constexpr int NB = LU_NB, IB = 8;
  if (n > 4096 || n < 1) return hipErrorInvalidValue;
  if (pivot != LU_PIVOT_PARTIAL && pivot != LU_PIVOT_TOURNAMENT) return hipErrorInvalidValue;
  const int nsteps = (n + NB - 1) / NB;
  // per-matrix scratch: ipiv (partial pivoting), or two candidate-set buffers
  // (64 sets x 64 rows) and the saved displaced rows (NB x NB), each [nbatch][...]
  int* ipiv = static_cast<int*>(scratch);
  int* cand0 = static_cast<int*>(scratch);
  int* cand1 = cand0 + (size_t)nbatch * 64 * 64;
  c2<T>* saved = reinterpret_cast<c2<T>*>(cand1 + (size_t)nbatch * 64 * 64);
  auto panel = [&](int s) {
    const int k0 = s * NB, nbk = min(NB, n - k0), rows = n - k0;
    if (rows <= 128) {
      // the whole panel in registers (either pivot choice: this is partial pivoting)
      tslu_root_kernel<T, NB, 128, true><<<nbatch, 512, 0, st>>>(W, mstride, n, k0, nbk, s, 0, nullptr, perm,
                                                                  perm_stride, nullptr, Linv, Uinv, inv_stride, info);
    } else if (rows <= 256 && pivot != LU_PIVOT_PARTIAL) {
      tslu_root_kernel<T, NB, 256, true><<<nbatch, 1024, 0, st>>>(W, mstride, n, k0, nbk, s, 0, nullptr, perm,
                                                                   perm_stride, nullptr, Linv, Uinv, inv_stride, info);
    } else if (pivot == LU_PIVOT_PARTIAL && rows <= (sizeof(T) == 4 ? 2 : 1) * RP_NTMAX) {
      // recursive panel: register leaves with rank-W updates between them
      int* sub = ipiv + (size_t)nbatch * n;
      if (sizeof(T) == 8 || rows <= RP_NTMAX) {
        // leaves of 8 columns in pairs: the odd leaf applies the even one's update to
        // itself, and one rank-16 update per pair serves the columns right of both
        constexpr int LW = 8;
        for (int q = 0; q < NB / LW; ++q) {
          if (q & 1)
            rpanel_leaf_kernel<T, 8, 256, 4, true><<<nbatch, 256, 0, st>>>(W, mstride, n, k0, q, sub, info);
          else
            rpanel_leaf_kernel<T, 8, 256, 4, false><<<nbatch, 256, 0, st>>>(W, mstride, n, k0, q, sub, info);
          if ((q & 1) && q < NB / LW - 1) {
            const int tiles = (n - (k0 + LW * (q - 1)) - 2 * LW + 63) / 64;
            rpanel_update_kernel<T, 2 * LW><<<dim3((unsigned)(nbatch * tiles)), 256, 0, st>>>(W, mstride, n, k0,
                                                                                            (q - 1) / 2, tiles);
          }
        }
        rpanel_finish_kernel<T, NB, LW><<<nbatch, 256, 0, st>>>(W, mstride, n, k0, s, sub, perm, perm_stride, Linv,
                                                                Uinv, inv_stride);
      } else if constexpr (sizeof(T) == 4) {
        // complex64 panels of 1025..2048 rows: leaves of 16 columns, two rows per thread
        constexpr int LW = 16;
        for (int q = 0; q < NB / LW; ++q) {
          rpanel_leaf_kernel<T, 16, 1024, 2, false><<<nbatch, 1024, 0, st>>>(W, mstride, n, k0, q, sub, info);
          if (q < NB / LW - 1) {
            const int tiles = (n - (k0 + LW * q) - LW + 63) / 64;
            rpanel_update_kernel<T, LW><<<dim3((unsigned)(nbatch * tiles)), 256, 0, st>>>(W, mstride, n, k0, q,
                                                                                           tiles);
          }
        }
        rpanel_finish_kernel<T, NB, LW><<<nbatch, 256, 0, st>>>(W, mstride, n, k0, s, sub, perm, perm_stride, Linv,
                                                                Uinv, inv_stride);
      }
    } else if (pivot == LU_PIVOT_PARTIAL) {
      // panel rows n - k0 <= threads * rows-per-thread
      if (n <= 1024)
        lu_panel_kernel<T, NB, IB, 512, 2><<<nbatch, 512, 0, st>>>(W, mstride, n, k0, s, ipiv, perm, perm_stride, Linv, Uinv, inv_stride, info);
      else if (n <= 2048)
        lu_panel_kernel<T, NB, IB, 1024, 2><<<nbatch, 1024, 0, st>>>(W, mstride, n, k0, s, ipiv, perm, perm_stride, Linv, Uinv, inv_stride, info);
      else
        lu_panel_kernel<T, NB, IB, 1024, 4><<<nbatch, 1024, 0, st>>>(W, mstride, n, k0, s, ipiv, perm, perm_stride, Linv, Uinv, inv_stride, info);
    } else {
      const int nch = (rows + TSLU_ROWS - 1) / TSLU_ROWS;     // <= 32 for n <= 4096
      tslu_local_kernel<T><<<dim3((unsigned)(nbatch * nch)), TSLU_NT, 0, st>>>(W, mstride, n, k0, nbk, nch, cand0);
      int nin = nch;
      int* a = cand0;
      int* bb = cand1;
      while (nin > 2) {
        const int npair = (nin + 1) / 2;
        tslu_merge_kernel<T><<<dim3((unsigned)(nbatch * npair)), TSLU_NT, 0, st>>>(W, mstride, n, k0, nbk, nin, a, bb);
        nin = npair;
        int* x = a; a = bb; bb = x;
      }
      tslu_root_kernel<T, NB, 128, false><<<nbatch, 512, 0, st>>>(W, mstride, n, k0, nbk, s, nin, a, perm,
                                                                   perm_stride, saved, Linv, Uinv, inv_stride, info);
      const int m = n - k0 - nbk;   // > 0 here
      const int tr = (m + 63) / 64;
      const long long groups = (nbatch + 7) / 8;
      lu_gemm_kernel<T, GEMM_PANEL><<<dim3((unsigned)(groups * 8 * tr)), 256, 0, st>>>(
          W, mstride, n, k0, nbk, s, nbatch, tr, 1, perm, perm_stride, Uinv, inv_stride, saved);
    }
  };
  const long long groups = (nbatch + 7) / 8;
  // lu_gemm_dma_kernel takes full 64-column panels and, in complex64, even orders
  auto dma_ok = [&](int nbk) { return nbk == NB && (sizeof(T) == 8 || n % 2 == 0); };
  auto timed_update = [&](int mode, int k0, int nbk, int s, int m, int kdepth) {
    const int tc = (m + 63) / 64;
    // the timers follow the paired update only (the dominant kernel)
    const bool timed = mode == GEMM_UPDATE2 && tm && tm->ev_enabled && tm->npairs < LuTimers::MAXP;
    if (timed) hipEventRecord(tm->ev[2 * tm->npairs], st);
    const dim3 grid((unsigned)(groups * 8 * tc * tc));
    if (mode == GEMM_UPDATE2 && dma_ok(nbk))
      lu_gemm_dma_kernel<T, GEMM_UPDATE2><<<grid, 256, 0, st>>>(W, mstride, n, k0, nbk, s, nbatch, tc, tc, perm,
                                                                 perm_stride, Linv, inv_stride);
    else if (mode == GEMM_UPDATE && dma_ok(nbk))
      lu_gemm_dma_kernel<T, GEMM_UPDATE><<<grid, 256, 0, st>>>(W, mstride, n, k0, nbk, s, nbatch, tc, tc, perm,
                                                                perm_stride, Linv, inv_stride);
    else if (mode == GEMM_UPDATE2)
      lu_gemm_kernel<T, GEMM_UPDATE2><<<grid, 256, 0, st>>>(W, mstride, n, k0, nbk, s, nbatch, tc, tc, perm,
                                                             perm_stride, Linv, inv_stride);
    else
      lu_gemm_kernel<T, GEMM_UPDATE><<<grid, 256, 0, st>>>(W, mstride, n, k0, nbk, s, nbatch, tc, tc, perm,
                                                            perm_stride, Linv, inv_stride);
    if (timed) {
      hipEventRecord(tm->ev[2 * tm->npairs + 1], st);
      tm->npairs++;
      tm->gemm_launches += 1;   // launches and flops of the timed launches only
      tm->gemm_flops += 8.0 * (double)m * (double)m * (double)kdepth * (double)nbatch;
    }
  };
  for (int s = 0; s < nsteps;) {
    const int k0 = s * NB, nbk = min(NB, n - k0), kend = k0 + nbk, m = n - kend;
    panel(s);
    if (m <= 0) break;
    const int tc = (m + 63) / 64;
    if (dma_ok(nbk))
      lu_gemm_dma_kernel<T, GEMM_TRSM><<<dim3((unsigned)(groups * 8 * tc)), 256, 0, st>>>(
          W, mstride, n, k0, nbk, s, nbatch, 1, tc, perm, perm_stride, Linv, inv_stride);
    else
      lu_gemm_kernel<T, GEMM_TRSM><<<dim3((unsigned)(groups * 8 * tc)), 256, 0, st>>>(
          W, mstride, n, k0, nbk, s, nbatch, 1, tc, perm, perm_stride, Linv, inv_stride);
    if (s + 1 == nsteps - 1 || m <= NB) {
      // the next panel is the last one: one plain update
      timed_update(GEMM_UPDATE, k0, nbk, s, m, nbk);
      ++s;
      continue;
    }
    // delayed pair (s, s+1): make panel s+1 current, factor it, then one pass over the
    // trailing matrix for both steps
    const int tr = (m + 63) / 64;
    if (dma_ok(nbk))
      lu_gemm_dma_kernel<T, GEMM_UPDATE><<<dim3((unsigned)(groups * 8 * tr)), 256, 0, st>>>(
          W, mstride, n, k0, nbk, s, nbatch, tr, 1, perm, perm_stride, Linv, inv_stride);
    else
      lu_gemm_kernel<T, GEMM_UPDATE><<<dim3((unsigned)(groups * 8 * tr)), 256, 0, st>>>(
          W, mstride, n, k0, nbk, s, nbatch, tr, 1, perm, perm_stride, Linv, inv_stride);
    panel(s + 1);
    const int k1 = kend, nb1 = min(NB, n - k1), m1 = n - k1 - nb1;   // m1 > 0 here
    const int tc1 = (m1 + 63) / 64;
    if (dma_ok(nb1))
      lu_gemm_dma_kernel<T, GEMM_PREUPD><<<dim3((unsigned)(groups * 8 * tc1)), 256, 0, st>>>(
          W, mstride, n, k1, nb1, s + 1, nbatch, 1, tc1, perm, perm_stride, Linv, inv_stride);
    else
      lu_gemm_kernel<T, GEMM_PREUPD><<<dim3((unsigned)(groups * 8 * tc1)), 256, 0, st>>>(
          W, mstride, n, k1, nb1, s + 1, nbatch, 1, tc1, perm, perm_stride, Linv, inv_stride);
    if (dma_ok(nb1))
      lu_gemm_dma_kernel<T, GEMM_TRSM_ID><<<dim3((unsigned)(groups * 8 * tc1)), 256, 0, st>>>(
          W, mstride, n, k1, nb1, s + 1, nbatch, 1, tc1, perm, perm_stride, Linv, inv_stride);
    else
      lu_gemm_kernel<T, GEMM_TRSM_ID><<<dim3((unsigned)(groups * 8 * tc1)), 256, 0, st>>>(
          W, mstride, n, k1, nb1, s + 1, nbatch, 1, tc1, perm, perm_stride, Linv, inv_stride);
    timed_update(GEMM_UPDATE2, k1, nb1, s + 1, m1, NB + nb1);
    s += 2;
  }
  return hipGetLastError();
}

// the solve kernels for JN column groups of 8 right-hand sides
template <typename T, int JN>
static void solve_launch(const c2<T>* W, long long mstride, int n, int nbatch, const int* perm, long long perm_stride,
                         const c2<T>* Linv, const c2<T>* Uinv, long long inv_stride, double2* X, long long xstride,
                         int m, bool trans, const int* active, hipStream_t st) {
  if (trans) {
    lu_solve_kernel<T, LU_NB, true, JN><<<nbatch, 256, 0, st>>>(W, mstride, n, perm, perm_stride, Linv, Uinv, inv_stride, X, xstride, m, active);
  } else if (m > LU_SOLVE_SPLIT_M && n >= LU_SOLVE_MFMA_N) {
    constexpr int NB = LU_NB, JB = JN > 2 ? 2 : 1;
    const int nsteps = (n + NB - 1) / NB;
    const long long groups = (nbatch + 7) / 8;
    for (int s = 0; s < nsteps; ++s) {
      const int kend = min(n, s * NB + NB);
      solve_topm_kernel<T, NB, true, JB><<<nbatch, 256, 0, st>>>(n, s, perm, perm_stride, Linv, inv_stride, X, xstride,
                                                               m, active);
      if (kend < n) {
        const int tiles = (n - kend + 63) / 64, wpm = (tiles + SOLVE_TPW - 1) / SOLVE_TPW;
        solve_rowsm_kernel<T, NB, JB><<<dim3((unsigned)(groups * 8 * wpm)), 256, 0, st>>>(
            W, mstride, n, s, kend, n, tiles, nbatch, X, xstride, m, active);
      }
    }
    for (int s = nsteps - 1; s >= 0; --s) {
      const int k0 = s * NB;
      solve_topm_kernel<T, NB, false, JB><<<nbatch, 256, 0, st>>>(n, s, perm, perm_stride, Uinv, inv_stride, X,
                                                                xstride, m, active);
      if (k0 > 0) {
        const int tiles = (k0 + 63) / 64, wpm = (tiles + SOLVE_TPW - 1) / SOLVE_TPW;
        solve_rowsm_kernel<T, NB, JB><<<dim3((unsigned)(groups * 8 * wpm)), 256, 0, st>>>(
            W, mstride, n, s, 0, k0, tiles, nbatch, X, xstride, m, active);
      }
    }
  } else if (n < LU_SOLVE_SPLIT_N || m > LU_SOLVE_SPLIT_M) {
    lu_solve_kernel<T, LU_NB, false, JN><<<nbatch, 256, 0, st>>>(W, mstride, n, perm, perm_stride, Linv, Uinv, inv_stride, X, xstride, m, active);
  } else {
    constexpr int NB = LU_NB;
    const int nsteps = (n + NB - 1) / NB;
    for (int s = 0; s < nsteps; ++s) {
      const int k0 = s * NB, kend = min(n, k0 + NB);
      if (m == 1)
        solve_top1_kernel<T, NB, true><<<nbatch, 256, 0, st>>>(W, mstride, n, s, perm, perm_stride, Linv, inv_stride,
                                                             X, xstride, active);
      else
        solve_top_kernel<T, NB, true, JN><<<nbatch, 256, 0, st>>>(W, mstride, n, s, perm, perm_stride, Linv,
                                                                inv_stride, X, xstride, m, active);
      if (kend < n && m == 1) {
        const int tiles = (n - kend + 15) / 16;
        solve_rows1_kernel<T, NB><<<dim3((unsigned)(nbatch * tiles)), 256, 0, st>>>(W, mstride, n, s, kend, n, tiles,
                                                                                X, xstride, active);
      } else if (kend < n) {
        const int tiles = (n - kend + 63) / 64;
        solve_rows_kernel<T, NB, JN><<<dim3((unsigned)(nbatch * tiles)), 256, 0, st>>>(W, mstride, n, s, kend, n, tiles,
                                                                                  X, xstride, m, active);
      }
    }
    for (int s = nsteps - 1; s >= 0; --s) {
      const int k0 = s * NB;
      if (m == 1)
        solve_top1_kernel<T, NB, false><<<nbatch, 256, 0, st>>>(W, mstride, n, s, perm, perm_stride, Uinv, inv_stride,
                                                              X, xstride, active);
      else
        solve_top_kernel<T, NB, false, JN><<<nbatch, 256, 0, st>>>(W, mstride, n, s, perm, perm_stride, Uinv,
                                                                 inv_stride, X, xstride, m, active);
      if (k0 > 0 && m == 1) {
        const int tiles = (k0 + 15) / 16;
        solve_rows1_kernel<T, NB><<<dim3((unsigned)(nbatch * tiles)), 256, 0, st>>>(W, mstride, n, s, 0, k0, tiles, X,
                                                                                xstride, active);
      } else if (k0 > 0) {
        const int tiles = (k0 + 63) / 64;
        solve_rows_kernel<T, NB, JN><<<dim3((unsigned)(nbatch * tiles)), 256, 0, st>>>(W, mstride, n, s, 0, k0, tiles,
                                                                                  X, xstride, m, active);
      }
    }
  }
}

template <typename T>
hipError_t lu_solve_batch(const c2<T>* W, long long mstride, int n, int nbatch, const int* perm, long long perm_stride,
                          const c2<T>* Linv, const c2<T>* Uinv, long long inv_stride, double2* X, long long xstride,
                          int m, bool trans, const int* active, hipStream_t st) {
  if (m > 32 || m < 1) return hipErrorInvalidValue;
  switch ((m + 7) / 8) {
    case 1: solve_launch<T, 1>(W, mstride, n, nbatch, perm, perm_stride, Linv, Uinv, inv_stride, X, xstride, m, trans, active, st); break;
    case 2: solve_launch<T, 2>(W, mstride, n, nbatch, perm, perm_stride, Linv, Uinv, inv_stride, X, xstride, m, trans, active, st); break;
    case 3: solve_launch<T, 3>(W, mstride, n, nbatch, perm, perm_stride, Linv, Uinv, inv_stride, X, xstride, m, trans, active, st); break;
    default: solve_launch<T, 4>(W, mstride, n, nbatch, perm, perm_stride, Linv, Uinv, inv_stride, X, xstride, m, trans, active, st); break;
  }
  return hipGetLastError();
}

template hipError_t lu_factor_batch<double>(c2<double>*, long long, int, int, void*, int*, long long, c2<double>*,
                                            c2<double>*, long long, int*, int, hipStream_t, LuTimers*);
template hipError_t lu_factor_batch<float>(c2<float>*, long long, int, int, void*, int*, long long, c2<float>*,
                                           c2<float>*, long long, int*, int, hipStream_t, LuTimers*);
template hipError_t lu_solve_batch<double>(const c2<double>*, long long, int, int, const int*, long long,
                                           const c2<double>*, const c2<double>*, long long, double2*, long long, int,
                                           bool, const int*, hipStream_t);
template hipError_t lu_solve_batch<float>(const c2<float>*, long long, int, int, const int*, long long,
                                          const c2<float>*, const c2<float>*, long long, double2*, long long, int,
                                          bool, const int*, hipStream_t);

}  // namespace nep
