// Blocked one-sided Jacobi SVD of many matrices at once (Step 4).
//
// Each centre-charge block M[r x c] is handled as X (n rows of length p,
// X = M if r <= c else M^T, n = min(r, c)) whose rows are made mutually
// orthogonal by orthogonal transformations accumulated in G (n x n), so that
// G X = diag(sigma) Z^T.  The rows are grouped in blocks of 32.  One sweep
// pairs every block with every other block once (round-robin, nb-1 rounds of
// nb/2 disjoint pairs).  A round of all matrices takes three launches, so
// that the pairs of the largest blocks are spread over many workgroups:
//   1. partial 64 x 64 Gram matrices of Y = [X_I; X_J] over column chunks of
//      256 (FP64 MFMA), one workgroup per (pair, chunk);
//   2. per pair, their sum S = Y Y^T (in chunk order) is diagonalised by
//      cyclic two-sided Jacobi in LDS (32 disjoint rotations per step),
//      accumulating Q with Q^T S Q diagonal;
//   3. Y <- Q^T Y and [G_I; G_J] <- Q^T [G_I; G_J] (FP64 MFMA), one workgroup
//      per (pair, chunk of 256 columns of X or of G).
// A pair whose rows are already orthogonal to the relative tolerance is left
// alone; a sweep in which no pair of a matrix moved ends that matrix.
//
// QR preconditioning (Drmac and Veselic's preconditioned one-sided Jacobi,
// here without column pivoting: the rows are sorted by norm first).  For a
// matrix of n >= kQrMinN rows, X^T = Q1 R1 and R1^T = Q2 R2 by blocked
// Householder QR (panels of kQrB reflectors, compact WY form), and the Jacobi
// sweeps orthogonalise the rows of R2 (n x n) instead of those of X; they need
// about half as many sweeps.  With G started as Q2^T P (P the norm sort), the
// accumulated G still satisfies G X_orig = (current rows), and the final rows
// are mapped back by Q1: F = [R2 rows after Jacobi, 0] Q1^T.  In the row
// storage used here row j of a factored matrix holds R[0..j][j] in entries
// 0..j and the reflector v_j (v_j[j] = 1 implicit) in entries j+1..len-1.
//
// Null rows: a row whose norm is at most zero_rel * |M|_F carries no
// trustworthy direction (its singular value is below the truncation floor and
// at the level of rounding in the other rows), and Jacobi rotations between
// such a row and a large one can fail to converge (the rotation angle
// underflows).  Pairs involving a null row are therefore left out of the
// convergence test, and k_bj_finish replaces every null row of Z by a unit
// vector orthogonalised (twice) against all other rows, keeping its norm as
// the singular value.  This keeps every returned set of singular vectors
// orthonormal, including the zero-weight states.
#include "internal.h"

#include <algorithm>
#include <cstring>
#include <functional>

namespace idmrg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BB = 32;          // rows per block
constexpr int PB = 2 * BB;      // rows per pair
constexpr int LD = PB + 1;      // LDS leading dimension
constexpr int kBjMaxN = 4096;   // largest min(r, c) of one matrix (LDS arrays of k_bj_finish)
constexpr int kBjMaxP = 8192;   // largest max(r, c) of one matrix

struct BjMat {                  // one matrix (device)
  int32_t n, p, prob, pad;
  int64_t x_off, g_off;
};

struct BjPair {                 // one block pair in one round (bj = -1: padding block)
  int32_t mat, bi, bj;
  int32_t g0, ng;               // its Gram chunks: items [g0, g0 + ng) of the round's Gram list
  int32_t pad[3];
};

struct BjItem {                 // one column chunk [c0, c1) of a pair: of X (which = 0) or G (which = 1)
  int32_t pair, c0, c1, which;
};

constexpr int kChunk = 256;     // columns per Gram or rotation chunk (four 64-column tiles)
constexpr int kQrB = 16;        // reflectors per QR panel
constexpr int kQrMinN = 64;     // matrices with fewer rows are not preconditioned
constexpr int kQrRows = 32;     // target rows per workgroup of the reflector application

struct QrMat {                  // one matrix of the QR preconditioning (device); offsets in the X base
  int32_t n, p, prob, qr;
  int64_t a, f, y, j, k, t1, t2, g;
};

struct QrItem {                 // target rows [r0, r1) of one matrix
  int32_t mat, r0, r1, pad;
};

// Operands are read through global-address-space pointers from clamped
// (always valid) indices; a tail that must read as zero is cleared with a mask
// the optimiser cannot turn into a branch around the load.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
  return (gptr<T>)(p);
}
__device__ __forceinline__ uint32_t lane_mask(bool c) {
  uint32_t m = c ? 0xffffffffu : 0u;
  asm("" : "+v"(m));
  return m;
}
__device__ __forceinline__ double keep(double v, uint32_t m) {
  return __longlong_as_double(__double_as_longlong(v) & (long long)(((uint64_t)m << 32) | m));
}

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// FP64 16x16x4 accumulator layout: register r of lane l holds C[l/16 + 4r][l%16].
template <typename F>
__device__ __forceinline__ void store64(const v4d acc[2][2], F put) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) put(wm + i * 16 + (lane >> 4) + 4 * r, wn + j * 16 + (lane & 15), acc[i][j][r]);
}

// Row of the pair's local row i (0..63) in its matrix, or -1 for a padding row.
__device__ __forceinline__ int pair_row(const BjPair& pr, int n, int i) {
  const int r = i < BB ? pr.bi * BB + i : pr.bj * BB + (i - BB);
  const bool ok = i < BB ? (pr.bi >= 0 && r < n) : (pr.bj >= 0 && r < n);
  return ok ? r : -1;
}

// 1. Partial Gram matrix of one pair over one column chunk [c0, c1) of X:
// P = Y[:, c0:c1] Y[:, c0:c1]^T (64 x 64, padding rows included; they are
// masked when the partials are summed).  Tiles of 64 rows (local rows
// k = wave + 4q, q < 16) x 64 columns are loaded whole, the next one into
// registers while the current one is multiplied; the staged tile
// T[k][i] = Y[i][c + k] serves as both MFMA operands.  Columns past c1 read
// as zero; padding rows read a real row (clamped).
__global__ __launch_bounds__(256) void k_bj_gram(const BjItem* __restrict__ items, const BjPair* __restrict__ pairs,
                                                 const BjMat* __restrict__ mats, void* const* __restrict__ bases,
                                                 const int32_t* __restrict__ done, double* __restrict__ partial) {
  __shared__ double T[PB][LD];
  const BjItem it = items[blockIdx.x];
  const BjPair pr = pairs[it.pair];
  if (done[pr.mat]) return;
  const BjMat mt = mats[pr.mat];
  const int n = mt.n, p = mt.p;
  const double* X = reinterpret_cast<double*>(bases[mt.prob * kNumBases + 2]) + mt.x_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  constexpr int NQ = PB / 4;
  const gptr<double> Xg = as_global(X);
  int offs[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = pair_row(pr, n, wave + 4 * q);
    offs[q] = (r >= 0 ? r : pr.bi * BB) * p;
  }
  const int c1 = it.c1;
  double v[NQ];
  auto ld = [&](int c0) {
    const int k = c0 + lane, kc = k < c1 ? k : c1 - 1;
    const uint32_t m = lane_mask(k < c1);
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = keep(Xg[offs[q] + kc], m);
  };
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0, 0, 0, 0};
  ld(it.c0);
  for (int c0 = it.c0; c0 < c1; c0 += PB) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) T[lane][wave + 4 * q] = v[q];
    __syncthreads();
    if (c0 + PB < c1) ld(c0 + PB);
#pragma unroll 4
    for (int kk = 0; kk < PB; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = T[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = T[kr][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  double* P = partial + (size_t)blockIdx.x * (PB * PB);
  store64(acc, [&](int i, int j, double x) { P[i * PB + j] = x; });
}

// 2. One workgroup per pair: S = sum of the pair's partial Gram matrices (in
// chunk order), masked on padding rows; if some pair of non-null rows is
// coupled beyond the tolerance, S is diagonalised by cyclic two-sided Jacobi
// (round-robin, 32 disjoint rotations per step, at most inner_sweeps sweeps)
// and the accumulated rotation Q (Q^T S Q diagonal) is written out; move[pair]
// says whether Q is to be applied.
__global__ __launch_bounds__(256) void k_bj_rotate(const BjPair* __restrict__ pairs, const BjMat* __restrict__ mats,
                                                   const int32_t* __restrict__ done, int32_t* __restrict__ changed,
                                                   const double* __restrict__ thr2, const double* __restrict__ partial,
                                                   double* __restrict__ Qout, int32_t* __restrict__ move, double tol,
                                                   int inner_sweeps) {
  __shared__ double S[PB][LD];
  __shared__ double Q[PB][LD];
  __shared__ double cs_[PB / 2], sn_[PB / 2];
  __shared__ int pidx[PB / 2], qidx[PB / 2];
  __shared__ int s_move;
  const BjPair pr = pairs[blockIdx.x];
  const int t = threadIdx.x;
  if (done[pr.mat]) {
    if (t == 0) move[blockIdx.x] = 0;
    return;
  }
  const int n = mats[pr.mat].n;
  {
    // element e = t + 256 k of S, k < NE; the chunks are summed in order, with all
    // loads of one chunk in flight together
    constexpr int NE = PB * PB / 256;
    double a[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) a[k] = 0.0;
    for (int g = 0; g < pr.ng; ++g) {
      const double* P = partial + (size_t)(pr.g0 + g) * (PB * PB) + t;
      double x[NE];
#pragma unroll
      for (int k = 0; k < NE; ++k) x[k] = P[256 * k];
#pragma unroll
      for (int k = 0; k < NE; ++k) a[k] += x[k];
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = t + 256 * k, i = e / PB, j = e % PB;
      S[i][j] = (pair_row(pr, n, i) >= 0 && pair_row(pr, n, j) >= 0) ? a[k] : 0.0;
      Q[i][j] = i == j ? 1.0 : 0.0;
    }
  }
  if (t == 0) s_move = 0;
  __syncthreads();
  // is any pair of non-null rows coupled beyond the tolerance?
  const double z2 = thr2[pr.mat];
  {
    bool mv = false;
    for (int e = t; e < PB * PB; e += 256) {
      const int i = e / PB, j = e % PB;
      if (i < j) {
        const double sij = S[i][j], sii = S[i][i], sjj = S[j][j];
        if (sii > z2 && sjj > z2 && fabs(sij) > tol * sqrt(sii) * sqrt(sjj)) mv = true;
      }
    }
    if (mv) s_move = 1;
  }
  __syncthreads();
  if (!s_move) {
    if (t == 0) move[blockIdx.x] = 0;
    return;
  }
  if (t == 0) changed[pr.mat] = 1;
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    for (int round = 0; round < PB - 1; ++round) {
      if (t < PB / 2) {
        auto L = [&](int x) { return x == 0 ? 0 : 1 + ((round + x - 1) % (PB - 1)); };
        int a = L(t), b = L(PB - 1 - t);
        if (a > b) { const int z = a; a = b; b = z; }
        const double app = S[a][a], aqq = S[b][b], apq = S[a][b];
        double c = 1.0, sn = 0.0;
        if (app > z2 && aqq > z2 && fabs(apq) > tol * sqrt(app) * sqrt(aqq)) {
          const double zeta = (aqq - app) / (2.0 * apq);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          sn = c * tt;
        }
        pidx[t] = a; qidx[t] = b; cs_[t] = c; sn_[t] = sn;
      }
      __syncthreads();
      // S <- J^T S J and Q <- Q J in one pass: thread-owned 2 x 2 blocks
      // (pair u of rows, pair v of columns) are rotated in place.  Thread t
      // owns blocks (t / 32 + 8k, t % 32), k < 4; all blocks of a step are
      // disjoint, so every load is issued before the first store.
      {
        constexpr int NB = (PB / 2) * (PB / 2) / 256;
        const int v = t % (PB / 2), u0 = t / (PB / 2);
        const int av = pidx[v], bv = qidx[v];
        const double cv = cs_[v], sv = sn_[v];
        int au[NB], bu[NB];
        double cu[NB], su[NB], m[NB][4], q[NB][4];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int u = u0 + (256 / (PB / 2)) * k;
          au[k] = pidx[u]; bu[k] = qidx[u]; cu[k] = cs_[u]; su[k] = sn_[u];
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          m[k][0] = S[au[k]][av]; m[k][1] = S[au[k]][bv]; m[k][2] = S[bu[k]][av]; m[k][3] = S[bu[k]][bv];
          q[k][0] = Q[au[k]][av]; q[k][1] = Q[au[k]][bv]; q[k][2] = Q[bu[k]][av]; q[k][3] = Q[bu[k]][bv];
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const double x00 = cv * m[k][0] - sv * m[k][1], x01 = sv * m[k][0] + cv * m[k][1];   // columns
          const double x10 = cv * m[k][2] - sv * m[k][3], x11 = sv * m[k][2] + cv * m[k][3];
          S[au[k]][av] = cu[k] * x00 - su[k] * x10;                                            // rows
          S[bu[k]][av] = su[k] * x00 + cu[k] * x10;
          S[au[k]][bv] = cu[k] * x01 - su[k] * x11;
          S[bu[k]][bv] = su[k] * x01 + cu[k] * x11;
          Q[au[k]][av] = cv * q[k][0] - sv * q[k][1];
          Q[au[k]][bv] = sv * q[k][0] + cv * q[k][1];
          Q[bu[k]][av] = cv * q[k][2] - sv * q[k][3];
          Q[bu[k]][bv] = sv * q[k][2] + cv * q[k][3];
        }
      }
      __syncthreads();
    }
    if (t == 0) s_move = 0;
    __syncthreads();
    bool mv = false;
    for (int e = t; e < PB * PB; e += 256) {
      const int i = e / PB, j = e % PB;
      if (i < j) {
        const double sij = S[i][j], sii = S[i][i], sjj = S[j][j];
        if (sii > z2 && sjj > z2 && fabs(sij) > tol * sqrt(sii) * sqrt(sjj)) mv = true;
      }
    }
    if (mv) s_move = 1;
    __syncthreads();
    if (!s_move) break;
  }
  double* Qg = Qout + (size_t)blockIdx.x * (PB * PB);
  for (int e = t; e < PB * PB; e += 256) Qg[e] = Q[e / PB][e % PB];
  if (t == 0) move[blockIdx.x] = 1;
}

// 3. Y <- Q^T Y on one column chunk [c0, c1) of X (the pair's rows) or of G.
// The A operand is Q (LDS); the B tile T[k][c] = rows of the pair at columns
// c + k is staged whole (the next one loaded into registers meanwhile).
// Padding rows need no masking: Q is the identity on them, so they only feed
// padding outputs, which are not stored.  Every output column depends only on
// the same input column, and a tile is read completely before any of it is
// written; reads are clamped into the chunk, so chunks of other workgroups
// are never touched.
__global__ __launch_bounds__(256) void k_bj_apply(const BjItem* __restrict__ items, const BjPair* __restrict__ pairs,
                                                  const BjMat* __restrict__ mats, void* const* __restrict__ bases,
                                                  const int32_t* __restrict__ done, const double* __restrict__ Qin,
                                                  const int32_t* __restrict__ move) {
  __shared__ double T[PB][LD];
  __shared__ double Q[PB][LD];
  const BjItem it = items[blockIdx.x];
  const BjPair pr = pairs[it.pair];
  if (done[pr.mat] || !move[it.pair]) return;
  const BjMat mt = mats[pr.mat];
  const int n = mt.n;
  const int len = it.which ? n : mt.p;
  double* Mx = reinterpret_cast<double*>(bases[mt.prob * kNumBases + (it.which ? 3 : 2)]) +
               (it.which ? mt.g_off : mt.x_off);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  {
    constexpr int NE = PB * PB / 256;
    const double* Qg = Qin + (size_t)it.pair * (PB * PB) + t;
    double x[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) x[k] = Qg[256 * k];
#pragma unroll
    for (int k = 0; k < NE; ++k) Q[(t + 256 * k) / PB][(t + 256 * k) % PB] = x[k];
  }
  constexpr int NQ = PB / 4;
  const gptr<double> Mg = as_global((const double*)Mx);
  int offs[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = pair_row(pr, n, wave + 4 * q);
    offs[q] = (r >= 0 ? r : pr.bi * BB) * len;
  }
  const int c1 = it.c1;
  double v[NQ];
  auto ld = [&](int c0) {
    const int col = c0 + lane < c1 ? c0 + lane : c1 - 1;
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = Mg[offs[q] + col];
  };
  ld(it.c0);
  v4d acc[2][2];
  for (int c0 = it.c0; c0 < c1; c0 += PB) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) T[wave + 4 * q][lane] = v[q];
    __syncthreads();
    if (c0 + PB < c1) ld(c0 + PB);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0, 0, 0, 0};
#pragma unroll 4
    for (int kk = 0; kk < PB; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = Q[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = T[kr][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    store64(acc, [&](int i, int j, double x) {
      const int r = pair_row(pr, n, i);
      if (r >= 0 && c0 + j < c1) Mx[(int64_t)r * len + c0 + j] = x;
    });
  }
}

// done[m] |= (no pair of m moved in this sweep); changed[m] = 0
// QR panel k of every preconditioned matrix, one workgroup each: the kQrB
// Householder reflectors of rows j0 = k kQrB .. j0 + jb - 1 (which = 1: the
// sorted X, rows of length p; which = 2: R1 in Y, rows of length n), applied
// within the panel, and the upper triangular T with H_j0 ... H_j0+jb-1 =
// I - V T V^T (16 x 16, zero padded).  The panel's entries j0 .. len - 1 are
// worked on in LDS when they fit (kQrVL per row), else in memory.  Reductions
// in a fixed order.
constexpr int kQrVLP = 1152;

__global__ __launch_bounds__(1024) void k_qr_panel(const QrMat* __restrict__ qm, void* const* __restrict__ bases,
                                                  int k, int which) {
  __shared__ double red[16];
  __shared__ double s_tau[kQrB];
  __shared__ double s_gram[kQrB][kQrB];
  __shared__ double s_T[kQrB * kQrB];
  __shared__ double Ps[kQrB * kQrVLP];
  const QrMat m = qm[blockIdx.x];
  const int n = m.n, j0 = k * kQrB;
  if (!m.qr || j0 >= n) return;
  const int jb = min(kQrB, n - j0), len = which == 1 ? m.p : n;
  const int vl = len - j0;
  const bool staged = vl <= kQrVLP;
  double* base = reinterpret_cast<double*>(bases[m.prob * kNumBases + 2]);
  double* F = base + (which == 1 ? m.a : m.y);
  double* T = base + (which == 1 ? m.t1 : m.t2) + (int64_t)k * kQrB * kQrB;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // entry e (j0 <= e < len) of panel row i
  auto at = [&](int i, int e) -> double& { return staged ? Ps[i * vl + (e - j0)] : F[(int64_t)(j0 + i) * len + e]; };
  if (staged) {
    for (int x = t; x < jb * vl; x += 1024) Ps[x] = F[(int64_t)(j0 + x / vl) * len + j0 + x % vl];
    __syncthreads();
  }
  for (int jj = 0; jj < jb; ++jj) {
    const int j = j0 + jj;
    double a = 0.0;
    for (int e = j + 1 + t; e < len; e += 1024) {
      const double v = at(jj, e);
      a += v * v;
    }
    a = wsum(a);
    if (lane == 0) red[wave] = a;
    __syncthreads();
    double sigma = 0.0;
    for (int w = 0; w < 16; ++w) sigma += red[w];
    const double alpha = at(jj, j);
    __syncthreads();   // every thread has read red and the diagonal entry
    double beta = alpha, tau = 0.0;
    if (sigma > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      const double scale = 1.0 / (alpha - beta);
      for (int e = j + 1 + t; e < len; e += 1024) at(jj, e) *= scale;
    }
    if (t == 0) {
      at(jj, j) = beta;
      s_tau[jj] = tau;
    }
    __syncthreads();
    for (int r = jj + 1 + wave; r < jb; r += 16) {
      const double yj = at(r, j);
      double w = 0.0;
      for (int e = j + 1 + lane; e < len; e += 64) w += at(jj, e) * at(r, e);
      w = wsum(w) + yj;
      const double tw = tau * w;
      for (int e = j + 1 + lane; e < len; e += 64) at(r, e) -= tw * at(jj, e);
      if (lane == 0) at(r, j) = yj - tw;
    }
    __syncthreads();
  }
  // s_gram[a][b] = v_a . v_b (a < b): v_b starts at its unit entry j0 + b, where v_a holds entry j0 + b of row a
  for (int pr = wave; pr < jb * jb; pr += 16) {
    const int ia = pr / jb, ib = pr % jb;
    if (ia >= ib) continue;
    double g = 0.0;
    for (int e = j0 + ib + 1 + lane; e < len; e += 64) g += at(ia, e) * at(ib, e);
    g = wsum(g) + at(ia, j0 + ib);
    if (lane == 0) s_gram[ia][ib] = g;
  }
  __syncthreads();
  if (staged)
    for (int x = t; x < jb * vl; x += 1024) F[(int64_t)(j0 + x / vl) * len + j0 + x % vl] = Ps[x];
  // T, column by column: T[jj][jj] = tau_jj, T[i][jj] = -tau_jj sum_{i <= l < jj} T[i][l] gram[l][jj]
  if (t < kQrB * kQrB) s_T[t] = 0.0;
  __syncthreads();
  for (int jj = 0; jj < jb; ++jj) {
    if (t < jj) {
      double acc = 0.0;
      for (int l = t; l < jj; ++l) acc += s_T[t * kQrB + l] * s_gram[l][jj];
      s_T[t * kQrB + jj] = -s_tau[jj] * acc;
    }
    if (t == jj) s_T[jj * kQrB + jj] = s_tau[jj];
    __syncthreads();
  }
  if (t < kQrB * kQrB) T[t] = s_T[t];
}

// Block reflector of panel k applied to rows [r0, r1) (one item per workgroup,
// eight waves, two rows per wave at a time):
//   mode 0 (factorisation, which = 1 or 2): rows r >= j0 + jb of the matrix
//     being factored, x_r <- (I - V T^T V^T) x_r on entries j0 .. len - 1;
//   mode 1 (Q applied; the panels run in reverse order): rows of the target
//     (which = 1: F, length p; which = 2: K, length n), x_r <- (I - V T V^T) x_r.
// The panel's reflectors, entries j0 .. len - 1 with their zeros and unit
// entries written out, are staged in LDS when they fit (kQrVL entries per
// reflector); otherwise they are read from memory.
constexpr int kQrVL = 1152;

__device__ __forceinline__ double qr_v(const double* F, int len, int j0, int jb, int i, int e) {
  const int ji = j0 + i;
  return (i >= jb || e < ji) ? 0.0 : (e == ji ? 1.0 : F[(int64_t)ji * len + e]);
}

template <bool STAGED>
__global__ __launch_bounds__(512) void k_qr_update(const QrMat* __restrict__ qm, const QrItem* __restrict__ items,
                                                   void* const* __restrict__ bases, int k, int which, int mode) {
  __shared__ double Ts[kQrB][kQrB];
  __shared__ double Vs[STAGED ? kQrB * kQrVL : 1];
  constexpr int RW = STAGED ? 2 : 1;   // rows per wave at a time
  const QrItem it = items[blockIdx.x];
  const QrMat m = qm[it.mat];
  const int n = m.n, j0 = k * kQrB;
  const int jb = min(kQrB, n - j0), len = which == 1 ? m.p : n;
  const int vl = len - j0;
  double* base = reinterpret_cast<double*>(bases[m.prob * kNumBases + 2]);
  const double* F = base + (which == 1 ? m.a : m.y);
  double* C = mode == 0 ? base + (which == 1 ? m.a : m.y) : base + (which == 1 ? m.f : m.k);
  const double* Tg = base + (which == 1 ? m.t1 : m.t2) + (int64_t)k * kQrB * kQrB;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t < kQrB * kQrB) Ts[t / kQrB][t % kQrB] = Tg[t];
  if (STAGED)
    for (int x = t; x < kQrB * vl; x += 512) Vs[x] = qr_v(F, len, j0, jb, x / vl, j0 + x % vl);
  __syncthreads();
  for (int r = it.r0 + RW * wave; r < it.r1; r += 8 * RW) {
    double* y[RW];
    bool live[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      live[q] = r + q < it.r1;
      y[q] = C + (int64_t)(live[q] ? r + q : r) * len;
    }
    double acc[RW][kQrB];
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
      for (int i = 0; i < kQrB; ++i) acc[q][i] = 0.0;
    for (int e = j0 + lane; e < len; e += 64) {
      double ye[RW];
#pragma unroll
      for (int q = 0; q < RW; ++q) ye[q] = y[q][e];
#pragma unroll
      for (int i = 0; i < kQrB; ++i) {
        const double v = STAGED ? Vs[i * vl + (e - j0)] : qr_v(F, len, j0, jb, i, e);
#pragma unroll
        for (int q = 0; q < RW; ++q) acc[q][i] += v * ye[q];
      }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
      for (int i = 0; i < kQrB; ++i) acc[q][i] = wsum(acc[q][i]);
    // u[q][b] = sum_a acc[q][a] T'[a][b] (T' = T or T^T): lane b of every 16 computes column b, then all lanes
    // take the 16 values (acc is the same in every lane after the reductions)
    double u[RW][kQrB];
    const int bl = lane & (kQrB - 1);
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      double s = 0.0;
      for (int a = 0; a < kQrB; ++a) s += acc[q][a] * (mode == 0 ? Ts[a][bl] : Ts[bl][a]);
#pragma unroll
      for (int b = 0; b < kQrB; ++b) u[q][b] = __shfl(s, b, 64);
    }
    for (int e = j0 + lane; e < len; e += 64) {
      double sv[RW];
#pragma unroll
      for (int q = 0; q < RW; ++q) sv[q] = 0.0;
#pragma unroll
      for (int i = 0; i < kQrB; ++i) {
        const double v = STAGED ? Vs[i * vl + (e - j0)] : qr_v(F, len, j0, jb, i, e);
#pragma unroll
        for (int q = 0; q < RW; ++q) sv[q] += u[q][i] * v;
      }
#pragma unroll
      for (int q = 0; q < RW; ++q)
        if (live[q]) y[q][e] -= sv[q];
    }
  }
}

// Copies between the stages, rows blockIdx.x, blockIdx.x + gridDim.x, ... of matrix blockIdx.y:
//   0: Y = R1 (row-major, from the factored sorted X: R1[i][j] = A[j][i] for i <= j)
//   1: J = R2 (from the factored Y), K = I
//   2: F = [J, 0] (rows of length p)
__global__ __launch_bounds__(256) void k_qr_copy(const QrMat* __restrict__ qm, void* const* __restrict__ bases,
                                                 int stage) {
  const QrMat m = qm[blockIdx.y];
  if (!m.qr) return;
  const int n = m.n, p = m.p;
  double* base = reinterpret_cast<double*>(bases[m.prob * kNumBases + 2]);
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    if (stage == 0) {
      double* y = base + m.y + (int64_t)i * n;
      for (int j = threadIdx.x; j < n; j += 256) y[j] = i <= j ? base[m.a + (int64_t)j * p + i] : 0.0;
    } else if (stage == 1) {
      double* jr = base + m.j + (int64_t)i * n;
      double* kr = base + m.k + (int64_t)i * n;
      for (int j = threadIdx.x; j < n; j += 256) {
        jr[j] = i <= j ? base[m.y + (int64_t)j * n + i] : 0.0;
        kr[j] = i == j ? 1.0 : 0.0;
      }
    } else {
      double* fr = base + m.f + (int64_t)i * p;
      const double* jr = base + m.j + (int64_t)i * n;
      for (int e = threadIdx.x; e < p; e += 256) fr[e] = e < n ? jr[e] : 0.0;
    }
  }
}

// G (the sort permutation P, G[i][idx[i]] = 1, idx also in S) <- K P with K = Q2^T:  G[i][idx[l]] = K[i][l].
// Rows blockIdx.y, blockIdx.y + gridDim.y, ... of matrix blockIdx.x.
__global__ __launch_bounds__(256) void k_qr_g0(const QrMat* __restrict__ qm, const SvdTask* __restrict__ tasks,
                                               void* const* __restrict__ bases) {
  const QrMat m = qm[blockIdx.x];
  if (!m.qr) return;
  const int n = m.n;
  double* G = reinterpret_cast<double*>(bases[m.prob * kNumBases + 3]) + m.g;
  const double* K = reinterpret_cast<double*>(bases[m.prob * kNumBases + 2]) + m.k;
  const double* S = reinterpret_cast<double*>(bases[m.prob * kNumBases + 6]) + tasks[blockIdx.x].s_off;
  for (int i = blockIdx.y; i < n; i += gridDim.y)
    for (int l = threadIdx.x; l < n; l += 256) G[(int64_t)i * n + (int)S[l]] = K[(int64_t)i * n + l];
}

__global__ void k_bj_sweep_end(int nm, int32_t* done, int32_t* changed) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nm) return;
  if (!changed[m]) done[m] = 1;
  changed[m] = 0;
}

// X = P M (r <= c) or P M^T (r > c) with the permutation P that puts the
// rows in order of decreasing norm (ties by index); G = P; thr2 = (zero_rel
// |M|_F)^2.  One workgroup per matrix.  Starting from norm-sorted rows (de
// Rijk's ordering) keeps rows of similar weight in the same blocks, which
// cuts the sweeps one-sided Jacobi needs on strongly graded matrices such as
// the blocks of a converged two-site state.
__global__ __launch_bounds__(256) void k_bj_init(const SvdTask* __restrict__ tasks, void* const* __restrict__ bases,
                                                 double* __restrict__ thr2, double zero_rel) {
  __shared__ double key[kBjMaxN];
  __shared__ int idx[kBjMaxN];
  __shared__ double red[4];
  const SvdTask tk = tasks[blockIdx.x];
  const bool tr = tk.r > tk.c;
  const int n = tr ? tk.c : tk.r, p = tr ? tk.r : tk.c;
  const double* M = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 1]) + tk.m_off;
  double* X = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 2]) + tk.x_off;
  double* G = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 3]) + tk.g_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // squared row norms of X (row i of X is row i of M, or column i of M)
  if (tr) {
    for (int i = t; i < n; i += 256) {
      double a = 0.0;
      for (int k = 0; k < p; ++k) {
        const double v = M[(int64_t)k * tk.c + i];
        a += v * v;
      }
      key[i] = a;
    }
  } else {
    for (int i = wave; i < n; i += 4) {
      double a = 0.0;
      for (int k = lane; k < p; k += 64) {
        const double v = M[(int64_t)i * p + k];
        a += v * v;
      }
      a = wsum(a);
      if (lane == 0) key[i] = a;
    }
  }
  int P2 = 1;
  while (P2 < n) P2 <<= 1;
  for (int i = t; i < P2; i += 256) {
    if (i >= n) key[i] = -1.0;   // sorts after every real row
    idx[i] = i;
  }
  __syncthreads();
  // |M|_F^2 in a fixed order
  double a = 0.0;
  for (int i = t; i < n; i += 256) a += key[i];
  a = wsum(a);
  if (lane == 0) red[wave] = a;
  // bitonic sort of (key descending, index ascending)
  for (int size = 2; size <= P2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = t; i < P2; i += 256) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;   // this run ends up in the requested order
          const double ki = key[i], kj = key[j];
          const int ii = idx[i], ij = idx[j];
          const bool i_first = ki > kj || (ki == kj && ii < ij);
          if (i_first != desc) {
            key[i] = kj; key[j] = ki;
            idx[i] = ij; idx[j] = ii;
          }
        }
      }
    }
  __syncthreads();
  for (int64_t e = t; e < (int64_t)n * p; e += 256) {
    const int i = (int)(e / p), k = (int)(e % p);
    const int src = idx[i];
    X[e] = tr ? M[(int64_t)k * tk.c + src] : M[(int64_t)src * p + k];
  }
  for (int64_t e = t; e < (int64_t)n * n; e += 256) G[e] = (e % n == idx[e / n]) ? 1.0 : 0.0;
  // the permutation also goes to S (free until the singular values are written) for the QR preconditioning
  double* S = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 6]) + tk.s_off;
  for (int i = t; i < n; i += 256) S[i] = (double)idx[i];
  if (t == 0) thr2[blockIdx.x] = zero_rel * zero_rel * (((red[0] + red[1]) + red[2]) + red[3]);
}

__device__ double block_norm2(const double* z, int p, double* red) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double a = 0.0;
  for (int k = t; k < p; k += 1024) a += z[k] * z[k];
  a = wsum(a);
  if (lane == 0) red[wave] = a;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < 16; ++w) s += red[w];
  __syncthreads();
  return s;
}

// sigma_i = |X_i| of every row, by the reduction k_bj_finish uses.
__global__ __launch_bounds__(1024) void k_bj_sigma(const SvdTask* __restrict__ tasks, void* const* __restrict__ bases) {
  const SvdTask tk = tasks[blockIdx.x];
  const bool tr = tk.r > tk.c;
  const int n = tr ? tk.c : tk.r, p = tr ? tk.r : tk.c;
  const double* X = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 2]) + tk.f_off;
  double* S = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 6]) + tk.s_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int i = wave; i < n; i += 16) {
    const double* xi = X + (int64_t)i * p;
    double a = 0.0;
    for (int k = lane; k < p; k += 64) a += xi[k] * xi[k];
    a = wsum(a);
    const double sg = sqrt(a);
    if (lane == 0) S[i] = !(sg > 1e-150) ? 0.0 : sg;
  }
}

// sigma_i = |X_i|, Z_i = X_i / sigma_i; null rows (|X_i|^2 <= thr2) are zeroed
// and then, if complete[m], become unit vectors orthogonalised (twice) against
// all other rows; then the singular vectors are written as U_full [r x n] and
// V_full [c x n].
__global__ __launch_bounds__(1024) void k_bj_finish(const SvdTask* __restrict__ tasks, void* const* __restrict__ bases,
                                                    const double* __restrict__ thr2,
                                                    const int32_t* __restrict__ complete) {
  __shared__ double red[16];
  __shared__ double coef[kBjMaxN];
  __shared__ unsigned char nul[kBjMaxN];
  __shared__ double cw[kBjMaxP];
  __shared__ unsigned char used[kBjMaxP];
  __shared__ double s_bv[16];
  __shared__ int s_bk[16];
  __shared__ int s_k;
  const SvdTask tk = tasks[blockIdx.x];
  const int r = tk.r, c = tk.c;
  const bool tr = r > c;
  const int n = tr ? c : r, p = tr ? r : c;
  double* X = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 2]) + tk.f_off;
  double* G = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 3]) + tk.g_off;
  double* Uf = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 4]) + tk.u_off;
  double* Vf = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 5]) + tk.v_off;
  double* S = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 6]) + tk.s_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const double z2 = thr2[blockIdx.x];
  for (int i = wave; i < n; i += 16) {
    double* xi = X + (int64_t)i * p;
    double a = 0.0;
    for (int k = lane; k < p; k += 64) a += xi[k] * xi[k];
    a = wsum(a);
    const double sg = sqrt(a);
    const bool tiny = !(sg > 1e-150);
    const bool null_row = tiny || !(a > z2);
    if (lane == 0) {
      S[i] = tiny ? 0.0 : sg;
      nul[i] = null_row ? 1 : 0;
    }
    const double inv = null_row ? 0.0 : 1.0 / sg;
    for (int k = lane; k < p; k += 64) xi[k] *= inv;
  }
  __syncthreads();
  // Completion: null row i becomes e_k, orthogonalised (twice) against all
  // other rows, for the unused coordinate k of least weight cw[k] = sum_q Z[q][k]^2
  // over the rows present so far.  Since the rows are orthonormal, the
  // residual of e_k has squared norm 1 - cw[k], which is largest for that k
  // and is positive while fewer than p rows are present.
  __shared__ int s_nnull;
  if (t == 0) {
    int cnt = 0;
    for (int i = 0; i < n; ++i) cnt += nul[i];
    s_nnull = cnt;
  }
  __syncthreads();
  if (s_nnull > 0 && complete[blockIdx.x]) {
    for (int k = t; k < p; k += 1024) {
      double a = 0.0;
      for (int q = 0; q < n; ++q) {
        const double z = X[(int64_t)q * p + k];
        a += z * z;
      }
      cw[k] = a;
      used[k] = 0;
    }
    __syncthreads();
    for (int i = 0; i < n; ++i) {
      if (!nul[i]) continue;              // uniform: nul is in LDS and was synchronised
      double* zi = X + (int64_t)i * p;
      bool ok = false;
      while (!ok) {
        double bv = 1e300;
        int bk = p;
        for (int k = t; k < p; k += 1024)
          if (!used[k] && cw[k] < bv) bv = cw[k], bk = k;   // k ascending: ties keep the lowest
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const double ov = __shfl_xor(bv, o, 64);
          const int ok2 = __shfl_xor(bk, o, 64);
          if (ov < bv || (ov == bv && ok2 < bk)) bv = ov, bk = ok2;
        }
        if (lane == 0) s_bv[wave] = bv, s_bk[wave] = bk;
        __syncthreads();
        if (t == 0) {
          double v = s_bv[0];
          int kb = s_bk[0];
          for (int w = 1; w < 16; ++w)
            if (s_bv[w] < v || (s_bv[w] == v && s_bk[w] < kb)) v = s_bv[w], kb = s_bk[w];
          s_k = kb;
          if (kb < p) used[kb] = 1;
        }
        __syncthreads();
        const int kk = s_k;
        if (kk >= p) break;                 // no coordinate left (not reached while rows < p)
        for (int k = t; k < p; k += 1024) zi[k] = (k == kk) ? 1.0 : 0.0;
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
          for (int q = wave; q < n; q += 16) {
            if (q == i) { if (lane == 0) coef[q] = 0.0; continue; }
            const double* zq = X + (int64_t)q * p;
            double d = 0.0;
            for (int k = lane; k < p; k += 64) d += zq[k] * zi[k];
            d = wsum(d);
            if (lane == 0) coef[q] = d;
          }
          __syncthreads();
          for (int k = t; k < p; k += 1024) {
            double acc = 0.0;
            for (int q = 0; q < n; ++q) acc += coef[q] * X[(int64_t)q * p + k];
            zi[k] -= acc;
          }
          __syncthreads();
        }
        const double nn = sqrt(block_norm2(zi, p, red));
        if (nn > 1e-8) {
          for (int k = t; k < p; k += 1024) zi[k] /= nn;
          ok = true;
        }
        __syncthreads();
      }
      for (int k = t; k < p; k += 1024) cw[k] += zi[k] * zi[k];
      __syncthreads();
    }
  }
  __syncthreads();
  if (!tr) {
    for (int64_t e = t; e < (int64_t)r * n; e += 1024) Uf[e] = G[(e % n) * (int64_t)n + e / n];
    for (int64_t e = t; e < (int64_t)c * n; e += 1024) Vf[e] = X[(e % n) * (int64_t)p + e / n];
  } else {
    for (int64_t e = t; e < (int64_t)r * n; e += 1024) Uf[e] = X[(e % n) * (int64_t)p + e / n];
    for (int64_t e = t; e < (int64_t)c * n; e += 1024) Vf[e] = G[(e % n) * (int64_t)n + e / n];
  }
}

int64_t qr_panels(int n) { return (n + kQrB - 1) / kQrB; }

}  // namespace

// Per matrix in the X base: the sorted rows A (n x p; with preconditioning, then its QR factorisation); with
// preconditioning also the final rows F (n x p), Y (R1, then its factorisation), J (R2, the Jacobi rows), K (Q2^T),
// each n x n, and the T matrices of both factorisations.
int64_t bj_x_elems(int n, int p) {
  if (n < kQrMinN) return (int64_t)n * p;
  return 2 * (int64_t)n * p + 3 * (int64_t)n * n + 2 * qr_panels(n) * kQrB * kQrB;
}

int64_t bj_f_rel(int n, int p) { return n < kQrMinN ? 0 : (int64_t)n * p; }

void bj_prepare(const std::vector<SvdTask>& svd, BjPlan& plan) {
  const int nm = (int)svd.size();
  plan = BjPlan{};
  plan.nm = nm;
  if (nm == 0) return;
  std::vector<BjMat> mats(nm);
  std::vector<QrMat> qm(nm);
  struct Round {
    std::vector<BjPair> pairs;
    std::vector<BjItem> gram, apply;
  };
  std::vector<Round> rounds;
  int npanel = 0;
  for (int m = 0; m < nm; ++m) {
    const SvdTask& t = svd[m];
    const bool tr = t.r > t.c;
    const int n = tr ? t.c : t.r, p0 = tr ? t.r : t.c;
    const bool qr = n >= kQrMinN;
    QrMat& q = qm[m];
    q.n = n; q.p = p0; q.prob = t.prob; q.qr = qr ? 1 : 0;
    q.a = t.x_off; q.f = t.f_off; q.g = t.g_off;
    q.y = q.f + (int64_t)n * p0; q.j = q.y + (int64_t)n * n; q.k = q.j + (int64_t)n * n;
    q.t1 = q.k + (int64_t)n * n; q.t2 = q.t1 + qr_panels(n) * kQrB * kQrB;
    if (qr) {
      if (t.f_off != t.x_off + bj_f_rel(n, p0)) throw std::runtime_error("internal: SVD task layout");
      ++plan.nqr;
      npanel = std::max<int>(npanel, (int)qr_panels(n));
    }
    // the Jacobi sweeps run on R2 (n x n) where preconditioned
    const int p = qr ? n : p0;
    mats[m] = BjMat{n, p, t.prob, 0, qr ? q.j : t.x_off, t.g_off};
    const int nb = (n + BB - 1) / BB;
    const int nbe = nb + (nb & 1);
    for (int rd = 0; rd < nbe - 1; ++rd) {
      if ((int)rounds.size() <= rd) rounds.emplace_back();
      for (int slot = 0; slot < nbe / 2; ++slot) {
        auto L = [&](int x) { return x == 0 ? 0 : 1 + ((rd + x - 1) % (nbe - 1)); };
        int a = L(slot), b = L(nbe - 1 - slot);
        if (a > b) std::swap(a, b);
        Round& R = rounds[rd];
        const int k = (int)R.pairs.size();
        BjPair pr{m, a, b < nb ? b : -1, (int)R.gram.size(), 0, {0, 0, 0}};
        for (int c0 = 0; c0 < p; c0 += kChunk) R.gram.push_back(BjItem{k, c0, std::min(p, c0 + kChunk), 0});
        pr.ng = (int)R.gram.size() - pr.g0;
        for (int c0 = 0; c0 < p; c0 += kChunk) R.apply.push_back(BjItem{k, c0, std::min(p, c0 + kChunk), 0});
        for (int c0 = 0; c0 < n; c0 += kChunk) R.apply.push_back(BjItem{k, c0, std::min(n, c0 + kChunk), 1});
        R.pairs.push_back(pr);
      }
    }
  }
  std::vector<char>& host = plan.host;
  auto put = [&](const void* p, size_t bytes) {
    const size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + std::max<size_t>(bytes, 8));
    if (bytes) std::memcpy(host.data() + off, p, bytes);
    return off;
  };
  plan.omats = put(mats.data(), mats.size() * sizeof(BjMat));
  plan.oqr = put(qm.data(), qm.size() * sizeof(QrMat));
  plan.npanel = npanel;
  plan.otrail.assign(npanel, 0);
  plan.ofull.assign(npanel, 0);
  plan.ntrail.assign(npanel, 0);
  plan.nfull.assign(npanel, 0);
  plan.vl1.assign(npanel, 0);
  plan.vl2.assign(npanel, 0);
  for (int k = 0; k < npanel; ++k) {
    std::vector<QrItem> trail, full;
    for (int m = 0; m < nm; ++m) {
      const QrMat& q = qm[m];
      if (!q.qr || k * kQrB >= q.n) continue;
      plan.vl1[k] = std::max(plan.vl1[k], q.p - k * kQrB);
      plan.vl2[k] = std::max(plan.vl2[k], q.n - k * kQrB);
      for (int r0 = (k + 1) * kQrB; r0 < q.n; r0 += kQrRows) trail.push_back(QrItem{m, r0, std::min(q.n, r0 + kQrRows), 0});
      for (int r0 = 0; r0 < q.n; r0 += kQrRows) full.push_back(QrItem{m, r0, std::min(q.n, r0 + kQrRows), 0});
    }
    plan.otrail[k] = put(trail.data(), trail.size() * sizeof(QrItem));
    plan.ofull[k] = put(full.data(), full.size() * sizeof(QrItem));
    plan.ntrail[k] = (int)trail.size();
    plan.nfull[k] = (int)full.size();
  }
  const size_t nr = rounds.size();
  plan.opair.resize(nr);
  plan.ogram.resize(nr);
  plan.oapply.resize(nr);
  plan.npair.resize(nr);
  plan.ngram.resize(nr);
  plan.napply.resize(nr);
  size_t max_pairs = 0, max_gram = 0;
  for (size_t r = 0; r < nr; ++r) {
    plan.opair[r] = put(rounds[r].pairs.data(), rounds[r].pairs.size() * sizeof(BjPair));
    plan.ogram[r] = put(rounds[r].gram.data(), rounds[r].gram.size() * sizeof(BjItem));
    plan.oapply[r] = put(rounds[r].apply.data(), rounds[r].apply.size() * sizeof(BjItem));
    plan.npair[r] = (int)rounds[r].pairs.size();
    plan.ngram[r] = (int)rounds[r].gram.size();
    plan.napply[r] = (int)rounds[r].apply.size();
    max_pairs = std::max(max_pairs, rounds[r].pairs.size());
    max_gram = std::max(max_gram, rounds[r].gram.size());
  }
  std::vector<int32_t> zeros(2 * (size_t)nm, 0);
  plan.oflags = put(zeros.data(), zeros.size() * 4);
  std::vector<double> zthr(nm, 0.0);
  plan.othr = put(zthr.data(), zthr.size() * 8);
  std::vector<int32_t> complete(nm, 1);
  plan.ocomp = put(complete.data(), complete.size() * 4);
  // per round: partial Gram matrices, rotations, move flags (reused by every round)
  const size_t tile = (size_t)PB * PB * sizeof(double);
  plan.b_partial = max_gram * tile;
  plan.b_q = max_pairs * tile;
  plan.scratch = plan.b_partial + plan.b_q + max_pairs * 4 + 256;
}

void bj_svd(const BjPlan& plan, void* const* dbases, const SvdTask* dtasks, BjScratch& scr, hipStream_t s,
            const char* dev, char* work, const std::function<void()>& sync) {
  const int nm = plan.nm;
  if (nm == 0) return;
  double* partial = (double*)work;
  double* Qs = (double*)(work + plan.b_partial);
  int32_t* move = (int32_t*)(work + plan.b_partial + plan.b_q);
  const BjMat* dmats = (const BjMat*)(dev + plan.omats);
  int32_t* done = (int32_t*)(dev + plan.oflags);
  int32_t* changed = done + nm;
  double* thr2 = (double*)(dev + plan.othr);
  hipLaunchKernelGGL(k_bj_init, dim3(nm), dim3(256), 0, s, dtasks, dbases, thr2, scr.zero_rel);
  const QrMat* dqr = (const QrMat*)(dev + plan.oqr);
  auto apply_panels = [&](int which, int mode, bool reverse) {
    for (int kk = 0; kk < plan.npanel; ++kk) {
      const int k = reverse ? plan.npanel - 1 - kk : kk;
      const int nit = mode == 0 ? plan.ntrail[k] : plan.nfull[k];
      const QrItem* it = (const QrItem*)(dev + (mode == 0 ? plan.otrail[k] : plan.ofull[k]));
      if (mode == 0) hipLaunchKernelGGL(k_qr_panel, dim3(nm), dim3(1024), 0, s, dqr, dbases, k, which);
      if (nit == 0) continue;
      // reflectors staged in LDS when every matrix's panel fits
      if ((which == 1 ? plan.vl1[k] : plan.vl2[k]) <= kQrVL)
        hipLaunchKernelGGL(k_qr_update<true>, dim3(nit), dim3(512), 0, s, dqr, it, dbases, k, which, mode);
      else
        hipLaunchKernelGGL(k_qr_update<false>, dim3(nit), dim3(512), 0, s, dqr, it, dbases, k, which, mode);
    }
  };
  if (plan.nqr > 0) {
    apply_panels(1, 0, false);                                                       // sorted X^T = Q1 R1
    hipLaunchKernelGGL(k_qr_copy, dim3(64, nm), dim3(256), 0, s, dqr, dbases, 0);   // Y = R1
    apply_panels(2, 0, false);                                                       // R1^T = Q2 R2
    hipLaunchKernelGGL(k_qr_copy, dim3(64, nm), dim3(256), 0, s, dqr, dbases, 1);   // J = R2, K = I
    apply_panels(2, 1, true);                                                        // K = Q2^T
    hipLaunchKernelGGL(k_qr_g0, dim3(nm, 64), dim3(256), 0, s, dqr, dtasks, dbases);  // G = Q2^T P
  }
  std::vector<int32_t> hdone(nm);
  int sweeps = 0;
  scr.converged = 0;
  scr.done_at.assign(nm, -1);
  const size_t nr = plan.opair.size();
  for (; sweeps < scr.max_sweeps; ++sweeps) {
    for (size_t r = 0; r < nr; ++r) {
      const BjPair* pr = (const BjPair*)(dev + plan.opair[r]);
      hipLaunchKernelGGL(k_bj_gram, dim3((unsigned)plan.ngram[r]), dim3(256), 0, s,
                         (const BjItem*)(dev + plan.ogram[r]), pr, dmats, dbases, (const int32_t*)done, partial);
      hipLaunchKernelGGL(k_bj_rotate, dim3((unsigned)plan.npair[r]), dim3(256), 0, s, pr, dmats,
                         (const int32_t*)done, changed, (const double*)thr2, (const double*)partial, Qs, move,
                         scr.tol, scr.inner_sweeps);
      hipLaunchKernelGGL(k_bj_apply, dim3((unsigned)plan.napply[r]), dim3(256), 0, s,
                         (const BjItem*)(dev + plan.oapply[r]), pr, dmats, dbases, (const int32_t*)done,
                         (const double*)Qs, (const int32_t*)move);
    }
    hipLaunchKernelGGL(k_bj_sweep_end, dim3((nm + 255) / 256), dim3(256), 0, s, nm, done, changed);
    if (hipMemcpyAsync(hdone.data(), done, nm * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      throw HipFailure("hipMemcpyAsync of Jacobi flags failed");
    sync();
    for (int m = 0; m < nm; ++m)
      if (hdone[m] && scr.done_at[m] < 0) scr.done_at[m] = sweeps + 1;
    if (std::all_of(hdone.begin(), hdone.end(), [](int32_t v) { return v != 0; })) {
      scr.converged = 1;
      break;
    }
  }
  scr.sweeps = std::min(sweeps + 1, scr.max_sweeps);
  if (plan.nqr > 0) {
    hipLaunchKernelGGL(k_qr_copy, dim3(64, nm), dim3(256), 0, s, dqr, dbases, 2);   // F = [J, 0]
    apply_panels(1, 1, true);                                                        // F = [J, 0] Q1^T
  }
  int32_t* dcomp = (int32_t*)(dev + plan.ocomp);
  std::vector<int32_t> complete(nm, 1);
  if (scr.need_completion) {
    hipLaunchKernelGGL(k_bj_sigma, dim3(nm), dim3(1024), 0, s, dtasks, dbases);
    scr.need_completion(complete);
    if (hipMemcpyAsync(dcomp, complete.data(), nm * 4, hipMemcpyHostToDevice, s) != hipSuccess)
      throw HipFailure("hipMemcpyAsync of completion flags failed");
    sync();   // the host vector must outlive the copy
  }
  scr.completed = (int)std::count(complete.begin(), complete.end(), 1);
  hipLaunchKernelGGL(k_bj_finish, dim3(nm), dim3(1024), 0, s, dtasks, dbases, (const double*)thr2,
                     (const int32_t*)dcomp);
}

}  // namespace idmrg
