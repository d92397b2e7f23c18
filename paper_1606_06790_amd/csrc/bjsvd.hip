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
  const double* X = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 2]) + tk.x_off;
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
  double* X = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 2]) + tk.x_off;
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

}  // namespace

void bj_prepare(const std::vector<SvdTask>& svd, BjPlan& plan) {
  const int nm = (int)svd.size();
  plan = BjPlan{};
  plan.nm = nm;
  if (nm == 0) return;
  std::vector<BjMat> mats(nm);
  struct Round {
    std::vector<BjPair> pairs;
    std::vector<BjItem> gram, apply;
  };
  std::vector<Round> rounds;
  for (int m = 0; m < nm; ++m) {
    const SvdTask& t = svd[m];
    const bool tr = t.r > t.c;
    const int n = tr ? t.c : t.r, p = tr ? t.r : t.c;
    mats[m] = BjMat{n, p, t.prob, 0, t.x_off, t.g_off};
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
