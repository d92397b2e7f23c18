// Truncation of the two-site state (Steps 4 and 6), all in FP64 on the device.
//
// k_jacobi: one workgroup (16 wave64) per centre-charge block M[r x c].  The
// rows of X (X = M if r <= c, else M^T; n = min(r, c) rows of length p) are
// orthogonalised by one-sided (Hestenes) Jacobi rotations in round-robin
// order, n/2 disjoint pairs per round, the rotations accumulated in G (n x n).
// Then G X = diag(sigma) Z^T: for X = M, U = G^T and V = Z; for X = M^T,
// U = Z and V = G^T.  The rows of Z are finally re-orthonormalised in order of
// decreasing sigma (classical Gram-Schmidt twice), and rows of zero norm are
// replaced by unit vectors orthogonalised the same way, so every returned
// singular vector set is orthonormal, including zero-weight states.
//
// k_select: one workgroup per problem.  Normalises the spectrum to
// sum lambda^2 = 1, ranks nonzero values (ties by charge, then index), and
// chooses the kept set, the discarded weight eps and eps'.
#include "internal.h"

namespace idmrg {
namespace {

constexpr int JT = 1024;
constexpr int JW = JT / 64;
constexpr int kSvdMaxN = 4096;

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ void rr_pair(int nn, int round, int slot, int& i, int& j) {
  // circle method: player 0 fixed, players 1..nn-1 rotate
  auto L = [&](int t) { return t == 0 ? 0 : 1 + ((round + t - 1) % (nn - 1)); };
  i = L(slot);
  j = L(nn - 1 - slot);
  if (i > j) { int x = i; i = j; j = x; }
}

// Euclidean norm of z[0..p) by the whole workgroup (fixed summation order).
__device__ double block_norm(const double* z, int p, double* s_red, double* s_val) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double a = 0.0;
  for (int k = t; k < p; k += JT) a += z[k] * z[k];
  a = wsum(a);
  if (lane == 0) s_red[wave] = a;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int w = 0; w < JW; ++w) s += s_red[w];
    *s_val = s;
  }
  __syncthreads();
  const double r = sqrt(*s_val);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(JT) void k_jacobi(const SvdTask* __restrict__ tasks, void* const* __restrict__ bases,
                                               int32_t* sweeps_out) {
  __shared__ int s_order[kSvdMaxN];
  __shared__ double s_coef[kSvdMaxN];
  __shared__ int s_rot;
  __shared__ double s_red[JW];
  __shared__ double s_val;
  const SvdTask tk = tasks[blockIdx.x];
  const int r = tk.r, c = tk.c;
  const bool tr = r > c;
  const int n = tr ? c : r, p = tr ? r : c;
  double* M = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 1]) + tk.m_off;
  double* X = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 2]) + tk.x_off;
  double* G = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 3]) + tk.g_off;
  double* Uf = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 4]) + tk.u_off;
  double* Vf = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 5]) + tk.v_off;
  double* S = reinterpret_cast<double*>(bases[tk.prob * kNumBases + 6]) + tk.s_off;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;

  for (int64_t e = t; e < (int64_t)n * p; e += JT) {
    const int i = (int)(e / p), k = (int)(e % p);
    X[e] = tr ? M[(int64_t)k * c + i] : M[(int64_t)i * c + k];
  }
  for (int64_t e = t; e < (int64_t)n * n; e += JT) G[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();

  const double tol = fmax(1e-15, 4.4e-16 * sqrt((double)p));
  const int nn = n + (n & 1);
  int sweep = 0;
  if (n > 1) {
    for (sweep = 0; sweep < 40; ++sweep) {
      if (t == 0) s_rot = 0;
      __syncthreads();
      for (int round = 0; round < nn - 1; ++round) {
        for (int slot = wave; slot < nn / 2; slot += JW) {
          int i, j;
          rr_pair(nn, round, slot, i, j);
          if (j >= n) continue;
          double* xi = X + (int64_t)i * p;
          double* xj = X + (int64_t)j * p;
          double a = 0.0, b = 0.0, g = 0.0;
          for (int k = lane; k < p; k += 64) {
            const double u = xi[k], v = xj[k];
            a += u * u;
            b += v * v;
            g += u * v;
          }
          a = wsum(a);
          b = wsum(b);
          g = wsum(g);
          if (g != 0.0 && fabs(g) > tol * sqrt(a * b)) {
            const double zeta = (b - a) / (2.0 * g);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
            for (int k = lane; k < p; k += 64) {
              const double u = xi[k], v = xj[k];
              xi[k] = cs * u - sn * v;
              xj[k] = sn * u + cs * v;
            }
            double* gi = G + (int64_t)i * n;
            double* gj = G + (int64_t)j * n;
            for (int k = lane; k < n; k += 64) {
              const double u = gi[k], v = gj[k];
              gi[k] = cs * u - sn * v;
              gj[k] = sn * u + cs * v;
            }
            if (lane == 0) s_rot = 1;
          }
        }
        __syncthreads();
      }
      const int rot = s_rot;
      __syncthreads();
      if (!rot) break;
    }
  }
  // singular values = row norms; Z rows = X rows / sigma
  for (int i = wave; i < n; i += JW) {
    double* xi = X + (int64_t)i * p;
    double a = 0.0;
    for (int k = lane; k < p; k += 64) a += xi[k] * xi[k];
    a = wsum(a);
    const double sg = sqrt(a);
    if (lane == 0) S[i] = sg;
    const double inv = sg > 0.0 ? 1.0 / sg : 0.0;
    for (int k = lane; k < p; k += 64) xi[k] *= inv;
  }
  __syncthreads();
  // Re-orthonormalise Z in order of decreasing sigma (ties by index).
  for (int i = t; i < n; i += JT) {
    const double si = S[i];
    int rk = 0;
    for (int k = 0; k < n; ++k) {
      const double sk = S[k];
      rk += (sk > si) || (sk == si && k < i);
    }
    s_order[rk] = i;
  }
  __syncthreads();
  int next_unit = 0;
  for (int q = 0; q < n; ++q) {
    double* zi = X + (int64_t)s_order[q] * p;
    bool accepted = false;
    for (int attempt = 0; attempt <= p && !accepted; ++attempt) {
      if (attempt > 0) {  // replace by the next unit vector
        for (int k = t; k < p; k += JT) zi[k] = (k == next_unit) ? 1.0 : 0.0;
        ++next_unit;
        __syncthreads();
      }
      const double before = block_norm(zi, p, s_red, &s_val);
      if (before == 0.0) continue;
      for (int pass = 0; pass < 2; ++pass) {
        for (int qq = wave; qq < q; qq += JW) {
          const double* zr = X + (int64_t)s_order[qq] * p;
          double d = 0.0;
          for (int k = lane; k < p; k += 64) d += zr[k] * zi[k];
          d = wsum(d);
          if (lane == 0) s_coef[qq] = d;
        }
        __syncthreads();
        for (int k = t; k < p; k += JT) {
          double acc = 0.0;
          for (int qq = 0; qq < q; ++qq) acc += s_coef[qq] * X[(int64_t)s_order[qq] * p + k];
          zi[k] -= acc;
        }
        __syncthreads();
      }
      const double after = block_norm(zi, p, s_red, &s_val);
      if (after > 1e-3 * before) {
        const double inv = 1.0 / after;
        for (int k = t; k < p; k += JT) zi[k] *= inv;
        accepted = true;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // outputs
  if (!tr) {
    // U [r x n] = G^T, V [c x n] = Z^T
    for (int64_t e = t; e < (int64_t)r * n; e += JT) {
      const int row = (int)(e / n), col = (int)(e % n);
      Uf[e] = G[(int64_t)col * n + row];
    }
    for (int64_t e = t; e < (int64_t)c * n; e += JT) {
      const int row = (int)(e / n), col = (int)(e % n);
      Vf[e] = X[(int64_t)col * p + row];
    }
  } else {
    for (int64_t e = t; e < (int64_t)r * n; e += JT) {
      const int row = (int)(e / n), col = (int)(e % n);
      Uf[e] = X[(int64_t)col * p + row];
    }
    for (int64_t e = t; e < (int64_t)c * n; e += JT) {
      const int row = (int)(e / n), col = (int)(e % n);
      Vf[e] = G[(int64_t)col * n + row];
    }
  }
  if (t == 0 && sweeps_out) sweeps_out[blockIdx.x] = sweep;
}


constexpr int ST = 1024;
constexpr int kSelMax = 8192;

__device__ double block_sum_st(double x, double* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int s = ST / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// One workgroup per problem.  Candidate c (0..ncand) belongs to sector sec[c]
// with index jj[c] inside that sector's decomposition (sectors in ascending
// charge).  Outputs: kept count per sector, for each sector its kept indices
// (colmap) and values (lam_sel) in output order, and scal = {eps, eps',
// cut_gap, m_kept}.
__global__ __launch_bounds__(ST) void k_select(const SelTask* __restrict__ tasks, const SelSector* __restrict__ secs,
                                               const double* __restrict__ S, int32_t* kept_per_sec,
                                               int32_t* colmap, double* lam_sel, double* scal) {
  __shared__ double lam[kSelMax];
  __shared__ int16_t sec[kSelMax];
  __shared__ int16_t jj[kSelMax];
  __shared__ int16_t pos[kSelMax];   // global output position, -1 if discarded
  __shared__ int16_t sorted[kSelMax];
  __shared__ double sh[ST];
  __shared__ int s_cnt[ST];
  __shared__ int s_mk, s_npos;
  __shared__ double s_gap;
  const SelTask tk = tasks[blockIdx.x];
  const int t = threadIdx.x;
  const int nc = tk.ncand;
  // load candidates
  for (int s = 0; s < tk.nsec; ++s) {
    const SelSector sc = secs[tk.sec0 + s];
    for (int k = t; k < sc.n; k += ST) {
      const int ci = sc.cand0 - tk.cand0 + k;
      lam[ci] = S[sc.s_off + k];
      sec[ci] = (int16_t)s;
      jj[ci] = (int16_t)k;
    }
  }
  __syncthreads();
  double acc = 0.0;
  for (int c = t; c < nc; c += ST) acc += lam[c] * lam[c];
  const double total = block_sum_st(acc, sh);
  const double inv = total > 0.0 ? 1.0 / sqrt(total) : 0.0;
  for (int c = t; c < nc; c += ST) lam[c] *= inv;
  __syncthreads();
  // ranks: nonzero values by (value desc, sector asc, index asc); zeros by (sector, index) = candidate order
  int my_npos = 0;
  for (int c = t; c < nc; c += ST) my_npos += lam[c] > tk.lam_floor;
  s_cnt[t] = my_npos;
  __syncthreads();
  if (t == 0) {
    int n = 0;
    for (int k = 0; k < ST; ++k) n += s_cnt[k];
    s_npos = n;
  }
  __syncthreads();
  const int npos = s_npos;
  for (int c = t; c < nc; c += ST) {
    const double lc = lam[c];
    if (lc > tk.lam_floor) {
      int rk = 0;
      for (int k = 0; k < nc; ++k) {
        const double lk = lam[k];
        if (lk > tk.lam_floor)
          rk += (lk > lc) || (lk == lc && (sec[k] < sec[c] || (sec[k] == sec[c] && jj[k] < jj[c])));
      }
      pos[c] = (int16_t)rk;
      sorted[rk] = (int16_t)c;
    } else {
      int zr = 0;
      for (int k = 0; k < c; ++k) zr += lam[k] <= tk.lam_floor;
      pos[c] = (int16_t)(npos + zr);
    }
  }
  __syncthreads();
  const int target = tk.m_max < nc ? tk.m_max : nc;
  if (t == 0) {
    int mk;
    double gap = -1.0;
    if (target < npos) {
      mk = target;
      while (mk > 0 && lam[sorted[mk - 1]] - lam[sorted[mk]] <= tk.deg_rel * lam[sorted[mk - 1]]) --mk;
      if (mk == 0) mk = target;
      gap = (lam[sorted[mk - 1]] - lam[sorted[mk]]) / lam[sorted[mk - 1]];
    } else {
      mk = target;
    }
    s_mk = mk;
    s_gap = gap;
  }
  __syncthreads();
  const int mk = s_mk;
  for (int c = t; c < nc; c += ST)
    if (pos[c] >= mk) pos[c] = -1;
  __syncthreads();
  // discarded weight (fixed order) and per-sector output order
  double dw = 0.0;
  for (int c = t; c < nc; c += ST)
    if (pos[c] < 0) dw += lam[c] * lam[c];
  const double eps = block_sum_st(dw, sh);
  for (int s = 0; s < tk.nsec; ++s) {
    const SelSector sc = secs[tk.sec0 + s];
    const int base = sc.cand0 - tk.cand0;
    int mine = 0;
    for (int k = t; k < sc.n; k += ST) {
      const int c = base + k;
      if (pos[c] < 0) continue;
      ++mine;
      int o = 0;
      for (int k2 = 0; k2 < sc.n; ++k2) {
        const int c2 = base + k2;
        o += pos[c2] >= 0 && pos[c2] < pos[c];
      }
      colmap[sc.cand0 + o] = k;
      lam_sel[sc.cand0 + o] = lam[c] > tk.lam_floor ? lam[c] : 0.0;
    }
    s_cnt[t] = mine;
    __syncthreads();
    if (t == 0) {
      int tot = 0;
      for (int k = 0; k < ST; ++k) tot += s_cnt[k];
      kept_per_sec[tk.sec0 + s] = tot;
    }
    __syncthreads();
  }
  if (t == 0) {
    double* o = scal + 4 * (int64_t)blockIdx.x;
    o[0] = eps;
    o[1] = eps / (1.0 + sqrt(fmax(0.0, 1.0 - eps)));
    o[2] = s_gap;
    o[3] = (double)mk;
  }
}

}  // namespace

void launch_svd(const SvdTask* tasks, int ntask, void* const* bases, int32_t* sweeps_out, hipStream_t s) {
  if (ntask == 0) return;
  hipLaunchKernelGGL(k_jacobi, dim3(ntask), dim3(JT), 0, s, tasks, bases, sweeps_out);
}

void launch_select(const SelTask* tasks, int ntask, const SelSector* secs, const double* S, int32_t* kept_per_sec,
                   int32_t* colmap, double* lam_sel, double* scal, hipStream_t s) {
  if (ntask == 0) return;
  hipLaunchKernelGGL(k_select, dim3(ntask), dim3(ST), 0, s, tasks, secs, S, kept_per_sec, colmap, lam_sel, scal);
}

}  // namespace idmrg
