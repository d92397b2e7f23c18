// Selection of the kept Schmidt states (Steps 4 and 6), in FP64 on the device.
//
// k_select: one workgroup per problem.  Normalises the spectrum to
// sum lambda^2 = 1, ranks nonzero values (ties by charge, then index), and
// chooses the kept set, the discarded weight eps and eps'.
#include "internal.h"

namespace idmrg {
namespace {

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
      // zero-weight states only when every candidate is kept (the whole block space);
      // a part of the null space would be an arbitrary choice
      mk = target == nc ? target : npos;
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

// flag[0] = 1 if any of x[0..n) is NaN or infinite (flag cleared by the caller).
__global__ __launch_bounds__(256) void k_check_finite(const double* __restrict__ x, int64_t n, int32_t* flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    bad |= !isfinite(x[i]);
  if (bad) flag[0] = 1;
}

}  // namespace

void launch_check_finite(const double* x, int64_t n, int32_t* flag, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, s, x, n, flag);
}

void launch_select(const SelTask* tasks, int ntask, const SelSector* secs, const double* S, int32_t* kept_per_sec,
                   int32_t* colmap, double* lam_sel, double* scal, hipStream_t s) {
  if (ntask == 0) return;
  hipLaunchKernelGGL(k_select, dim3(ntask), dim3(ST), 0, s, tasks, secs, S, kept_per_sec, colmap, lam_sel, scal);
}

}  // namespace idmrg
