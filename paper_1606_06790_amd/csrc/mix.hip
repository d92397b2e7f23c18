// Bandwidth-bound kernels of the plans: the MPO channel mixing between the two
// environment GEMMs (and plain block copies), diagonal scalings with column
// selection, element conversions for the mixed-precision policies, and the
// packs of FP64 blocks into the fragment layout of the split-bf16 GEMM.
//
// A mix tile is 32 rows x 64 columns; 256 threads each produce 8 outputs of
// one column, so every row segment is read and written as 512 contiguous bytes.
#include "internal.h"

namespace idmrg {
namespace {

constexpr int MR = 32, MC = 64;

template <typename T>
__device__ __forceinline__ double ld_as_double(const void* base, int64_t idx) {
  return (double)reinterpret_cast<const T*>(base)[idx];
}

__device__ __forceinline__ uint32_t split_bf16(float x) {
  // hi = round-to-nearest-even bf16 of x; lo = bf16(x - hi)
  uint32_t u = __float_as_uint(x);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  uint32_t hi = r & 0xffff0000u;
  float rem = x - __uint_as_float(hi);
  uint32_t v = __float_as_uint(rem);
  uint32_t r2 = v + 0x7fffu + ((v >> 16) & 1u);
  return (hi >> 16) | (r2 & 0xffff0000u);
}

__device__ __forceinline__ int find_tile(const int32_t* tile0, int stride_words, int ntask, int tile) {
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tile0[(int64_t)mid * stride_words] <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Output tag of the mix kernel: split-bf16 pairs in the fragment layout.
struct FragOut {};

template <typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void mix_kernel(const MixTask* __restrict__ tasks, const MixSrc* __restrict__ srcs,
                                                  int ntask, void* const* __restrict__ bases,
                                                  const int32_t* __restrict__ active) {
  const int tile = blockIdx.x;
  const int ti = find_tile(&tasks[0].tile0, sizeof(MixTask) / 4, ntask, tile);
  const MixTask& tk = tasks[ti];
  if (active && !active[tk.prob]) return;
  const int local = tile - tk.tile0;
  const int r0 = (local / tk.tiles_c) * MR;
  const int c = (local % tk.tiles_c) * MC + (threadIdx.x & 63);
  const int rbase = r0 + (threadIdx.x >> 6);
  if (c >= tk.cols) return;
  double acc[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) acc[e] = 0.0;
  for (int k = 0; k < tk.nsrc; ++k) {
    const MixSrc& s = srcs[tk.src0 + k];
    const TIN* base = reinterpret_cast<const TIN*>(bases[tk.prob * kNumBases + s.base]) + s.off;
    const double coef = s.coef;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = rbase + 4 * e;
      if (r < tk.rows) {
        const int64_t idx = s.trans ? ((int64_t)c * s.ld + r) : ((int64_t)r * s.ld + c);
        acc[e] += coef * (double)base[idx];
      }
    }
  }
  if constexpr (std::is_same<TOUT, FragOut>::value) {
    // element (r0 + r, c0 + c) of the fragment matrix: the word of its hi part is in
    // fragment (row / 16, k / 32) at lane (row % 16) + 16 (k % 32 / 8); the lo part
    // is half a fragment (256 words) further
    uint16_t* dst = reinterpret_cast<uint16_t*>(bases[tk.prob * kNumBases + tk.dbase]) + 2 * tk.doff;
    const int kk = tk.c0 + c;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = rbase + 4 * e;
      if (r < tk.rows) {
        const int R = tk.r0 + r;
        const int64_t w = ((int64_t)(R >> 4) * tk.ldd + (kk >> 5)) * kFragWords +
                          ((R & 15) + 16 * ((kk & 31) >> 3)) * 4 + ((kk & 7) >> 1);
        const uint32_t v = split_bf16((float)acc[e]);
        dst[2 * w + (kk & 1)] = (uint16_t)(v & 0xffffu);
        dst[2 * (w + kFragWords / 2) + (kk & 1)] = (uint16_t)(v >> 16);
      }
    }
  } else {
    TOUT* dst = reinterpret_cast<TOUT*>(bases[tk.prob * kNumBases + tk.dbase]) + tk.doff;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = rbase + 4 * e;
      if (r < tk.rows) dst[(int64_t)r * tk.ldd + c] = (TOUT)acc[e];
    }
  }
}

// One thread per (fragment, lane): the 8 values of one row in one 32-wide k
// block, stored as 16 bytes of the hi plane and 16 bytes of the lo plane, so a
// wave writes 2 KB contiguously.  Values outside [R x K] are zeros.
__global__ __launch_bounds__(256) void pack_kernel(const PackTask* __restrict__ tasks, int ntask,
                                                   void* const* __restrict__ sbases, void* const* __restrict__ dbases,
                                                   const int32_t* __restrict__ active) {
  const int tile = blockIdx.x;
  const PackTask& tk = tasks[find_tile(&tasks[0].tile0, sizeof(PackTask) / 4, ntask, tile)];
  if (active && !active[tk.prob]) return;
  const int64_t f = (int64_t)(tile - tk.tile0) * 4 + (threadIdx.x >> 6);
  if (f >= (int64_t)tk.RB * tk.KB) return;
  const int lane = threadIdx.x & 63;
  const int r = (int)(f / tk.KB) * kFragRows + (lane & 15);
  const int k0 = (int)(f % tk.KB) * kFragK + 8 * (lane >> 4);
  const double* S = reinterpret_cast<const double*>(sbases[tk.prob * kNumBases + tk.sbase]) + tk.soff;
  uint32_t h[4], l[4];
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    uint32_t pr[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int k = k0 + e + u;
      double v = 0.0;
      if (r < tk.R && k < tk.K) v = tk.trans ? S[(int64_t)k * tk.ld + r] : S[(int64_t)r * tk.ld + k];
      pr[u] = split_bf16((float)v);
    }
    h[e / 2] = (pr[0] & 0xffffu) | (pr[1] << 16);
    l[e / 2] = (pr[0] >> 16) | (pr[1] & 0xffff0000u);
  }
  uint4* D = reinterpret_cast<uint4*>(reinterpret_cast<uint32_t*>(dbases[tk.prob * kNumBases + tk.dbase]) + tk.doff +
                                      f * kFragWords);
  D[lane] = make_uint4(h[0], h[1], h[2], h[3]);
  D[64 + lane] = make_uint4(l[0], l[1], l[2], l[3]);
}

__global__ __launch_bounds__(256) void scale_kernel(const ScaleTask* __restrict__ tasks, const int32_t* __restrict__ colmaps,
                                                    int ntask, double lam_floor, void* const* __restrict__ bases) {
  const int tile = blockIdx.x;
  const int ti = find_tile(&tasks[0].tile0, sizeof(ScaleTask) / 4, ntask, tile);
  const ScaleTask& tk = tasks[ti];
  const int local = tile - tk.tile0;
  const int r0 = (local / tk.tiles_c) * MR;
  const int c = (local % tk.tiles_c) * MC + (threadIdx.x & 63);
  if (c >= tk.cols) return;
  const double* S = reinterpret_cast<const double*>(bases[tk.prob * kNumBases + tk.sbase]) + tk.soff;
  double* D = reinterpret_cast<double*>(bases[tk.prob * kNumBases + tk.dbase]) + tk.doff;
  const int sc = tk.colmap >= 0 ? colmaps[tk.colmap + c] : c;
  double cs = 1.0;
  if (tk.cbase >= 0) cs = reinterpret_cast<const double*>(bases[tk.prob * kNumBases + tk.cbase])[tk.coff + c];
  const double* rs = tk.rbase >= 0 ? reinterpret_cast<const double*>(bases[tk.prob * kNumBases + tk.rbase]) + tk.roff
                                   : nullptr;
  for (int e = 0; e < 8; ++e) {
    const int r = r0 + (threadIdx.x >> 6) + 4 * e;
    if (r >= tk.rows) break;
    double f = cs;
    if (rs) {
      const double x = rs[r];
      f *= tk.invert_row ? (x > lam_floor ? 1.0 / x : 0.0) : x;
    }
    D[(int64_t)r * tk.ldd + c] = S[(int64_t)r * tk.lds + sc] * f;
  }
}

__global__ void convert_kernel(int kind, const void* __restrict__ src, void* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (kind == 0) {
      reinterpret_cast<float*>(dst)[i] = (float)reinterpret_cast<const double*>(src)[i];
    } else {
      reinterpret_cast<double*>(dst)[i] = (double)reinterpret_cast<const float*>(src)[i];
    }
  }
}

}  // namespace

void launch_mix(int tin, int tout, const MixTask* tasks, const MixSrc* srcs, int ntask, int ntiles,
                void* const* bases, const int32_t* active, hipStream_t s) {
  if (ntask == 0 || ntiles == 0) return;
  dim3 grid(ntiles), block(256);
  if (tin == 0 && tout == 0)
    hipLaunchKernelGGL((mix_kernel<double, double>), grid, block, 0, s, tasks, srcs, ntask, bases, active);
  else if (tin == 1 && tout == 1)
    hipLaunchKernelGGL((mix_kernel<float, float>), grid, block, 0, s, tasks, srcs, ntask, bases, active);
  else if (tin == 1 && tout == 3)
    hipLaunchKernelGGL((mix_kernel<float, FragOut>), grid, block, 0, s, tasks, srcs, ntask, bases, active);
  else if (tin == 0 && tout == 1)
    hipLaunchKernelGGL((mix_kernel<double, float>), grid, block, 0, s, tasks, srcs, ntask, bases, active);
}

void launch_pack(const PackTask* tasks, int ntask, int ntiles, void* const* sbases, void* const* dbases,
                 const int32_t* active, hipStream_t s) {
  if (ntask == 0 || ntiles == 0) return;
  hipLaunchKernelGGL(pack_kernel, dim3(ntiles), dim3(256), 0, s, tasks, ntask, sbases, dbases, active);
}

void launch_scale(const ScaleTask* tasks, const int32_t* colmaps, int ntask, int ntiles, double lam_floor,
                  void* const* bases, hipStream_t s) {
  if (ntask == 0 || ntiles == 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3(ntiles), dim3(256), 0, s, tasks, colmaps, ntask, lam_floor, bases);
}

void launch_convert(int kind, const void* src, void* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(convert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, kind, src, dst, n);
}

}  // namespace idmrg
