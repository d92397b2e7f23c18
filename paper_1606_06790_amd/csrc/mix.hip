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
  TOUT* dst = reinterpret_cast<TOUT*>(bases[tk.prob * kNumBases + tk.dbase]) + tk.doff;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int r = rbase + 4 * e;
    if (r < tk.rows) dst[(int64_t)r * tk.ldd + c] = (TOUT)acc[e];
  }
}

// Word offset, inside its fragment matrix (kb k-fragments per row block), of
// the 8-value chunk of the hi plane that holds row r, columns k8 .. k8 + 7
// (k8 a multiple of 8); the lo plane's chunk is half a fragment further.
__device__ __forceinline__ int64_t frag_chunk(int r, int k8, int kb) {
  return ((int64_t)(r >> 4) * kb + (k8 >> 5)) * kFragWords + ((r & 15) + 16 * ((k8 & 31) >> 3)) * 4;
}

// Split-bf16 pairs of 8 consecutive values, as the hi and lo chunks of a fragment lane.
__device__ __forceinline__ void split8(const float (&v)[8], uint4& hi, uint4& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const uint32_t p0 = split_bf16(v[e]), p1 = split_bf16(v[e + 1]);
    h[e / 2] = (p0 & 0xffffu) | (p1 << 16);
    l[e / 2] = (p0 >> 16) | (p1 & 0xffff0000u);
  }
  hi = make_uint4(h[0], h[1], h[2], h[3]);
  lo = make_uint4(l[0], l[1], l[2], l[3]);
}

// The mixing of the fragment form: FP32 sources whose non-transposed rows start
// on 16-byte boundaries with lengths that are multiples of 4 (the padded T1 and
// x copies; checked on the host), output either plain FP32 (FRAG = false) or
// split-bf16 pairs in the fragment layout (FRAG = true, T3).  Same 32 x 64 tiles
// as mix_kernel; thread t takes columns 4 (t % 16) .. + 3 of rows t / 16 and
// t / 16 + 16, so 16 lanes read 256 contiguous bytes of a row per 16-byte load.
// In the fragment output a thread stores half a lane chunk (8 bytes of the hi
// plane, 8 of the lo plane); columns past the task's end within its 4 are
// zeros, and the other half of a chunk past the end keeps the zeros the buffer
// was cleared with.  Accumulation in double as in mix_kernel.
template <bool FRAG>
__global__ __launch_bounds__(256) void mix4_kernel(const MixTask* __restrict__ tasks, const MixSrc* __restrict__ srcs,
                                                   int ntask, void* const* __restrict__ bases,
                                                   const int32_t* __restrict__ active) {
  const int tile = blockIdx.x;
  const MixTask& tk = tasks[find_tile(&tasks[0].tile0, sizeof(MixTask) / 4, ntask, tile)];
  if (active && !active[tk.prob]) return;
  const int local = tile - tk.tile0;
  const int r0 = (local / tk.tiles_c) * MR + (threadIdx.x >> 4);
  const int c = (local % tk.tiles_c) * MC + 4 * (threadIdx.x & 15);
  if (c >= tk.cols) return;
  const int nc = min(4, tk.cols - c);
  double acc[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[h][e] = 0.0;
  for (int k = 0; k < tk.nsrc; ++k) {
    const MixSrc& s = srcs[tk.src0 + k];
    const float* S = reinterpret_cast<const float*>(bases[tk.prob * kNumBases + s.base]) + s.off;
    const double coef = s.coef;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = r0 + 16 * h;
      if (r >= tk.rows) continue;
      if (!s.trans) {
        // 16-byte aligned by the layout; the columns past nc are row padding or the
        // next columns of the same row, read but not used
        const float4 q = *reinterpret_cast<const float4*>(&S[(int64_t)r * s.ld + c]);
        const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[h][e] += coef * (double)qv[e];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (e < nc) acc[h][e] += coef * (double)S[(int64_t)(c + e) * s.ld + r];
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = r0 + 16 * h;
    if (r >= tk.rows) continue;
    if constexpr (FRAG) {
      uint32_t hw[2], lw[2];
#pragma unroll
      for (int e = 0; e < 4; e += 2) {
        const uint32_t p0 = split_bf16(e < nc ? (float)acc[h][e] : 0.f);
        const uint32_t p1 = split_bf16(e + 1 < nc ? (float)acc[h][e + 1] : 0.f);
        hw[e / 2] = (p0 & 0xffffu) | (p1 << 16);
        lw[e / 2] = (p0 >> 16) | (p1 & 0xffff0000u);
      }
      const int kk = tk.c0 + c;   // a multiple of 4: half (kk % 8) / 4 of a lane chunk
      uint32_t* D = reinterpret_cast<uint32_t*>(bases[tk.prob * kNumBases + tk.dbase]) + tk.doff +
                    frag_chunk(tk.r0 + r, kk & ~7, tk.ldd) + ((kk & 4) >> 1);
      *reinterpret_cast<uint2*>(D) = make_uint2(hw[0], hw[1]);
      *reinterpret_cast<uint2*>(D + kFragWords / 2) = make_uint2(lw[0], lw[1]);
    } else {
      float* D = reinterpret_cast<float*>(bases[tk.prob * kNumBases + tk.dbase]) + tk.doff + (int64_t)r * tk.ldd + c;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (e < nc) D[e] = (float)acc[h][e];
    }
  }
}

// One thread per row chunk: 8 consecutive columns of one row, stored as the
// 16-byte hi and lo chunks of one fragment lane.  Threads run over (row block,
// chunk, row % 16), so 16 consecutive threads write 256 contiguous bytes.
// Values outside [R x K] are zeros.
__global__ __launch_bounds__(256) void pack_kernel(const PackTask* __restrict__ tasks, int ntask,
                                                   void* const* __restrict__ sbases, void* const* __restrict__ dbases,
                                                   const double* __restrict__ sig,
                                                   const int32_t* __restrict__ active) {
  const int tile = blockIdx.x;
  const PackTask& tk = tasks[find_tile(&tasks[0].tile0, sizeof(PackTask) / 4, ntask, tile)];
  if (active && !active[tk.prob]) return;
  const int64_t i = (int64_t)(tile - tk.tile0) * 256 + threadIdx.x;
  if (i >= (int64_t)tk.RB * tk.nch * 16) return;
  const int rr = (int)(i & 15);
  const int64_t q = i >> 4;
  const int ch = (int)(q % tk.nch);
  const int r = (int)(q / tk.nch) * kFragRows + rr;
  const int k0 = 8 * ch;
  const double* S = reinterpret_cast<const double*>(sbases[tk.prob * kNumBases + tk.sbase]) + tk.soff;
  const double shift = tk.shift_slot >= 0 ? sig[tk.shift_slot] : 0.0;
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = k0 + e;
    double x = 0.0;
    if (r < tk.R && k < tk.K) {
      x = tk.trans ? S[(int64_t)k * tk.ld + r] : S[(int64_t)r * tk.ld + k];
      if (tk.xbase >= 0) {   // FP32 copy in the source's orientation
        float* X = reinterpret_cast<float*>(dbases[tk.prob * kNumBases + tk.xbase]) + tk.xoff;
        if (tk.trans) X[(int64_t)k * tk.xld + r] = (float)x;
        else X[(int64_t)r * tk.xld + k] = (float)x;
      }
    }
    if (r - tk.dr0 == k - tk.dk0 && (unsigned)(r - tk.dr0) < (unsigned)tk.dlen) x -= shift;
    v[e] = (float)x;
  }
  uint4 hi, lo;
  split8(v, hi, lo);
  uint4* D = reinterpret_cast<uint4*>(reinterpret_cast<uint32_t*>(dbases[tk.prob * kNumBases + tk.dbase]) + tk.doff +
                                      frag_chunk(r, tk.kc0 + k0, tk.KB));
  D[0] = hi;
  D[kFragWords / 8] = lo;
}

// Deterministic block sum (256 threads, fixed tree).
__device__ double block_sum256(double x, double* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// out[t] = sum of the diagonal of task t; one workgroup per task.
__global__ __launch_bounds__(256) void diag_sum_kernel(const DiagTask* __restrict__ tasks,
                                                       void* const* __restrict__ bases, double* __restrict__ out) {
  __shared__ double sh[256];
  const DiagTask tk = tasks[blockIdx.x];
  const double* S = reinterpret_cast<const double*>(bases[tk.prob * kNumBases + tk.base]) + tk.off;
  double a = 0.0;
  for (int i = threadIdx.x; i < tk.len; i += 256) a += S[(int64_t)i * (tk.ld + 1)];
  a = block_sum256(a, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = a;
}

// sig[2p + side] = mean diagonal element of problem p's tasks on that side (if flagged), summed in task
// order by one thread (the same order on every call); shift[t] = sig of task t.
__global__ void sigma_kernel(const DiagTask* __restrict__ tasks, int ntask, int nleft,
                             const double* __restrict__ sums, const int32_t* __restrict__ flags, int P,
                             double* __restrict__ sig, double* __restrict__ shift) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < 2 * P; ++q) {
    const int p = q >> 1, side = q & 1;
    double sum = 0.0, n = 0.0;
    for (int t = 0; t < ntask; ++t)
      if (tasks[t].prob == p && (t < nleft ? 0 : 1) == side) {
        sum += sums[t];
        n += tasks[t].len;
      }
    sig[q] = (flags[q] && n > 0.0) ? sum / n : 0.0;
  }
  for (int t = 0; t < ntask; ++t) shift[t] = sig[2 * tasks[t].prob + (t < nleft ? 0 : 1)];
}

// The diagonal of an FP32 copy rewritten from its FP64 source minus shift[t],
// rounded once: d32[i, i] = float(d64[i, i] - shift).
__global__ __launch_bounds__(256) void diag_shift_kernel(const DiagTask* __restrict__ tasks,
                                                         void* const* __restrict__ src,
                                                         void* const* __restrict__ dst,
                                                         const double* __restrict__ shift) {
  const DiagTask tk = tasks[blockIdx.x];
  const double* S = reinterpret_cast<const double*>(src[tk.prob * kNumBases + tk.base]) + tk.off;
  float* D = reinterpret_cast<float*>(dst[tk.prob * kNumBases + tk.base]) + tk.off;
  const double sg = shift[blockIdx.x];
  for (int i = threadIdx.x; i < tk.len; i += 256) {
    const int64_t e = (int64_t)i * (tk.ld + 1);
    D[e] = (float)(S[e] - sg);
  }
}

__global__ void convert_add_kernel(const float* __restrict__ src, const double* __restrict__ x,
                                   const double* __restrict__ sig, int prob, double* __restrict__ dst, int64_t n) {
  const double sigma = sig[2 * prob] + sig[2 * prob + 1];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i] + sigma * x[i];
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
  else if (tin == 4 && tout == 1)
    hipLaunchKernelGGL(mix4_kernel<false>, grid, block, 0, s, tasks, srcs, ntask, bases, active);
  else if (tin == 4 && tout == 3)
    hipLaunchKernelGGL(mix4_kernel<true>, grid, block, 0, s, tasks, srcs, ntask, bases, active);
  else if (tin == 0 && tout == 1)
    hipLaunchKernelGGL((mix_kernel<double, float>), grid, block, 0, s, tasks, srcs, ntask, bases, active);
}

__global__ __launch_bounds__(256) void overlap_seg_kernel(const OverlapSeg* __restrict__ segs,
                                                          void* const* __restrict__ bases,
                                                          double* __restrict__ partial) {
  __shared__ double sh[256];
  const OverlapSeg g = segs[blockIdx.x];
  const double* L = reinterpret_cast<const double*>(bases[g.item * kNumBases + 0]) + g.aoff;
  const double* R = reinterpret_cast<const double*>(bases[g.item * kNumBases + 1]) + g.boff;
  const int64_t n = (int64_t)g.rows * g.cols;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += 256) {
    const int64_t i = e / g.cols, j = e - i * g.cols;
    acc += L[i * g.lda + j] * R[i * g.ldb + j];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void overlap_sum_kernel(const int32_t* __restrict__ seg0, int nitem, const double* __restrict__ partial,
                                   double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nitem) return;
  double s = 0.0;
  for (int g = seg0[k]; g < seg0[k + 1]; ++g) s += partial[g];
  out[k] = s;
}

void launch_overlap(const OverlapSeg* segs, int nseg, const int32_t* seg0, int nitem, void* const* bases,
                    double* partial, double* out, hipStream_t s) {
  if (nseg > 0) hipLaunchKernelGGL(overlap_seg_kernel, dim3(nseg), dim3(256), 0, s, segs, bases, partial);
  hipLaunchKernelGGL(overlap_sum_kernel, dim3((nitem + 63) / 64), dim3(64), 0, s, seg0, nitem,
                     (const double*)partial, out);
}

void launch_diag_sum(const DiagTask* tasks, int ntask, void* const* bases, double* out, hipStream_t s) {
  if (ntask == 0) return;
  hipLaunchKernelGGL(diag_sum_kernel, dim3(ntask), dim3(256), 0, s, tasks, bases, out);
}

void launch_sigma(const DiagTask* tasks, int ntask, int nleft, const double* sums, const int32_t* flags, int P,
                  double* sig, double* shift, hipStream_t s) {
  hipLaunchKernelGGL(sigma_kernel, dim3(1), dim3(64), 0, s, tasks, ntask, nleft, sums, flags, P, sig, shift);
}

void launch_diag_shift_f32(const DiagTask* tasks, int ntask, void* const* src, void* const* dst, const double* shift,
                           hipStream_t s) {
  if (ntask == 0) return;
  hipLaunchKernelGGL(diag_shift_kernel, dim3(ntask), dim3(256), 0, s, tasks, src, dst, shift);
}

void launch_convert_add(const float* src, const double* x, const double* sig, int prob, double* dst, int64_t n,
                        hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(convert_add_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, x, sig, prob, dst, n);
}

void launch_pack(const PackTask* tasks, int ntask, int ntiles, void* const* sbases, void* const* dbases,
                 const double* sig, const int32_t* active, hipStream_t s) {
  if (ntask == 0 || ntiles == 0) return;
  hipLaunchKernelGGL(pack_kernel, dim3(ntiles), dim3(256), 0, s, tasks, ntask, sbases, dbases, sig, active);
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
