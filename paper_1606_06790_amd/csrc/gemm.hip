// Grouped GEMM on CDNA4 matrix cores (gfx950).
//
// One launch runs every task of a plan: the blocks of all l/2 superblocks and
// all symmetry sectors.  Each workgroup (256 threads = 4 wave64) owns one
// 64 x 64 output tile; the 4 waves form a 2 x 2 grid of 32 x 32 sub-tiles made
// of 2 x 2 MFMA 16 x 16 tiles.  K advances in steps of 16 through LDS.
//
// FP64 uses v_mfma_f64_16x16x4_f64, FP32 uses v_mfma_f32_16x16x4_f32 (both:
// A operand lane l holds A[l%16][l/16], B operand B[l/16][l%16], accumulator
// register r of lane l holds C[4*(l/16)+r][l%16] for FP32 and the bf16 shape,
// but C[l/16+4r][l%16] for FP64, as measured on gfx950).  The split-bf16 policy
// (bf16x3) uses v_mfma_f32_16x16x32_bf16 with operands a = hi + lo and three
// products hi*hi + hi*lo + lo*hi, FP32 accumulation.
#include "internal.h"

namespace idmrg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 16, LDS_LD = 65;

__device__ __forceinline__ int find_task(const GemmTask* tasks, int ntask, int tile) {
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ void mfma_16x16x4(T a, T b, typename std::conditional<std::is_same<T, double>::value, v4d, v4f>::type& c);

template <>
__device__ __forceinline__ void mfma_16x16x4<double>(double a, double b, v4d& c) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mfma_16x16x4<float>(float a, float b, v4f& c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// MODE: 0 = NN, 1 = NT (B given as [N x K]), 2 = TN (A given as [K x M]).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const GemmTask* __restrict__ tasks, int ntask,
                                                        void* const* __restrict__ bases,
                                                        const int32_t* __restrict__ active) {
  using acc_t = typename std::conditional<std::is_same<T, double>::value, v4d, v4f>::type;
  __shared__ T As[BK][LDS_LD];
  __shared__ T Bs[BK][LDS_LD];

  const int tile = blockIdx.x;
  const GemmTask& tk = tasks[find_task(tasks, ntask, tile)];
  if (active && !active[tk.prob]) return;
  const int local = tile - tk.tile0;
  const int m0 = (local / tk.tiles_n) * BM;
  const int n0 = (local % tk.tiles_n) * BN;
  const int M = tk.M, N = tk.N, K = tk.K;
  const T* __restrict__ A = reinterpret_cast<const T*>(bases[tk.prob * kNumBases + tk.abase]) + tk.aoff;
  const T* __restrict__ B = reinterpret_cast<const T*>(bases[tk.prob * kNumBases + tk.bbase]) + tk.boff;
  T* __restrict__ C = reinterpret_cast<T*>(bases[tk.prob * kNumBases + tk.cbase]) + tk.coff;
  const int lda = tk.lda, ldb = tk.ldb, ldc = tk.ldc;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

  acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += BK) {
    // ---- stage A tile [BM x BK] into As[k][m]
    if (MODE == 2) {
      const int k = t >> 4, mq = (t & 15) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = m0 + mq + e, gk = k0 + k;
        As[k][mq + e] = (gi < M && gk < K) ? A[(int64_t)gk * lda + gi] : T(0);
      }
    } else {
      const int i = t >> 2, kq = (t & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = m0 + i, gk = k0 + kq + e;
        As[kq + e][i] = (gi < M && gk < K) ? A[(int64_t)gi * lda + gk] : T(0);
      }
    }
    // ---- stage B tile [BK x BN] into Bs[k][n]
    if (MODE == 1) {
      const int n = t >> 2, kq = (t & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gn = n0 + n, gk = k0 + kq + e;
        Bs[kq + e][n] = (gn < N && gk < K) ? B[(int64_t)gn * ldb + gk] : T(0);
      }
    } else {
      const int k = t >> 4, nq = (t & 15) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gn = n0 + nq + e, gk = k0 + k;
        Bs[k][nq + e] = (gn < N && gk < K) ? B[(int64_t)gk * ldb + gn] : T(0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) mfma_16x16x4<T>(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }

  // ---- epilogue: C (+)= acc
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // FP64 16x16x4 keeps C[l/16 + 4r][l%16] in register r of lane l; FP32 keeps C[4(l/16) + r][l%16]
        const int gi = m0 + wm + i * 16 + (std::is_same<T, double>::value ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gi < M && gn < N) {
          T* p = C + (int64_t)gi * ldc + gn;
          *p = tk.beta ? (*p + acc[i][j][r]) : acc[i][j][r];
        }
      }
}

// ------------------------------------------------------------------ bf16x3
// Operands are packed pairs: the low 16 bits hold hi (bf16), the high 16 bits
// hold lo = bf16(x - hi).  K advances in steps of 32 (one MFMA 16x16x32).

constexpr int BK3 = 32, LDS3 = 33;

__device__ __forceinline__ uint32_t ld_pair(const uint32_t* p) { return *p; }

template <int MODE>
__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(const GemmTask* __restrict__ tasks, int ntask,
                                                          void* const* __restrict__ bases,
                                                          const int32_t* __restrict__ active) {
  // LDS tiles kept as [row][k] so that each lane reads 8 consecutive k values.
  __shared__ uint32_t As[BM][LDS3];
  __shared__ uint32_t Bs[BN][LDS3];

  const int tile = blockIdx.x;
  const GemmTask& tk = tasks[find_task(tasks, ntask, tile)];
  if (active && !active[tk.prob]) return;
  const int local = tile - tk.tile0;
  const int m0 = (local / tk.tiles_n) * BM;
  const int n0 = (local % tk.tiles_n) * BN;
  const int M = tk.M, N = tk.N, K = tk.K;
  const uint32_t* __restrict__ A =
      reinterpret_cast<const uint32_t*>(bases[tk.prob * kNumBases + tk.abase]) + tk.aoff;
  const uint32_t* __restrict__ B =
      reinterpret_cast<const uint32_t*>(bases[tk.prob * kNumBases + tk.bbase]) + tk.boff;
  float* __restrict__ C = reinterpret_cast<float*>(bases[tk.prob * kNumBases + tk.cbase]) + tk.coff;
  const int lda = tk.lda, ldb = tk.ldb, ldc = tk.ldc;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += BK3) {
    // A tile [64 x 32]: 2048 pairs, 8 per thread
    if (MODE == 2) {
      const int k = t >> 3, mq = (t & 7) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gi = m0 + mq + e, gk = k0 + k;
        As[mq + e][k] = (gi < M && gk < K) ? ld_pair(A + (int64_t)gk * lda + gi) : 0u;
      }
    } else {
      const int i = t >> 2, kq = (t & 3) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gi = m0 + i, gk = k0 + kq + e;
        As[i][kq + e] = (gi < M && gk < K) ? ld_pair(A + (int64_t)gi * lda + gk) : 0u;
      }
    }
    if (MODE == 1) {
      const int n = t >> 2, kq = (t & 3) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gn = n0 + n, gk = k0 + kq + e;
        Bs[n][kq + e] = (gn < N && gk < K) ? ld_pair(B + (int64_t)gn * ldb + gk) : 0u;
      }
    } else {
      const int k = t >> 3, nq = (t & 7) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gn = n0 + nq + e, gk = k0 + k;
        Bs[nq + e][k] = (gn < N && gk < K) ? ld_pair(B + (int64_t)gk * ldb + gn) : 0u;
      }
    }
    __syncthreads();
    const int kb = 8 * (lane >> 4);
    v8bf ahi[2], alo[2], bhi[2], blo[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint32_t* row = &As[wm + i * 16 + (lane & 15)][kb];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t pr = row[e];
        ahi[i][e] = __builtin_bit_cast(__bf16, (uint16_t)(pr & 0xffffu));
        alo[i][e] = __builtin_bit_cast(__bf16, (uint16_t)(pr >> 16));
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t* row = &Bs[wn + j * 16 + (lane & 15)][kb];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t pr = row[e];
        bhi[j][e] = __builtin_bit_cast(__bf16, (uint16_t)(pr & 0xffffu));
        blo[j][e] = __builtin_bit_cast(__bf16, (uint16_t)(pr >> 16));
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], bhi[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], blo[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], bhi[j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gi < M && gn < N) {
          float* p = C + (int64_t)gi * ldc + gn;
          *p = tk.beta ? (*p + acc[i][j][r]) : acc[i][j][r];
        }
      }
}

}  // namespace

void launch_gemm(Prec prec, int mode, const GemmTask* tasks, int ntask, int ntiles, void* const* bases,
                 const int32_t* active, hipStream_t s) {
  if (ntask == 0 || ntiles == 0) return;
  dim3 grid(ntiles), block(256);
  switch (prec) {
    case Prec::F64:
      if (mode == 0) hipLaunchKernelGGL((gemm_mfma_kernel<double, 0>), grid, block, 0, s, tasks, ntask, bases, active);
      else if (mode == 1) hipLaunchKernelGGL((gemm_mfma_kernel<double, 1>), grid, block, 0, s, tasks, ntask, bases, active);
      else hipLaunchKernelGGL((gemm_mfma_kernel<double, 2>), grid, block, 0, s, tasks, ntask, bases, active);
      break;
    case Prec::F32:
      if (mode == 0) hipLaunchKernelGGL((gemm_mfma_kernel<float, 0>), grid, block, 0, s, tasks, ntask, bases, active);
      else if (mode == 1) hipLaunchKernelGGL((gemm_mfma_kernel<float, 1>), grid, block, 0, s, tasks, ntask, bases, active);
      else hipLaunchKernelGGL((gemm_mfma_kernel<float, 2>), grid, block, 0, s, tasks, ntask, bases, active);
      break;
    case Prec::BF16X3:
      if (mode == 0) hipLaunchKernelGGL((gemm_bf16x3_kernel<0>), grid, block, 0, s, tasks, ntask, bases, active);
      else if (mode == 1) hipLaunchKernelGGL((gemm_bf16x3_kernel<1>), grid, block, 0, s, tasks, ntask, bases, active);
      else hipLaunchKernelGGL((gemm_bf16x3_kernel<2>), grid, block, 0, s, tasks, ntask, bases, active);
      break;
  }
}

}  // namespace idmrg
