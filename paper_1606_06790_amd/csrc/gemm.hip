// Grouped GEMM on CDNA4 matrix cores (gfx950).
//
// One launch runs every task of a plan: the blocks of all l/2 superblocks and
// all symmetry sectors.  Each workgroup (256 threads = 4 wave64, 2 x 2) owns
// one BM x BN output tile.
//
// FP64 uses v_mfma_f64_16x16x4_f64 and FP32 v_mfma_f32_16x16x4_f32: the A
// operand of lane l is A[l%16][l/16], the B operand B[l/16][l%16]; register r
// of lane l holds C[4*(l/16)+r][l%16] for FP32 but C[l/16+4r][l%16] for FP64
// (measured on gfx950).  The split-bf16 policy (bf16x3) uses
// v_mfma_f32_16x16x32_bf16 (A: lane l holds A[l%16][8*(l/16)+0..7], B:
// B[8*(l/16)+0..7][l%16], C as FP32) with operands a = hi + lo and the three
// products lo*hi + hi*lo + hi*hi accumulated in FP32; its operands come
// pre-packed in that lane order (the fragment layout).
//
// Workgroups are dispatched round-robin over the 8 XCDs; xcd_tile() renumbers
// them so that each XCD receives a contiguous range of tiles, and the tiles of
// one output row band (which share their A operand) meet in one L2.
#include "internal.h"

namespace idmrg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;

// Logical tile of this workgroup (grid = kXcd * ceil(ntiles / kXcd)), or -1.
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int per = (ntiles + kXcd - 1) / kXcd;
  const int t = (int)(blockIdx.x % kXcd) * per + (int)(blockIdx.x / kXcd);
  return t < ntiles ? t : -1;
}

// Operands are read through global-address-space pointers (global_load, not
// flat_load) and out-of-range values are cleared with a bit mask instead of a
// select: the load then stays unconditional and the slab's loads are all in
// flight together (a select lets the compiler sink each load into its own
// branch and wait for it there).
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
  return (gptr<T>)(p);
}
// All-ones or zero, hidden from the optimiser (an empty register-only asm), so
// that `value & mask` is not rewritten into a select that the compiler turns
// into a branch around the load.
__device__ __forceinline__ uint32_t lane_mask(bool c) {
  uint32_t m = c ? 0xffffffffu : 0u;
  asm("" : "+v"(m));
  return m;
}
__device__ __forceinline__ uint32_t keep(uint32_t v, uint32_t m) { return v & m; }
__device__ __forceinline__ float keep(float v, uint32_t m) { return __uint_as_float(__float_as_uint(v) & m); }
__device__ __forceinline__ double keep(double v, uint32_t m) {
  return __longlong_as_double(__double_as_longlong(v) & (long long)(((uint64_t)m << 32) | m));
}

__device__ __forceinline__ int find_task(const GemmTask* tasks, int ntask, int tile) {
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
struct AccOf;
template <>
struct AccOf<double> { typedef v4d type; };
template <>
struct AccOf<float> { typedef v4f type; };

__device__ __forceinline__ void mfma_16x16x4(double a, double b, v4d& c) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ void mfma_16x16x4(float a, float b, v4f& c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Tile BM x BN per workgroup (2 x 2 waves of (BM/2) x (BN/2)), K in steps of
// 16.  The next K-slab is fetched from global memory into registers while the
// current one is consumed from LDS (two LDS buffers, one barrier per slab).
// MODE: 0 = NN, 1 = NT (B given as [N x K]), 2 = TN (A given as [K x M]).
template <typename T, int MODE, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const GemmTask* __restrict__ tasks, int ntask,
                                                        void* const* __restrict__ bases,
                                                        const int32_t* __restrict__ active, int ntiles) {
  using acc_t = typename AccOf<T>::type;
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2, TI = WM / 16, TJ = WN / 16;
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  __shared__ T As[2][BK][BM + 1];
  __shared__ T Bs[2][BK][BN + 1];

  const int tile = xcd_tile(ntiles);
  if (tile < 0) return;
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
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  // Slab element idx = e * 256 + t: consecutive threads take consecutive
  // memory addresses (16 threads per row of a K-contiguous operand, a whole
  // row of an M- or N-contiguous one), so every load instruction of a wave
  // covers whole cache lines.  Loads are unconditional: indices are clamped
  // into the matrix (offsets from the task base fit in 32 bits, checked on the
  // host).  Rows of A beyond M and columns of B beyond N only feed outputs that
  // are not stored; past K, A is cleared so those terms vanish (B there holds
  // clamped finite values).  For a K-contiguous operand the thread's rows are
  // fixed and its k is one per slab; for an M/N-contiguous one its column is
  // fixed and its rows of k vary with e.
  constexpr int AR = 256 / BK;    // rows (A, MODE 0/1) covered per e
  constexpr int AK = 256 / BM;    // k rows (A, MODE 2) covered per e
  constexpr int BR = 256 / BK;    // rows (B, MODE 1) per e
  constexpr int BKR = 256 / BN;   // k rows (B, MODE 0) per e
  int aoffs[NA], boffs[NB];
  int acol = 0, bcol = 0;
  if (MODE == 2) {
    const int gm = m0 + t % BM;
    acol = gm < M ? gm : M - 1;
  } else {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int gi = m0 + AR * e + t / BK;
      aoffs[e] = (gi < M ? gi : M - 1) * lda;
    }
  }
  if (MODE == 1) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int gn = n0 + BR * e + t / BK;
      boffs[e] = (gn < N ? gn : N - 1) * ldb;
    }
  } else {
    const int gn = n0 + t % BN;
    bcol = gn < N ? gn : N - 1;
  }
  T ra[NA], rb[NB];
  const gptr<T> Ag = as_global(A);
  const gptr<T> Bg = as_global(B);
  auto load = [&](int k0) {
    if (MODE == 2) {
#pragma unroll
      for (int e = 0; e < NA; ++e) {
        const int gk = k0 + AK * e + t / BM;
        ra[e] = keep(Ag[(gk < K ? gk : K - 1) * lda + acol], lane_mask(gk < K));
      }
    } else {
      const int gk = k0 + t % BK;
      const int ck = gk < K ? gk : K - 1;
      const uint32_t km = lane_mask(gk < K);
#pragma unroll
      for (int e = 0; e < NA; ++e) ra[e] = keep(Ag[aoffs[e] + ck], km);
    }
    if (MODE == 1) {
      const int gk = k0 + t % BK;
      const int ck = gk < K ? gk : K - 1;
#pragma unroll
      for (int e = 0; e < NB; ++e) rb[e] = Bg[boffs[e] + ck];
    } else {
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int gk = k0 + BKR * e + t / BN;
        rb[e] = Bg[(gk < K ? gk : K - 1) * ldb + bcol];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = e * 256 + t;
      if (MODE == 2) As[buf][idx / BM][idx % BM] = ra[e]; else As[buf][idx % BK][idx / BK] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = e * 256 + t;
      if (MODE == 1) Bs[buf][idx % BK][idx / BK] = rb[e]; else Bs[buf][idx / BN][idx % BN] = rb[e];
    }
  };

  acc_t acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  if (K > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int k0 = 0, it = 0; k0 < K; k0 += BK, ++it) {
    const int cur = it & 1;
    const bool more = k0 + BK < K;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T a[TI], b[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) a[i] = As[cur][kr][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TJ; ++j) b[j] = Bs[cur][kr][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) mfma_16x16x4(a[i], b[j], acc[i][j]);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm + i * 16 + (std::is_same<T, double>::value ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gi < M && gn < N) {
          T* p = C + (int64_t)gi * ldc + gn;
          *p = tk.beta ? (*p + acc[i][j][r]) : acc[i][j][r];
        }
      }
}

// ------------------------------------------------------------------ bf16x3
// Operands A[M x K] and B^T[N x K] are in the fragment layout (internal.h): a
// fragment is one MFMA operand of 16 rows x 32 k, its hi plane then its lo
// plane, 64 lanes x 16 bytes each, and the fragments of a row block are
// consecutive in k.  Tile BM x BN (64 or 128 each), K-slab 32, 2 x 2 waves of
// (BM/2) x (BN/2).  Per slab the workgroup copies BM/16 + BN/16 fragments
// straight from global memory into LDS (global_load_lds_dwordx4: 16 bytes per
// lane, lane l to LDS base + 16 l, so each wave copies 64 consecutive chunks
// of a fragment; the global offsets are fixed per thread and the slab moves a
// uniform base; rows past the operand repeat its last row block).  Each wave
// then reads its operands with conflict-free 16-byte LDS reads.  Zero padding
// of the layout makes the K tail exact.  Two LDS stages: the copy of slab k + 1
// is in flight while slab k is multiplied.  (A third stage does not pay: at
// 96 KB of LDS only one workgroup fits on a CU.)

// Byte address of an LDS location (the 32-bit offset ds_read takes).
__device__ __forceinline__ uint32_t lds_addr(const v4u* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) v4u*)(p);
}

// 16 bytes per lane from global memory straight to LDS: lane l writes dst + 16 l
// (dst must be the same for the whole wave).
__device__ __forceinline__ void lds_copy16(gptr<char> src, v4u* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// STAGE only names the call site (0: H_eff stage 1, 1: stage 2), so that
// profiles tell the two apart; the code is the same.
template <int STAGE, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(const GemmTask* __restrict__ tasks, int ntask,
                                                          void* const* __restrict__ bases,
                                                          const int32_t* __restrict__ active, int ntiles) {
  constexpr int FA = BM / 16, FB = BN / 16;    // fragments per slab
  constexpr int UA = FA / 2, UB = FB / 2;      // 16-byte copies per thread per slab (2 fragments per 256 threads)
  constexpr int TI = BM / 32, TJ = BN / 32;    // 16 x 16 MFMA tiles per wave
  constexpr uint32_t kFragBytes = kFragWords * 4;
  __shared__ v4u As[2][FA * 128], Bs[2][FB * 128];
  const int tile = xcd_tile(ntiles);
  if (tile < 0) return;
  const GemmTask& tk = tasks[find_task(tasks, ntask, tile)];
  if (active && !active[tk.prob]) return;
  const int local = tile - tk.tile0;
  const int m0 = (local / tk.tiles_n) * BM;
  const int n0 = (local % tk.tiles_n) * BN;
  const int M = tk.M, N = tk.N;
  const int KB = (tk.K + kFragK - 1) / kFragK;
  const int RA = (M + kFragRows - 1) / kFragRows, RB = (N + kFragRows - 1) / kFragRows;
  const char* A = reinterpret_cast<const char*>(bases[tk.prob * kNumBases + tk.abase]) + tk.aoff * 4;
  const char* B = reinterpret_cast<const char*>(bases[tk.prob * kNumBases + tk.bbase]) + tk.boff * 4;
  float* __restrict__ C = reinterpret_cast<float*>(bases[tk.prob * kNumBases + tk.cbase]) + tk.coff;
  const int ldc = tk.ldc;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // Copy u of thread t: fragment 2u + t/128 of the slab, chunk t % 128 of it
  // (byte offsets of slab 0: 32-bit, checked on the host).  LDS destination of
  // the wave: chunk 64 (wave % 2) of that fragment.
  const int half = t >> 7, within = t & 127;
  uint32_t ao[UA], bo[UB];
#pragma unroll
  for (int u = 0; u < UA; ++u) {
    const int rb = min(m0 / kFragRows + 2 * u + half, RA - 1);
    ao[u] = (uint32_t)rb * (uint32_t)KB * kFragBytes + within * 16u;
  }
#pragma unroll
  for (int u = 0; u < UB; ++u) {
    const int rb = min(n0 / kFragRows + 2 * u + half, RB - 1);
    bo[u] = (uint32_t)rb * (uint32_t)KB * kFragBytes + within * 16u;
  }
  const int wdst = half * 128 + (wave & 1) * 64;
  auto copy = [&](int kb, int st) {
    const gptr<char> Ak = as_global(A + (size_t)kb * kFragBytes);
    const gptr<char> Bk = as_global(B + (size_t)kb * kFragBytes);
#pragma unroll
    for (int u = 0; u < UA; ++u) lds_copy16(Ak + ao[u], &As[st][u * 256 + wdst]);
#pragma unroll
    for (int u = 0; u < UB; ++u) lds_copy16(Bk + bo[u], &Bs[st][u * 256 + wdst]);
  };

  v4f acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = v4f{0, 0, 0, 0};

  if (KB > 0) copy(0, 0);
  for (int kb = 0; kb < KB; ++kb) {
    const int cur = kb & 1;
    // this slab's copy has landed in every wave; the other stage is free
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    v8bf ah[TI], al[TI], bh[TJ], bl[TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const int f = wr * TI + i;
      ah[i] = __builtin_bit_cast(v8bf, As[cur][f * 128 + lane]);
      al[i] = __builtin_bit_cast(v8bf, As[cur][f * 128 + 64 + lane]);
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int f = wc * TJ + j;
      bh[j] = __builtin_bit_cast(v8bf, Bs[cur][f * 128 + lane]);
      bl[j] = __builtin_bit_cast(v8bf, Bs[cur][f * 128 + 64 + lane]);
    }
    // The next slab's copy goes out after this slab's LDS reads: the compiler
    // makes an LDS read that follows an LDS copy wait for it, and the reads are
    // what the MFMAs wait on.  It lands during the MFMAs.
    if (kb + 1 < KB) copy(kb + 1, cur ^ 1);
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wr * (BM / 2) + i * 16 + 4 * (lane >> 4) + r;
        const int gn = n0 + wc * (BN / 2) + j * 16 + (lane & 15);
        if (gi < M && gn < N) {
          float* p = C + (int64_t)gi * ldc + gn;
          *p = tk.beta ? (*p + acc[i][j][r]) : acc[i][j][r];
        }
      }
}

// The same product with a 256 x 128 tile: 8 waves (4 x 2) of 64 x 64 (the
// same register footprint per wave as the 128 x 128 tile, so still two waves
// per SIMD), three LDS stages of 48 KB (144 KB, one workgroup per CU), and the
// copies of each slab issued two slabs ahead, so that a copy has two slabs of
// MFMA work (~1500 cycles per SIMD) to land instead of one.  Slab k + 2 goes
// into the stage that slab k - 1 used; the barrier at the top of slab k, after
// each thread has waited for its own copies of slab k, makes every copy of
// slab k visible and ends every read of slab k - 1.  The barrier carries no
// memory fence (a fence would wait for the copies in flight as well).
template <int STAGE>
__global__ __launch_bounds__(512) void gemm_bf16x3_w8_kernel(const GemmTask* __restrict__ tasks, int ntask,
                                                             void* const* __restrict__ bases,
                                                             const int32_t* __restrict__ active, int ntiles) {
  constexpr int BM = 256, BN = 128, NS = 3;
  constexpr int FA = BM / 16, FB = BN / 16;    // fragments per slab
  constexpr int UA = FA / 4, UB = FB / 4;      // 16-byte copies per thread per slab (4 fragments per 512 threads)
  constexpr int NCOPY = UA + UB;
  constexpr int TI = 4, TJ = 4;                // 16 x 16 MFMA tiles per wave
  constexpr uint32_t kFragBytes = kFragWords * 4;
  __shared__ v4u As[NS][FA * 128], Bs[NS][FB * 128];
  const int tile = xcd_tile(ntiles);
  if (tile < 0) return;
  const GemmTask& tk = tasks[find_task(tasks, ntask, tile)];
  if (active && !active[tk.prob]) return;
  const int local = tile - tk.tile0;
  const int m0 = (local / tk.tiles_n) * BM;
  const int n0 = (local % tk.tiles_n) * BN;
  const int M = tk.M, N = tk.N;
  const int KB = (tk.K + kFragK - 1) / kFragK;
  const int RA = (M + kFragRows - 1) / kFragRows, RB = (N + kFragRows - 1) / kFragRows;
  const char* A = reinterpret_cast<const char*>(bases[tk.prob * kNumBases + tk.abase]) + tk.aoff * 4;
  const char* B = reinterpret_cast<const char*>(bases[tk.prob * kNumBases + tk.bbase]) + tk.boff * 4;
  float* __restrict__ C = reinterpret_cast<float*>(bases[tk.prob * kNumBases + tk.cbase]) + tk.coff;
  const int ldc = tk.ldc;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // Copy u of thread t: fragment 4u + t/128 of the slab, chunk t % 128 of it; the
  // LDS destination of the wave is chunk 64 (wave % 2) of that fragment.
  const int quarter = t >> 7, within = t & 127;
  uint32_t ao[UA], bo[UB];
#pragma unroll
  for (int u = 0; u < UA; ++u) {
    const int rb = min(m0 / kFragRows + 4 * u + quarter, RA - 1);
    ao[u] = (uint32_t)rb * (uint32_t)KB * kFragBytes + within * 16u;
  }
#pragma unroll
  for (int u = 0; u < UB; ++u) {
    const int rb = min(n0 / kFragRows + 4 * u + quarter, RB - 1);
    bo[u] = (uint32_t)rb * (uint32_t)KB * kFragBytes + within * 16u;
  }
  const int wdst = quarter * 128 + (wave & 1) * 64;
  auto copy = [&](int kb, int st) {
    const gptr<char> Ak = as_global(A + (size_t)kb * kFragBytes);
    const gptr<char> Bk = as_global(B + (size_t)kb * kFragBytes);
#pragma unroll
    for (int u = 0; u < UA; ++u) lds_copy16(Ak + ao[u], &As[st][u * 512 + wdst]);
#pragma unroll
    for (int u = 0; u < UB; ++u) lds_copy16(Bk + bo[u], &Bs[st][u * 512 + wdst]);
  };

  v4f acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = v4f{0, 0, 0, 0};

  if (KB > 0) copy(0, 0);
  if (KB > 1) copy(1, 1);
  int cur = 0;
  for (int kb = 0; kb < KB; ++kb) {
    // this thread's copies of slab kb have landed (those of slab kb + 1 may still be in flight)
    if (kb + 1 < KB)
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"(NCOPY) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    if (kb + 2 < KB) copy(kb + 2, cur == 0 ? 2 : cur - 1);
    // The wave's 16 operand reads in one asm block that ends with their own
    // wait: the compiler would otherwise make an LDS read that follows the
    // copies wait for all of them (it cannot tell that they write other
    // stages), which is the one-slab pipeline again.  Outputs are early-clobber,
    // so no read lands in an address register that a later read still needs.
    const uint32_t abase = lds_addr(&As[cur][wr * TI * 128 + lane]);
    const uint32_t bbase = lds_addr(&Bs[cur][wc * TJ * 128 + lane]);
    v4u r[16];
    asm volatile(
        "ds_read_b128 %0, %16 offset:0\n\t"
        "ds_read_b128 %1, %16 offset:1024\n\t"
        "ds_read_b128 %2, %16 offset:2048\n\t"
        "ds_read_b128 %3, %16 offset:3072\n\t"
        "ds_read_b128 %4, %16 offset:4096\n\t"
        "ds_read_b128 %5, %16 offset:5120\n\t"
        "ds_read_b128 %6, %16 offset:6144\n\t"
        "ds_read_b128 %7, %16 offset:7168\n\t"
        "ds_read_b128 %8, %17 offset:0\n\t"
        "ds_read_b128 %9, %17 offset:1024\n\t"
        "ds_read_b128 %10, %17 offset:2048\n\t"
        "ds_read_b128 %11, %17 offset:3072\n\t"
        "ds_read_b128 %12, %17 offset:4096\n\t"
        "ds_read_b128 %13, %17 offset:5120\n\t"
        "ds_read_b128 %14, %17 offset:6144\n\t"
        "ds_read_b128 %15, %17 offset:7168\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]),
          "=&v"(r[7]), "=&v"(r[8]), "=&v"(r[9]), "=&v"(r[10]), "=&v"(r[11]), "=&v"(r[12]), "=&v"(r[13]),
          "=&v"(r[14]), "=&v"(r[15])
        : "v"(abase), "v"(bbase)
        : "memory");
    v8bf ah[TI], al[TI], bh[TJ], bl[TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      ah[i] = __builtin_bit_cast(v8bf, r[2 * i]);
      al[i] = __builtin_bit_cast(v8bf, r[2 * i + 1]);
      bh[i] = __builtin_bit_cast(v8bf, r[8 + 2 * i]);
      bl[i] = __builtin_bit_cast(v8bf, r[8 + 2 * i + 1]);
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    cur = cur == NS - 1 ? 0 : cur + 1;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wr * 64 + i * 16 + 4 * (lane >> 4) + r;
        const int gn = n0 + wc * 64 + j * 16 + (lane & 15);
        if (gi < M && gn < N) {
          float* p = C + (int64_t)gi * ldc + gn;
          *p = tk.beta ? (*p + acc[i][j][r]) : acc[i][j][r];
        }
      }
}

}  // namespace

template <typename T, int BM, int BN>
static void launch_tile(int mode, dim3 grid, hipStream_t s, const GemmTask* tasks, int ntask, void* const* bases,
                        const int32_t* active, int ntiles) {
  if (mode == 0)
    hipLaunchKernelGGL((gemm_mfma_kernel<T, 0, BM, BN>), grid, dim3(256), 0, s, tasks, ntask, bases, active, ntiles);
  else if (mode == 1)
    hipLaunchKernelGGL((gemm_mfma_kernel<T, 1, BM, BN>), grid, dim3(256), 0, s, tasks, ntask, bases, active, ntiles);
  else
    hipLaunchKernelGGL((gemm_mfma_kernel<T, 2, BM, BN>), grid, dim3(256), 0, s, tasks, ntask, bases, active, ntiles);
}

template <typename T>
static void launch_t(int tiling, int mode, dim3 grid, hipStream_t s, const GemmTask* tasks, int ntask,
                     void* const* bases, const int32_t* active, int ntiles) {
  switch (tiling) {
    case 1: launch_tile<T, 128, 64>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case 2: launch_tile<T, 64, 128>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case 3: launch_tile<T, 128, 128>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    default: launch_tile<T, 64, 64>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
  }
}

template <int BM, int BN>
static void launch_b3(int mode, dim3 grid, hipStream_t s, const GemmTask* tasks, int ntask, void* const* bases,
                      const int32_t* active, int ntiles) {
  if (mode == 0)
    hipLaunchKernelGGL((gemm_bf16x3_kernel<0, BM, BN>), grid, dim3(256), 0, s, tasks, ntask, bases, active, ntiles);
  else
    hipLaunchKernelGGL((gemm_bf16x3_kernel<1, BM, BN>), grid, dim3(256), 0, s, tasks, ntask, bases, active, ntiles);
}

static void launch_bf16x3(int tiling, int mode, dim3 grid, hipStream_t s, const GemmTask* tasks, int ntask,
                          void* const* bases, const int32_t* active, int ntiles) {
  if (tiling == 4) {   // 256 x 128, eight waves, three stages
    if (mode == 0)
      hipLaunchKernelGGL(gemm_bf16x3_w8_kernel<0>, grid, dim3(512), 0, s, tasks, ntask, bases, active, ntiles);
    else
      hipLaunchKernelGGL(gemm_bf16x3_w8_kernel<1>, grid, dim3(512), 0, s, tasks, ntask, bases, active, ntiles);
    return;
  }
  switch (tiling) {
    case 0: launch_b3<64, 64>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case 1: launch_b3<128, 64>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case 2: launch_b3<64, 128>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    default: launch_b3<128, 128>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
  }
}

void launch_gemm(Prec prec, int mode, const GemmTask* tasks, int ntask, int ntiles, void* const* bases,
                 const int32_t* active, hipStream_t s, int tiling) {
  if (ntask == 0 || ntiles == 0) return;
  dim3 grid(kXcd * ((ntiles + kXcd - 1) / kXcd)), block(256);
  switch (prec) {
    case Prec::F64: launch_t<double>(tiling, mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case Prec::F32: launch_t<float>(tiling, mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case Prec::BF16X3: launch_bf16x3(tiling, mode, grid, s, tasks, ntask, bases, active, ntiles); break;
  }
}

}  // namespace idmrg
