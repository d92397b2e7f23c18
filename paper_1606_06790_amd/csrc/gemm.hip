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
// one output row band (which share their A operand) meet in one L2.  The
// ranges, stored after the task table, split the tiles at equal estimated work
// (K + 64 per tile), so that no XCD gets more than its share of long-K tasks.
#include "internal.h"

namespace idmrg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;

static_assert(kXcd + 1 == kXcdRanges, "one range per XCD");

// Logical tile of this workgroup (grid = kXcd * the largest range), or -1.
__device__ __forceinline__ int xcd_tile(const GemmTask* tasks, int ntask) {
  const int32_t* xr = reinterpret_cast<const int32_t*>(tasks + ntask);
  const int x = (int)(blockIdx.x % kXcd);
  const int t = xr[x] + (int)(blockIdx.x / kXcd);
  return t < xr[x + 1] ? t : -1;
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

  const int tile = xcd_tile(tasks, ntask);
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
  const int tile = xcd_tile(tasks, ntask);
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

// The 128 x 128 tile as a persistent kernel: kPersistPerCu workgroups per CU,
// each going through a fixed sequence of tiles of its XCD's range, with the
// copy pipeline running on across tile boundaries.  The first slab of the next
// tile is copied while the last slab of the current one is multiplied, and its
// result is stored while that copy is in flight, so a tile costs no pipeline
// fill (with K of a few hundred, one fill is a sizeable part of a tile).
// Within a tile everything is as in gemm_bf16x3_kernel<STAGE, 128, 128>: the
// same slabs, fragments, MFMA order and stores, so the results are identical.
constexpr int kPersistPerCu = 2, kCus = 256;

// Plan tables read through the constant address space with wave-uniform
// indices become scalar loads: they then wait on lgkmcnt, not on vmcnt, so
// looking up the next tile does not wait for the copies in flight.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}
__device__ __forceinline__ int find_task_c(cptr<GemmTask> tasks, int ntask, int tile) {
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int STAGE>
__global__ __launch_bounds__(256) void gemm_bf16x3_persist_kernel(const GemmTask* __restrict__ tasks_, int ntask,
                                                                  void* const* __restrict__ bases_,
                                                                  const int32_t* __restrict__ active_, int ntiles) {
  constexpr int BM = 128, BN = 128;
  constexpr int FA = BM / 16, FB = BN / 16;
  constexpr int UA = FA / 2, UB = FB / 2;
  constexpr int TI = BM / 32, TJ = BN / 32;
  constexpr uint32_t kFragBytes = kFragWords * 4;
  __shared__ v4u As[2][FA * 128], Bs[2][FB * 128];
  const cptr<GemmTask> tasks = as_const(tasks_);
  const cptr<void*> bases = as_const(bases_);
  const cptr<int32_t> active = active_ ? as_const(active_) : nullptr;
  // this workgroup's tiles: start, start + step, ... below t1 (workgroups go round-robin over the XCDs)
  const int G = (int)gridDim.x, xcd = (int)(blockIdx.x % kXcd), slot = (int)(blockIdx.x / kXcd);
  const cptr<int32_t> xr = as_const(reinterpret_cast<const int32_t*>(tasks_ + ntask));
  const int t0 = xr[xcd], t1 = xr[xcd + 1], step = G / kXcd;
  // a tile's task, looked up once when the copy cursor reaches the tile
  struct Tile {
    int t, kb, m0, n0, M, N, K, ldc, beta;
    int64_t coff;
    const char *A, *B;
    float* C;
  };
  // next tile at or after t of this workgroup whose problem is active, with its task (t = t1: none left)
  auto fetch = [&](int t, Tile& x) {
    for (; t < t1; t += step) {
      const int ti = __builtin_amdgcn_readfirstlane(find_task_c(tasks, ntask, t));
      const int prob = tasks[ti].prob;
      if (active && !active[prob]) continue;
      const int local = t - tasks[ti].tile0, tiles_n = tasks[ti].tiles_n;
      x.t = t;
      x.m0 = (local / tiles_n) * BM;
      x.n0 = (local % tiles_n) * BN;
      x.M = tasks[ti].M; x.N = tasks[ti].N; x.K = tasks[ti].K; x.ldc = tasks[ti].ldc; x.beta = tasks[ti].beta;
      x.kb = (x.K + kFragK - 1) / kFragK;
      x.A = reinterpret_cast<const char*>(bases[prob * kNumBases + tasks[ti].abase]) + tasks[ti].aoff * 4;
      x.B = reinterpret_cast<const char*>(bases[prob * kNumBases + tasks[ti].bbase]) + tasks[ti].boff * 4;
      x.C = reinterpret_cast<float*>(bases[prob * kNumBases + tasks[ti].cbase]) + tasks[ti].coff;
      return;
    }
    x.t = t1;
  };
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = t >> 7, within = t & 127;
  const int wdst = half * 128 + (wave & 1) * 64;

  v4f acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = v4f{0, 0, 0, 0};
  // store the accumulators as tile x (and clear them)
  auto store_tile = [&](const Tile& x) {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = x.m0 + wr * (BM / 2) + i * 16 + 4 * (lane >> 4) + r;
          const int gn = x.n0 + wc * (BN / 2) + j * 16 + (lane & 15);
          if (gi < x.M && gn < x.N) {
            float* p = x.C + (int64_t)gi * x.ldc + gn;
            *p = x.beta ? (*p + acc[i][j][r]) : acc[i][j][r];
          }
        }
        acc[i][j] = v4f{0, 0, 0, 0};
      }
  };
  // the result of a tile with K = 0: zero (or C unchanged where the task accumulates)
  auto zero_tile = [&](const Tile& x) {
    if (x.beta) return;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = x.m0 + wr * (BM / 2) + i * 16 + 4 * (lane >> 4) + r;
          const int gn = x.n0 + wc * (BN / 2) + j * 16 + (lane & 15);
          if (gi < x.M && gn < x.N) x.C[(int64_t)gi * x.ldc + gn] = 0.f;
        }
  };
  // next tile with slabs at or after t (the copy cursor passes over tiles with K = 0; the multiplying side
  // gives them their result)
  auto next_copy_tile = [&](int t, Tile& x) {
    for (fetch(t, x); x.t < t1 && x.kb == 0; fetch(x.t + step, x)) {
    }
  };
  auto next_mul_tile = [&](int t, Tile& x) {
    for (fetch(t, x); x.t < t1 && x.kb == 0; fetch(x.t + step, x)) zero_tile(x);
  };

  // copy cursor: tile cx, slab kc
  Tile cx, mx;
  int kc = 0;
  uint32_t ao[UA], bo[UB];
  auto set_offsets = [&]() {
    const int RA = (cx.M + kFragRows - 1) / kFragRows, RB = (cx.N + kFragRows - 1) / kFragRows;
#pragma unroll
    for (int u = 0; u < UA; ++u)
      ao[u] = (uint32_t)min(cx.m0 / kFragRows + 2 * u + half, RA - 1) * (uint32_t)cx.kb * kFragBytes + within * 16u;
#pragma unroll
    for (int u = 0; u < UB; ++u)
      bo[u] = (uint32_t)min(cx.n0 / kFragRows + 2 * u + half, RB - 1) * (uint32_t)cx.kb * kFragBytes + within * 16u;
  };
  // issue the copy at the cursor into stage st and advance the cursor
  auto copy_next = [&](int st) {
    const gptr<char> Ak = as_global(cx.A + (size_t)kc * kFragBytes);
    const gptr<char> Bk = as_global(cx.B + (size_t)kc * kFragBytes);
#pragma unroll
    for (int u = 0; u < UA; ++u) lds_copy16(Ak + ao[u], &As[st][u * 256 + wdst]);
#pragma unroll
    for (int u = 0; u < UB; ++u) lds_copy16(Bk + bo[u], &Bs[st][u * 256 + wdst]);
    if (++kc == cx.kb) {
      kc = 0;
      next_copy_tile(cx.t + step, cx);
      if (cx.t < t1) set_offsets();
    }
  };

  next_mul_tile(t0 + slot, mx);   // the tile being multiplied, at slab km
  if (mx.t >= t1) return;
  cx = mx;
  set_offsets();
  copy_next(0);
  int cur = 0;
  for (;;) {
    for (int km = 0; km < mx.kb; ++km, cur ^= 1) {
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
      if (cx.t < t1) copy_next(cur ^ 1);
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    // the tile is done: store it while the next tile's first slab is in flight
    store_tile(mx);
    next_mul_tile(mx.t + step, mx);
    if (mx.t >= t1) break;
  }
}

// The 256 x 128 eight-wave tile with its operand reads software-pipelined:
// while the MFMAs of slab k run from one register set, the wave reads slab
// k + 1 from LDS into the other, and the copies of slab k + 3 are in flight
// into the third LDS stage.  So a wave does not wait for LDS data before its
// MFMAs, and a copy has two slabs of MFMA work to land.  Step k:
//   * wait for this thread's copies of slab k + 1 (those of k + 2 may still
//     be in flight); barrier: every copy of slab k + 1 is visible, and every
//     wave has finished reading slab k's stage (in step k - 1);
//   * copy slab k + 3 into slab k's stage;
//   * one asm block: the 16 reads of slab k + 1 interleaved with the 48 MFMAs
//     of slab k (one read per three MFMAs), then a wait for the reads.
// The reads and MFMAs are written out in asm because the compiler treats every
// LDS read that follows an LDS copy as dependent on it, whichever stage it
// writes, and would wait for all copies in flight before the first read.  The
// block waits for its own reads before it ends, so no read is in flight outside
// it.  The MFMAs of one block go over the 16 tiles of the wave in three passes
// (lo*hi, hi*lo, hi*hi), so two MFMAs on one accumulator are 16 apart.  The
// s_nop at the start of each block and after the loop give the wait states
// between these MFMAs and the vector instructions around them.  The read after
// the last slab takes a stale stage into registers that nothing uses.
template <int STAGE>
__global__ __launch_bounds__(512) void gemm_bf16x3_pipe_kernel(const GemmTask* __restrict__ tasks, int ntask,
                                                               void* const* __restrict__ bases,
                                                               const int32_t* __restrict__ active, int ntiles) {
  constexpr int BM = 256, BN = 128, NS = 3;
  constexpr int FA = BM / 16, FB = BN / 16;    // fragments per slab
  constexpr int UA = FA / 4, UB = FB / 4;      // 16-byte copies per thread per slab
  constexpr int NCOPY = UA + UB;
  constexpr int TI = 4, TJ = 4;                // 16 x 16 MFMA tiles per wave (64 x 64)
  constexpr uint32_t kFragBytes = kFragWords * 4;
  __shared__ v4u As[NS][FA * 128], Bs[NS][FB * 128];
  const int tile = xcd_tile(tasks, ntask);
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

  // Copy u of thread t: fragment 4u + t/128 of the slab, chunk t % 128 of it;
  // the LDS destination of the wave is chunk 64 (wave % 2) of that fragment.
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
  // LDS byte addresses of this wave's operands in stage st
  auto a_at = [&](int st) { return lds_addr(&As[st][wr * TI * 128 + lane]); };
  auto b_at = [&](int st) { return lds_addr(&Bs[st][wc * TJ * 128 + lane]); };

  v4f acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = v4f{0, 0, 0, 0};
  v4u F0[16], F1[16];

  if (KB > 0) copy(0, 0);
  if (KB > 1) copy(1, 1);
  if (KB > 2) copy(2, 2);
  if (KB > 2)
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * NCOPY) : "memory");
  else if (KB > 1)
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(NCOPY) : "memory");
  else
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  {
    const uint32_t abase = a_at(0), bbase = b_at(0);
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
        : "=&v"(F0[0]), "=&v"(F0[1]), "=&v"(F0[2]), "=&v"(F0[3]), "=&v"(F0[4]), "=&v"(F0[5]), "=&v"(F0[6]),
          "=&v"(F0[7]), "=&v"(F0[8]), "=&v"(F0[9]), "=&v"(F0[10]), "=&v"(F0[11]), "=&v"(F0[12]),
          "=&v"(F0[13]), "=&v"(F0[14]), "=&v"(F0[15])
        : "v"(abase), "v"(bbase)
        : "memory");
  }

  // One step k: FC holds slab k, FN receives slab k + 1.
#define IDMRG_PIPE_STEP(k, FC, FN)                                                                     \
  do {                                                                                                 \
    if ((k) + 2 < KB)                                                                                  \
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"(NCOPY) : "memory");                                     \
    else                                                                                               \
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");                                                 \
    __builtin_amdgcn_s_barrier();                                                                      \
    const int st = (k) % NS;                                                                           \
    if ((k) + 3 < KB) copy((k) + 3, st);                                                               \
    const int nx = st == NS - 1 ? 0 : st + 1;                                                          \
    const uint32_t abase = a_at(nx), bbase = b_at(nx);                                                 \
    asm volatile(                                                                                      \
IDMRG_PIPE_ASM                                                                                         \
        : "=&v"(FN[0]), "=&v"(FN[1]), "=&v"(FN[2]), "=&v"(FN[3]), "=&v"(FN[4]), "=&v"(FN[5]),          \
          "=&v"(FN[6]), "=&v"(FN[7]), "=&v"(FN[8]), "=&v"(FN[9]), "=&v"(FN[10]), "=&v"(FN[11]),        \
          "=&v"(FN[12]), "=&v"(FN[13]), "=&v"(FN[14]), "=&v"(FN[15]),                                  \
          "+v"(acc[0][0]), "+v"(acc[0][1]), "+v"(acc[0][2]), "+v"(acc[0][3]), "+v"(acc[1][0]),         \
          "+v"(acc[1][1]), "+v"(acc[1][2]), "+v"(acc[1][3]), "+v"(acc[2][0]), "+v"(acc[2][1]),         \
          "+v"(acc[2][2]), "+v"(acc[2][3]), "+v"(acc[3][0]), "+v"(acc[3][1]), "+v"(acc[3][2]),         \
          "+v"(acc[3][3])                                                                              \
        : "v"(FC[0]), "v"(FC[1]), "v"(FC[2]), "v"(FC[3]), "v"(FC[4]), "v"(FC[5]), "v"(FC[6]),          \
          "v"(FC[7]), "v"(FC[8]), "v"(FC[9]), "v"(FC[10]), "v"(FC[11]), "v"(FC[12]), "v"(FC[13]),      \
          "v"(FC[14]), "v"(FC[15]), "v"(abase), "v"(bbase)                                             \
        : "memory");                                                                                   \
  } while (0)
#define IDMRG_PIPE_ASM \
      "s_nop 2\n\t" \
      "ds_read_b128 %0, %48 offset:0\n\t" \
      "v_mfma_f32_16x16x32_bf16 %16, %33, %40, %16\n\t" \
      "v_mfma_f32_16x16x32_bf16 %17, %33, %42, %17\n\t" \
      "v_mfma_f32_16x16x32_bf16 %18, %33, %44, %18\n\t" \
      "ds_read_b128 %1, %48 offset:1024\n\t" \
      "v_mfma_f32_16x16x32_bf16 %19, %33, %46, %19\n\t" \
      "v_mfma_f32_16x16x32_bf16 %20, %35, %40, %20\n\t" \
      "v_mfma_f32_16x16x32_bf16 %21, %35, %42, %21\n\t" \
      "ds_read_b128 %8, %49 offset:0\n\t" \
      "v_mfma_f32_16x16x32_bf16 %22, %35, %44, %22\n\t" \
      "v_mfma_f32_16x16x32_bf16 %23, %35, %46, %23\n\t" \
      "v_mfma_f32_16x16x32_bf16 %24, %37, %40, %24\n\t" \
      "ds_read_b128 %9, %49 offset:1024\n\t" \
      "v_mfma_f32_16x16x32_bf16 %25, %37, %42, %25\n\t" \
      "v_mfma_f32_16x16x32_bf16 %26, %37, %44, %26\n\t" \
      "v_mfma_f32_16x16x32_bf16 %27, %37, %46, %27\n\t" \
      "ds_read_b128 %2, %48 offset:2048\n\t" \
      "v_mfma_f32_16x16x32_bf16 %28, %39, %40, %28\n\t" \
      "v_mfma_f32_16x16x32_bf16 %29, %39, %42, %29\n\t" \
      "v_mfma_f32_16x16x32_bf16 %30, %39, %44, %30\n\t" \
      "ds_read_b128 %3, %48 offset:3072\n\t" \
      "v_mfma_f32_16x16x32_bf16 %31, %39, %46, %31\n\t" \
      "v_mfma_f32_16x16x32_bf16 %16, %32, %41, %16\n\t" \
      "v_mfma_f32_16x16x32_bf16 %17, %32, %43, %17\n\t" \
      "ds_read_b128 %10, %49 offset:2048\n\t" \
      "v_mfma_f32_16x16x32_bf16 %18, %32, %45, %18\n\t" \
      "v_mfma_f32_16x16x32_bf16 %19, %32, %47, %19\n\t" \
      "v_mfma_f32_16x16x32_bf16 %20, %34, %41, %20\n\t" \
      "ds_read_b128 %11, %49 offset:3072\n\t" \
      "v_mfma_f32_16x16x32_bf16 %21, %34, %43, %21\n\t" \
      "v_mfma_f32_16x16x32_bf16 %22, %34, %45, %22\n\t" \
      "v_mfma_f32_16x16x32_bf16 %23, %34, %47, %23\n\t" \
      "ds_read_b128 %4, %48 offset:4096\n\t" \
      "v_mfma_f32_16x16x32_bf16 %24, %36, %41, %24\n\t" \
      "v_mfma_f32_16x16x32_bf16 %25, %36, %43, %25\n\t" \
      "v_mfma_f32_16x16x32_bf16 %26, %36, %45, %26\n\t" \
      "ds_read_b128 %5, %48 offset:5120\n\t" \
      "v_mfma_f32_16x16x32_bf16 %27, %36, %47, %27\n\t" \
      "v_mfma_f32_16x16x32_bf16 %28, %38, %41, %28\n\t" \
      "v_mfma_f32_16x16x32_bf16 %29, %38, %43, %29\n\t" \
      "ds_read_b128 %12, %49 offset:4096\n\t" \
      "v_mfma_f32_16x16x32_bf16 %30, %38, %45, %30\n\t" \
      "v_mfma_f32_16x16x32_bf16 %31, %38, %47, %31\n\t" \
      "v_mfma_f32_16x16x32_bf16 %16, %32, %40, %16\n\t" \
      "ds_read_b128 %13, %49 offset:5120\n\t" \
      "v_mfma_f32_16x16x32_bf16 %17, %32, %42, %17\n\t" \
      "v_mfma_f32_16x16x32_bf16 %18, %32, %44, %18\n\t" \
      "v_mfma_f32_16x16x32_bf16 %19, %32, %46, %19\n\t" \
      "ds_read_b128 %6, %48 offset:6144\n\t" \
      "v_mfma_f32_16x16x32_bf16 %20, %34, %40, %20\n\t" \
      "v_mfma_f32_16x16x32_bf16 %21, %34, %42, %21\n\t" \
      "v_mfma_f32_16x16x32_bf16 %22, %34, %44, %22\n\t" \
      "ds_read_b128 %7, %48 offset:7168\n\t" \
      "v_mfma_f32_16x16x32_bf16 %23, %34, %46, %23\n\t" \
      "v_mfma_f32_16x16x32_bf16 %24, %36, %40, %24\n\t" \
      "v_mfma_f32_16x16x32_bf16 %25, %36, %42, %25\n\t" \
      "ds_read_b128 %14, %49 offset:6144\n\t" \
      "v_mfma_f32_16x16x32_bf16 %26, %36, %44, %26\n\t" \
      "v_mfma_f32_16x16x32_bf16 %27, %36, %46, %27\n\t" \
      "v_mfma_f32_16x16x32_bf16 %28, %38, %40, %28\n\t" \
      "ds_read_b128 %15, %49 offset:7168\n\t" \
      "v_mfma_f32_16x16x32_bf16 %29, %38, %42, %29\n\t" \
      "v_mfma_f32_16x16x32_bf16 %30, %38, %44, %30\n\t" \
      "v_mfma_f32_16x16x32_bf16 %31, %38, %46, %31\n\t" \
      "s_waitcnt lgkmcnt(0)\n\t"

  int k = 0;
  for (; k + 1 < KB; k += 2) {
    IDMRG_PIPE_STEP(k, F0, F1);
    IDMRG_PIPE_STEP(k + 1, F1, F0);
  }
  if (k < KB) IDMRG_PIPE_STEP(k, F0, F1);
#undef IDMRG_PIPE_STEP
#undef IDMRG_PIPE_ASM
  // wait states between the last MFMAs and the stores that read their results;
  // the register sets are named here so that every asm output has a use
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7"
               : "+v"(acc[0][0]), "+v"(acc[0][1]), "+v"(acc[0][2]), "+v"(acc[0][3]), "+v"(acc[1][0]),
                 "+v"(acc[1][1]), "+v"(acc[1][2]), "+v"(acc[1][3]), "+v"(acc[2][0]), "+v"(acc[2][1]),
                 "+v"(acc[2][2]), "+v"(acc[2][3]), "+v"(acc[3][0]), "+v"(acc[3][1]), "+v"(acc[3][2]),
                 "+v"(acc[3][3]));
#pragma unroll
  for (int i = 0; i < 16; ++i) asm volatile("" ::"v"(F0[i]), "v"(F1[i]));
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
  if (tiling == 5) {   // 128 x 128, persistent workgroups, pipelined across tiles
    const int g = std::min(ntiles, kPersistPerCu * kCus);
    const dim3 pgrid(kXcd * ((g + kXcd - 1) / kXcd));
    if (mode == 0)
      hipLaunchKernelGGL(gemm_bf16x3_persist_kernel<0>, pgrid, dim3(256), 0, s, tasks, ntask, bases, active, ntiles);
    else
      hipLaunchKernelGGL(gemm_bf16x3_persist_kernel<1>, pgrid, dim3(256), 0, s, tasks, ntask, bases, active, ntiles);
    return;
  }
  if (tiling == 4) {   // 256 x 128, eight waves, three stages, pipelined operand reads
    if (mode == 0)
      hipLaunchKernelGGL(gemm_bf16x3_pipe_kernel<0>, grid, dim3(512), 0, s, tasks, ntask, bases, active, ntiles);
    else
      hipLaunchKernelGGL(gemm_bf16x3_pipe_kernel<1>, grid, dim3(512), 0, s, tasks, ntask, bases, active, ntiles);
    return;
  }
  switch (tiling) {
    case 0: launch_b3<64, 64>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case 1: launch_b3<128, 64>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case 2: launch_b3<64, 128>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    default: launch_b3<128, 128>(mode, grid, s, tasks, ntask, bases, active, ntiles); break;
  }
}

void launch_gemm(Prec prec, int mode, const GemmTask* tasks, int ntask, int ntiles, int xmax, void* const* bases,
                 const int32_t* active, hipStream_t s, int tiling) {
  if (ntask == 0 || ntiles == 0) return;
  if (xmax <= 0 || xmax > ntiles) throw InvalidArg("internal: GEMM tile ranges");
  dim3 grid(kXcd * xmax), block(256);
  switch (prec) {
    case Prec::F64: launch_t<double>(tiling, mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case Prec::F32: launch_t<float>(tiling, mode, grid, s, tasks, ntask, bases, active, ntiles); break;
    case Prec::BF16X3: launch_bf16x3(tiling, mode, grid, s, tasks, ntask, bases, active, ntiles); break;
  }
}

}  // namespace idmrg
