// C-ABI entry points (idmrg.h): validation, work plans, the device scratch
// layout of each call, plan upload and the launch sequences of the five calls.
//
// Every call runs in two phases.  The plan phase is host work only: it
// validates the descriptors, builds the task lists of the grouped kernels and
// lays out the call's device scratch as one block (idmrg_workspace_size
// returns that block's size).  The bind phase takes the block from the
// caller's workspace (or from scratch the library owns), copies the task lists
// to the device through a pinned staging ring allocated with the context, and
// enqueues the kernels.  The plan of the last call of each kind is kept, keyed
// by a hash of everything it depends on, so that a size query followed by the
// call plans once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <tuple>

#include "idmrg.h"
#include "internal.h"
#include "plan.h"

using namespace idmrg;

// ------------------------------------------------------------------ context

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double flops;
};

struct RingSlot {
  size_t begin, end;
  hipEvent_t ev;
};

// A call needs more device scratch than the attached workspace holds, or the
// library could not allocate its own.
struct OutOfWorkspace {
  std::string what;
};

constexpr size_t kRingBytes = size_t(32) << 20;   // pinned staging ring of the plan uploads
constexpr size_t kRingChunk = size_t(8) << 20;    // largest single staged copy
constexpr size_t kRingSlotsMax = 256;             // copies tracked before the oldest is waited for
constexpr int kOps = 8;
constexpr int kPlanWays = 8;   // cached plans per operation (a unit cell's pieces differ in shape)

// Scratch of heff_apply_static: a file-scope device array, one copy per GPU,
// held until the process ends.  Host code never passes its name to a kernel:
// the address comes from hipGetSymbolAddress on each device (idmrg_create).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

struct CallPlan;

}  // namespace

struct idmrg_ctx {
  int device = 0;
  // profiling (see idmrg_profile)
  bool prof = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  int64_t prof_n[IDMRG_PROF_CLASSES] = {};
  double prof_ms[IDMRG_PROF_CLASSES] = {};
  double prof_flops[IDMRG_PROF_CLASSES] = {};
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;   // graph capture only (nothing executes on it); created on first use
  std::string err;
  // device scratch of the calls: the caller's workspace if one is attached, else the library's own block
  char* user_ws = nullptr;
  size_t user_ws_n = 0;
  DevBuf own;
  // pinned staging ring of the plan uploads (allocated with the context)
  char* ring = nullptr;
  size_t ring_head = 0;
  std::deque<RingSlot> ring_busy;
  std::vector<hipEvent_t> ring_events;
  idmrg_stats stats = {};
  void* static_scratch = nullptr;   // this device's copy of `scratch` (heff_apply_static)
  // GEMM tile autotuner: measured best tiling per (precision, stage, shape bucket), and the
  // trial time of each tiling (ms, -1 if not tried)
  std::map<std::tuple<int, int, int, int, int>, int> tune;
  std::map<std::tuple<int, int, int, int, int>, std::vector<float>> tune_ms;
  hipEvent_t tev[6][4] = {};   // [variant][stage-1 start, stage-1 end, stage-2 start, stage-2 end]
  // the plan of the last call of each kind and the hash of its inputs
  uint64_t cache_key[kOps][kPlanWays] = {};
  uint64_t cache_used[kOps][kPlanWays] = {};
  uint64_t cache_tick = 0;
  std::shared_ptr<CallPlan> cache[kOps][kPlanWays];
};

namespace {

void sync(idmrg_ctx* c) {
  ++c->stats.stream_syncs;
  IDMRG_HIP(hipStreamSynchronize(c->stream));
}

hipEvent_t take_event(idmrg_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  IDMRG_HIP(hipEventCreate(&e));
  return e;
}

// Brackets the launches issued during its lifetime with events (if profiling).
struct Prof {
  idmrg_ctx* c;
  ProfRec r{};
  Prof(idmrg_ctx* ctx, int cls, double flops) : c(ctx) {
    if (!c->prof) return;
    r.cls = cls;
    r.flops = flops;
    r.a = take_event(c);
    r.b = take_event(c);
    IDMRG_HIP(hipEventRecord(r.a, c->stream));
  }
  ~Prof() {
    if (!c->prof) return;
    if (hipEventRecord(r.b, c->stream) == hipSuccess) c->pending.push_back(r);
  }
};

void prof_collect(idmrg_ctx* c) {
  if (c->pending.empty()) return;
  sync(c);
  for (auto& r : c->pending) {
    float ms = 0.f;
    IDMRG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    c->prof_n[r.cls] += 1;
    c->prof_ms[r.cls] += ms;
    c->prof_flops[r.cls] += r.flops;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->pending.clear();
}

// ------------------------------------------------------------------ device scratch and uploads

// Byte layout of one call's scratch block; every region starts on a 256-byte boundary.
struct Layout {
  size_t total = 0;
  size_t add(size_t bytes) {
    const size_t o = (total + 255) / 256 * 256;
    total = o + std::max<size_t>(bytes, 8);
    return o;
  }
};

// The scratch block of a call: the attached workspace, or the library's own
// block, grown (after the stream has drained) when a call needs more.
char* acquire(idmrg_ctx* c, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  if (c->user_ws) {
    if (bytes > c->user_ws_n)
      throw OutOfWorkspace{"the attached workspace holds " + std::to_string(c->user_ws_n) +
                           " bytes; this call needs " + std::to_string(bytes) + " (idmrg_workspace_size)"};
    return c->user_ws;
  }
  if (c->own.n < bytes) {
    sync(c);   // queued work may still use the old block
    const size_t want = (std::max(bytes, c->own.n + c->own.n / 4) + 4095) / 4096 * 4096;
    if (c->own.p) IDMRG_HIP(hipFree(c->own.p));
    c->own = DevBuf{};
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      throw OutOfWorkspace{"device allocation of " + std::to_string(want) + " bytes of scratch failed"};
    }
    c->own = DevBuf{p, want};
    ++c->stats.device_allocs;
  }
  return (char*)c->own.p;
}

// The ring's events are created with the context (kRingSlotsMax of them, as
// many as copies are ever tracked), so an upload creates nothing.
hipEvent_t ring_event(idmrg_ctx* c) {
  if (c->ring_events.empty()) throw HipFailure("internal: staging ring out of events");
  hipEvent_t e = c->ring_events.back();
  c->ring_events.pop_back();
  return e;
}

// Waits for the copy that last read ring slot k and for every older one (a
// stream runs its copies in order), and releases them.
void ring_release_through(idmrg_ctx* c, size_t k) {
  IDMRG_HIP(hipEventSynchronize(c->ring_busy[k].ev));
  for (size_t i = 0; i <= k; ++i) {
    c->ring_events.push_back(c->ring_busy.front().ev);
    c->ring_busy.pop_front();
  }
}

// Copies host bytes to device memory at dst, asynchronously on the context
// stream, through the pinned ring: a region of the ring is rewritten only after
// the copy that last read it has run, so the host blocks only when more than
// the ring's worth of uploads is still queued.
void stage(idmrg_ctx* c, void* dst, const void* src, size_t bytes) {
  const char* s = (const char*)src;
  char* d = (char*)dst;
  while (bytes > 0) {
    const size_t n = std::min(bytes, kRingChunk);
    size_t off = (c->ring_head + 255) / 256 * 256;
    if (off + n > kRingBytes) off = 0;
    size_t last = SIZE_MAX;
    for (size_t i = 0; i < c->ring_busy.size(); ++i)
      if (c->ring_busy[i].begin < off + n && off < c->ring_busy[i].end) last = i;
    if (last != SIZE_MAX) ring_release_through(c, last);
    if (c->ring_busy.size() >= kRingSlotsMax) ring_release_through(c, 0);
    std::memcpy(c->ring + off, s, n);
    IDMRG_HIP(hipMemcpyAsync(d, c->ring + off, n, hipMemcpyHostToDevice, c->stream));
    hipEvent_t ev = ring_event(c);
    IDMRG_HIP(hipEventRecord(ev, c->stream));
    c->ring_busy.push_back(RingSlot{off, off + n, ev});
    c->ring_head = off + n;
    c->stats.staged_bytes += (int64_t)n;
    s += n;
    d += n;
    bytes -= n;
  }
}

// Collects host arrays into one upload; offsets aligned to 256 bytes.
// reserve() leaves room for data known only when the call binds (pointer tables).
struct Packer {
  std::vector<char> host;
  size_t add(const void* p, size_t bytes) {
    const size_t off = reserve(bytes);
    if (bytes) std::memcpy(host.data() + off, p, bytes);
    return off;
  }
  template <typename T>
  size_t add(const std::vector<T>& v) { return add(v.data(), v.size() * sizeof(T)); }
  size_t reserve(size_t bytes) {
    const size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + std::max<size_t>(bytes, 8));
    return off;
  }
  template <typename T>
  void patch(size_t off, const std::vector<T>& v) {
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
  }
};

template <typename F>
int guarded(idmrg_ctx* c, F&& f) {
  if (!c) return IDMRG_EINVAL;
  try {
    c->err.clear();
    IDMRG_HIP(hipSetDevice(c->device));
    return f();
  } catch (const InvalidArg& e) {
    c->err = e.what;
    return IDMRG_EINVAL;
  } catch (const HipFailure& e) {
    c->err = e.what;
    return IDMRG_EHIP;
  } catch (const OutOfWorkspace& e) {
    c->err = e.what;
    return IDMRG_ENOMEM;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return IDMRG_ENOMEM;
  } catch (...) {
    c->err = "unexpected internal error";
    return IDMRG_EUNSUPPORTED;
  }
}

// The caller's buffer at p must hold n elements of esize bytes inside one device allocation.
void check_dev(const void* p, int64_t n, size_t esize, const std::string& what) {
  if (!p) throw InvalidArg(what + ": null pointer");
  if (n <= 0) return;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    throw InvalidArg(what + ": not a device allocation of this context's device");
  }
  if ((const char*)p + (size_t)n * esize > (const char*)base + size) throw InvalidArg(what + ": buffer too small");
}

void check_nprob(int nprob) {
  if (nprob < 1 || nprob > 64) throw InvalidArg("nprob must be 1..64");
}

// ------------------------------------------------------------------ plan cache

// FNV-1a over everything a plan depends on (legs, MPO tensors and charges, options).
struct Hash {
  uint64_t h = 1469598103934665603ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  }
  template <typename T>
  void val(const T& v) { bytes(&v, sizeof(T)); }
  template <typename T>
  void arr(const T* p, int64_t n) {
    val(n);
    if (p && n > 0 && n < (int64_t(1) << 24)) bytes(p, (size_t)n * sizeof(T));
    else val(p);
  }
  void leg(const idmrg_leg& l) {
    arr(l.q, l.nsec);
    arr(l.dim, l.nsec);
  }
  void mpo(const idmrg_mpo* m) {
    val(m == nullptr);
    if (!m) return;
    val(m->dl);
    val(m->dr);
    val(m->d);
    const int64_t nw = (m->dl > 0 && m->dr > 0 && m->d > 0 && m->dl < 4096 && m->dr < 4096 && m->d < 64)
                           ? (int64_t)m->dl * m->dr * m->d * m->d : 0;
    arr(m->w, nw);
    arr(m->ql, m->dl);
    arr(m->qr, m->dr);
    arr(m->qp, m->d);
  }
};

struct CallPlan {
  virtual ~CallPlan() = default;
  Layout lay;
};

// The cached plan of kind `op` if one of its entries has this key, else a new
// one from build(), cached in place of the least recently used entry.
template <typename T, typename F>
std::shared_ptr<T> plan_of(idmrg_ctx* c, int op, uint64_t key, F&& build) {
  int victim = 0;
  for (int w = 0; w < kPlanWays; ++w) {
    if (c->cache[op][w] && c->cache_key[op][w] == key) {
      auto p = std::dynamic_pointer_cast<T>(c->cache[op][w]);
      if (p) {
        c->cache_used[op][w] = ++c->cache_tick;
        return p;
      }
    }
    if (c->cache_used[op][w] < c->cache_used[op][victim]) victim = w;
  }
  c->cache[op][victim].reset();
  auto p = std::make_shared<T>();
  build(*p);
  ++c->stats.plan_builds;
  c->cache[op][victim] = p;
  c->cache_key[op][victim] = key;
  c->cache_used[op][victim] = ++c->cache_tick;
  return p;
}

// ------------------------------------------------------------------ H_eff execution

// Output tilings of the GEMM kernels: code c < 4 -> (c & 1 ? 128 : 64) x (c & 2 ? 128 : 64) (four waves);
// code 4 -> 256 x 128 (split-bf16 only: eight waves, three LDS stages, the
// operand reads of each slab overlapped with the previous slab's MFMAs);
// code 5 -> 128 x 128 (split-bf16 only: persistent workgroups, the copy
// pipeline running on across tiles).
constexpr int kTilings = 6;
static_assert(sizeof(idmrg_ctx::tev) / sizeof(idmrg_ctx::tev[0]) >= kTilings, "one event row per tiling variant");

struct HeffExec {
  HeffPlan plan;
  int P = 0;
  Prec prec = Prec::F64;
  bool frag = false;
  // every tiling variant of both GEMM stages is uploaded; sel[stage] is the one in use
  std::vector<GemmList> var[2];
  int tiles[2][kTilings] = {};
  int code[kTilings] = {};
  int nvar = 1;
  int sel[2] = {0, 0};
  bool need_tune[2] = {false, false};
  std::tuple<int, int, int, int, int> key[2];
  double flops_g1 = 0, flops_g2 = 0, flops_mix = 0;
  std::vector<int64_t> npsi;
  std::vector<char> has_shift;   // per problem: the low-precision copies carry an energy shift
  // scratch regions (byte offsets in the call's block) and per-problem element offsets inside them
  size_t oT1 = 0, oT3 = 0, nT3bytes = 0, oEnv = 0, oVec = 0, oSums = 0, oShift = 0, oSig = 0, oPlan = 0;
  std::vector<int64_t> o1, o3, oL, oR, oXmix, oYlow, oXlow;
  std::vector<DiagTask> diag;
  size_t nDL = 0;
  // the uploaded plan: task lists (offsets in pk) and the pointer tables patched at bind
  Packer pk;
  size_t av[2][kTilings] = {}, aMY = 0, aSY = 0, aMT = 0, aST = 0, aHB = 0, aSB = 0, aPX = 0, aPL = 0, aPR = 0,
         aDiag = 0, aFlags = 0;
  // bound pointers
  GemmTask* gv[2][kTilings] = {};
  MixTask *mY = nullptr, *mT = nullptr;
  MixSrc *sY = nullptr, *sT = nullptr;
  void** bases = nullptr;      // device [P][8]
  void** sbases = nullptr;     // low precision: FP64 sources of the packs and diagonals (0 L, 1 R, 2 x)
  PackTask* pX = nullptr;
  double* sig = nullptr;       // device [P][2] energy shifts
  std::vector<void*> xmix, ylow;
};

int ilog2(double x) { return x >= 1.0 ? (int)std::floor(std::log2(x)) : 0; }

// Shape bucket of one GEMM stage: precision, stage, log2 of the flops and of
// the flop-weighted mean N and K (the tile choice depends on these, not on
// the exact block dimensions, which change a little every iteration).
std::tuple<int, int, int, int, int> tune_key(Prec prec, int stage, const GemmList& g) {
  double f = 0, fn = 0, fk = 0;
  for (const auto& t : g.t) {
    const double w = 2.0 * t.M * (double)t.N * t.K;
    f += w;
    fn += w * t.N;
    fk += w * t.K;
  }
  return std::make_tuple((int)prec, stage, ilog2(f), f > 0 ? ilog2(fn / f) : 0, f > 0 ? ilog2(fk / f) : 0);
}

// After the trial matvecs of every variant have completed: keep the fastest
// tiling of each stage that still needed tuning, and remember it.
void tune_resolve(idmrg_ctx* c, HeffExec& ex, int ntried) {
  if (ntried < 1) return;
  for (int st = 0; st < 2; ++st) {
    if (!ex.need_tune[st]) continue;
    int best = -1;
    float bms = 0.f;
    for (int v = 0; v < ntried; ++v) {
      float ms = 0.f;
      IDMRG_HIP(hipEventElapsedTime(&ms, c->tev[v][2 * st], c->tev[v][2 * st + 1]));
      if (best < 0 || ms < bms) best = v, bms = ms;
    }
    ex.sel[st] = best;
    ex.need_tune[st] = false;
    if (ntried == ex.nvar) {
      c->tune[ex.key[st]] = best;
      std::vector<float> ms(IDMRG_TUNE_VARIANTS, -1.f);
      for (int v = 0; v < ntried; ++v)
        IDMRG_HIP(hipEventElapsedTime(&ms[ex.code[v]], c->tev[v][2 * st], c->tev[v][2 * st + 1]));
      c->tune_ms[ex.key[st]] = ms;
    }
  }
}

void hash_heff(Hash& h, int P, const idmrg_heff* H) {
  h.val(P);
  for (int p = 0; p < P; ++p) {
    h.leg(H[p].left);
    h.leg(H[p].right);
    h.mpo(H[p].w1);
    h.mpo(H[p].w2);
  }
}

// Plan phase: task lists for P problems, their host-side bounds checks, and the
// scratch regions (added to lay).  No device work.
void heff_plan(idmrg_ctx* c, HeffExec& ex, int P, const idmrg_heff* H, int prec, Layout& lay) {
  if (prec < 0 || prec > 2) throw InvalidArg("unknown precision policy");
  ex.P = P;
  ex.prec = (Prec)prec;
  ex.frag = ex.prec == Prec::BF16X3;
  const bool frag = ex.frag;
  for (int p = 0; p < P; ++p) {
    if (!H[p].w1 || !H[p].w2) throw InvalidArg("null field in idmrg_heff");
    const Leg A = make_leg(H[p].left, "heff.left"), B = make_leg(H[p].right, "heff.right");
    const Mpo W1 = make_mpo(H[p].w1, "heff.w1"), W2 = make_mpo(H[p].w2, "heff.w2");
    if (W1.dr != W2.dl || W1.qr != W2.ql) throw InvalidArg("w1 columns and w2 rows differ");
    if (W1.qp != W2.qp) throw InvalidArg("w1 and w2 local charges differ");
    build_heff(ex.plan, p, A, B, W1, W2);
    if (ex.plan.n_psi[p] == 0) throw InvalidArg("two-site state has no allowed block");
  }
  ex.npsi = ex.plan.n_psi;
  // Tile variants.  The tile shape does not change the order in which any
  // output element accumulates over k, so all variants give identical results.
  ex.nvar = frag ? 6 : 4;
  for (int v = 0; v < ex.nvar; ++v) ex.code[v] = v;
  for (int st = 0; st < 2; ++st) {
    const GemmList& base = st == 0 ? (frag ? ex.plan.f1 : ex.plan.g1) : (frag ? ex.plan.f2 : ex.plan.g2);
    ex.var[st].clear();
    for (int v = 0; v < ex.nvar; ++v) {
      ex.var[st].push_back(base);
      if (ex.code[v] == 4)
        ex.var[st][v].retile(256, 128);
      else if (ex.code[v] == 5)
        ex.var[st][v].retile(128, 128);
      else
        ex.var[st][v].retile(ex.code[v] & 1 ? 128 : 64, ex.code[v] & 2 ? 128 : 64);
      ex.tiles[st][v] = ex.var[st][v].tiles;
    }
    ex.key[st] = tune_key(ex.prec, st, base);
    auto it = c->tune.find(ex.key[st]);
    ex.need_tune[st] = ex.nvar > 1 && it == c->tune.end();
    if (it != c->tune.end()) {
      ex.sel[st] = it->second;
    } else {   // untuned default: padding heuristic, except 64 x 64 for FP64 (its larger tiles run one wave per SIMD)
      GemmList h = base;
      h.choose_tile(ex.prec != Prec::F64);
      ex.sel[st] = h.tiling();
    }
  }
  ex.flops_g1 = ex.plan.g1.flops();
  ex.flops_g2 = ex.plan.g2.flops();
  ex.flops_mix = ex.plan.mixY.flops() + ex.plan.mixT.flops();
  {
    std::vector<int64_t> sz((size_t)P * kNumBases, -1);
    for (int p = 0; p < P; ++p) {
      int64_t* z = &sz[(size_t)p * kNumBases];
      z[0] = ex.plan.n_L[p]; z[1] = ex.plan.n_R[p]; z[2] = z[3] = z[6] = ex.plan.n_psi[p];
      z[4] = ex.plan.n_T1[p]; z[5] = ex.plan.n_T3[p];
    }
    if (!frag) {
      check_gemm(ex.plan.g1, 0, sz, "heff gemm1");
      check_mix(ex.plan.mixY, sz, "heff mixY");
      check_mix(ex.plan.mixT, sz, "heff mixT");
      check_gemm(ex.plan.g2, 1, sz, "heff gemm2");
    } else {
      std::vector<int64_t> ss = sz;   // FP64 sources of the packs: 0 L, 1 R, 2 x
      for (int p = 0; p < P; ++p) {
        int64_t* z = &sz[(size_t)p * kNumBases];
        z[0] = ex.plan.n_Lf[p]; z[1] = ex.plan.n_Rf[p]; z[2] = ex.plan.n_Xf[p]; z[5] = ex.plan.n_T3f[p];
        z[4] = ex.plan.n_T1f[p]; z[6] = ex.plan.n_Xm[p];
      }
      check_gemm_frag(ex.plan.f1, sz, "heff gemm1");
      check_mix(ex.plan.mixYf, sz, "heff mixY");
      check_mix_v4(ex.plan.mixYf, sz, "heff mixY");
      check_mix_frag(ex.plan.mixTf, sz, "heff mixT");
      check_mix_v4(ex.plan.mixTf, sz, "heff mixT");
      check_gemm_frag(ex.plan.f2, sz, "heff gemm2");
      check_pack(ex.plan.packL, ss, sz, "heff pack L");
      check_pack(ex.plan.packR, ss, sz, "heff pack R");
      check_pack(ex.plan.packX, ss, sz, "heff pack x");
    }
  }
  const size_t es = ex.prec == Prec::F64 ? 8 : 4;   // accumulator / T1 element size
  // sub-buffers start at multiples of 64 elements (256 bytes), which the 16-byte accesses of the split-bf16 kernels need
  auto round64 = [](int64_t n) { return (n + 63) / 64 * 64; };
  int64_t nT1 = 0, nT3 = 0;
  ex.o1.assign(P, 0);
  ex.o3.assign(P, 0);
  for (int p = 0; p < P; ++p) {
    ex.o1[p] = nT1;
    ex.o3[p] = nT3;
    nT1 += round64((frag ? ex.plan.n_T1f[p] : ex.plan.n_T1[p]) + 1);
    nT3 += round64((frag ? ex.plan.n_T3f[p] : ex.plan.n_T3[p]) + 1);
  }
  ex.oT1 = lay.add(nT1 * es);
  ex.nT3bytes = nT3 * es;
  ex.oT3 = lay.add(ex.nT3bytes);
  ex.has_shift.assign(P, 0);
  if (ex.prec != Prec::F64) {
    // 4-byte units: FP32 L, R, x (also the mixing operand), y; or, for split-bf16,
    // fragment-layout L, R, x, plus FP32 x for the mixing and y
    const std::vector<int64_t>& nL = frag ? ex.plan.n_Lf : ex.plan.n_L;
    const std::vector<int64_t>& nR = frag ? ex.plan.n_Rf : ex.plan.n_R;
    int64_t nenv = 0, nvec = 0;
    ex.oL.assign(P, 0);
    ex.oR.assign(P, 0);
    ex.oXmix.assign(P, 0);
    ex.oYlow.assign(P, 0);
    ex.oXlow.assign(P, -1);
    for (int p = 0; p < P; ++p) {
      ex.oL[p] = nenv;
      nenv += round64(nL[p]);
      ex.oR[p] = nenv;
      nenv += round64(nR[p]);
      ex.oXmix[p] = nvec;   // split-bf16: the row-padded copy the x pack writes
      nvec += round64(frag ? ex.plan.n_Xm[p] : ex.npsi[p]);
      ex.oYlow[p] = nvec;
      nvec += round64(ex.npsi[p]);
      if (frag) {
        ex.oXlow[p] = nvec;
        nvec += round64(ex.plan.n_Xf[p]);
      }
      ex.has_shift[p] = (char)(ex.plan.shiftL[p] || ex.plan.shiftR[p]);
    }
    ex.oEnv = lay.add(nenv * 4);
    ex.oVec = lay.add(nvec * 4);
    // energy shift of the low-precision copies (see plan.h): diagonal sums, per-task and per-problem shifts
    ex.diag = ex.plan.diagL;
    ex.diag.insert(ex.diag.end(), ex.plan.diagR.begin(), ex.plan.diagR.end());
    ex.nDL = ex.plan.diagL.size();
    ex.oSums = lay.add(ex.diag.size() * 8);
    ex.oShift = lay.add(ex.diag.size() * 8);
    ex.oSig = lay.add((size_t)P * 2 * 8);
  }
  // the upload: tile variants of both stages, mixing lists, pointer tables, packs, diagonals, shift flags
  Packer& pk = ex.pk;
  pk.host.clear();
  for (int st = 0; st < 2; ++st)
    for (int v = 0; v < ex.nvar; ++v) ex.av[st][v] = pk.add(ex.var[st][v].upload());
  const MixList& mY = frag ? ex.plan.mixYf : ex.plan.mixY;
  const MixList& mT = frag ? ex.plan.mixTf : ex.plan.mixT;
  ex.aMY = pk.add(mY.t);
  ex.aSY = pk.add(mY.src);
  ex.aMT = pk.add(mT.t);
  ex.aST = pk.add(mT.src);
  ex.aHB = pk.reserve((size_t)P * kNumBases * sizeof(void*));
  if (ex.prec != Prec::F64) {
    ex.aSB = pk.reserve((size_t)P * kNumBases * sizeof(void*));
    ex.aDiag = pk.add(ex.diag);
    std::vector<int32_t> flags(2 * (size_t)P);
    for (int p = 0; p < P; ++p) {
      flags[2 * p] = ex.plan.shiftL[p];
      flags[2 * p + 1] = ex.plan.shiftR[p];
    }
    ex.aFlags = pk.add(flags);
  }
  if (frag) {
    ex.aPX = pk.add(ex.plan.packX.t);
    ex.aPL = pk.add(ex.plan.packL.t);
    ex.aPR = pk.add(ex.plan.packR.t);
  }
  ex.oPlan = lay.add(pk.host.size());
}

// Bind phase: the scratch regions at `base`, the vectors x / y (device, FP64),
// the plan upload and the per-operator work (low-precision copies of L and R
// with their energy shifts).
void heff_bind(idmrg_ctx* c, HeffExec& ex, char* base, const idmrg_heff* H, const std::vector<double*>& x,
               const std::vector<double*>& y) {
  const int P = ex.P;
  const bool frag = ex.frag;
  hipStream_t s = c->stream;
  for (int p = 0; p < P; ++p) {
    if (!H[p].L || !H[p].R) throw InvalidArg("null field in idmrg_heff");
    check_dev(H[p].L, ex.plan.n_L[p], 8, "heff.L");
    check_dev(H[p].R, ex.plan.n_R[p], 8, "heff.R");
    check_dev(x[p], ex.plan.n_psi[p], 8, "x");
    check_dev(y[p], ex.plan.n_psi[p], 8, "y");
  }
  const size_t es = ex.prec == Prec::F64 ? 8 : 4;
  char* T1 = base + ex.oT1;
  char* T3 = base + ex.oT3;
  std::vector<void*> hb((size_t)P * kNumBases, nullptr), sb;
  ex.xmix.assign(P, nullptr);
  ex.ylow.assign(P, nullptr);
  char* env = base + ex.oEnv;
  char* vec = base + ex.oVec;
  for (int p = 0; p < P; ++p) {
    void** b = &hb[(size_t)p * kNumBases];
    b[4] = T1 + ex.o1[p] * es;
    b[5] = T3 + ex.o3[p] * es;
    if (ex.prec == Prec::F64) {
      b[0] = (void*)H[p].L;
      b[1] = (void*)H[p].R;
      b[2] = x[p];
      b[3] = y[p];
      b[6] = x[p];
    } else {
      ex.xmix[p] = vec + ex.oXmix[p] * 4;
      ex.ylow[p] = vec + ex.oYlow[p] * 4;
      b[0] = env + ex.oL[p] * 4;
      b[1] = env + ex.oR[p] * 4;
      b[2] = frag ? (void*)(vec + ex.oXlow[p] * 4) : ex.xmix[p];
      b[3] = ex.ylow[p];
      b[6] = ex.xmix[p];
    }
  }
  ex.pk.patch(ex.aHB, hb);
  if (ex.prec != Prec::F64) {
    sb.assign((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      sb[(size_t)p * kNumBases + 0] = (void*)H[p].L;
      sb[(size_t)p * kNumBases + 1] = (void*)H[p].R;
      sb[(size_t)p * kNumBases + 2] = x[p];
    }
    ex.pk.patch(ex.aSB, sb);
  }
  char* dev = base + ex.oPlan;
  stage(c, dev, ex.pk.host.data(), ex.pk.host.size());
  for (int st = 0; st < 2; ++st)
    for (int v = 0; v < ex.nvar; ++v) ex.gv[st][v] = (GemmTask*)(dev + ex.av[st][v]);
  ex.mY = (MixTask*)(dev + ex.aMY);
  ex.sY = (MixSrc*)(dev + ex.aSY);
  ex.mT = (MixTask*)(dev + ex.aMT);
  ex.sT = (MixSrc*)(dev + ex.aST);
  ex.bases = (void**)(dev + ex.aHB);
  ex.sbases = ex.prec != Prec::F64 ? (void**)(dev + ex.aSB) : nullptr;
  // the fragment form of T3 is written only inside its blocks: its padding stays zero from here on
  if (frag) IDMRG_HIP(hipMemsetAsync(T3, 0, ex.nT3bytes, s));
  if (ex.prec == Prec::F64) return;
  if (!frag)
    for (int p = 0; p < P; ++p) {
      launch_convert(0, H[p].L, hb[(size_t)p * kNumBases + 0], ex.plan.n_L[p], s);
      launch_convert(0, H[p].R, hb[(size_t)p * kNumBases + 1], ex.plan.n_R[p], s);
    }
  // energy shifts of the low-precision copies: sL, sR = mean diagonal of the H_L and H_R blocks
  ex.sig = (double*)(base + ex.oSig);
  double* shift = (double*)(base + ex.oShift);
  const DiagTask* dt = (const DiagTask*)(dev + ex.aDiag);
  if (!ex.diag.empty()) {
    launch_diag_sum(dt, (int)ex.diag.size(), ex.sbases, (double*)(base + ex.oSums), s);
    launch_sigma(dt, (int)ex.diag.size(), (int)ex.nDL, (const double*)(base + ex.oSums),
                 (const int32_t*)(dev + ex.aFlags), P, ex.sig, shift, s);
  } else {
    IDMRG_HIP(hipMemsetAsync(ex.sig, 0, (size_t)P * 2 * 8, s));
  }
  if (ex.prec == Prec::F32 && !ex.diag.empty())   // the FP32 copies of the H_L, H_R diagonals, shifted
    launch_diag_shift_f32(dt, (int)ex.diag.size(), ex.sbases, ex.bases, shift, s);
  if (frag) {
    // operands fixed for the whole operator: packed once here
    ex.pX = (PackTask*)(dev + ex.aPX);
    launch_pack((PackTask*)(dev + ex.aPL), (int)ex.plan.packL.t.size(), ex.plan.packL.tiles, ex.sbases, ex.bases,
                ex.sig, nullptr, s);
    launch_pack((PackTask*)(dev + ex.aPR), (int)ex.plan.packR.t.size(), ex.plan.packR.tiles, ex.sbases, ex.bases,
                ex.sig, nullptr, s);
  }
  IDMRG_HIP(hipGetLastError());
}

// y = H x for every problem (x, y: the FP64 vectors given at bind).
// trial >= 0: run tiling variant `trial` in both stages and bracket each stage with the tuning events.
void heff_run(idmrg_ctx* c, HeffExec& ex, const std::vector<double*>& x, const std::vector<double*>& y,
              const int32_t* active, int trial = -1) {
  hipStream_t s = c->stream;
  if (ex.prec != Prec::F64) {
    Prof pr(c, 3, 0.0);
    if (ex.frag)   // also writes the padded FP32 copy of x for the mixing
      launch_pack(ex.pX, (int)ex.plan.packX.t.size(), ex.plan.packX.tiles, ex.sbases, ex.bases, ex.sig, active, s);
    else
      for (int p = 0; p < ex.P; ++p) launch_convert(0, x[p], ex.xmix[p], ex.npsi[p], s);
  }
  const bool frag = ex.frag;
  const int tin = ex.prec == Prec::F64 ? 0 : (frag ? 4 : 1);
  const int toutT = ex.prec == Prec::F64 ? 0 : (ex.prec == Prec::F32 ? 1 : 3);
  const int toutY = ex.prec == Prec::F64 ? 0 : 1;
  const int lo = ex.prec == Prec::F64 ? 0 : 9;   // profile classes of the low-precision policies
  const int v1 = trial >= 0 ? trial : ex.sel[0], v2 = trial >= 0 ? trial : ex.sel[1];
  {
    Prof pr(c, lo + 0, ex.flops_g1);
    if (trial >= 0) IDMRG_HIP(hipEventRecord(c->tev[trial][0], s));
    launch_gemm(ex.prec, 0, ex.gv[0][v1], (int)ex.plan.g1.t.size(), ex.tiles[0][v1], ex.var[0][v1].xmax, ex.bases,
                active, s,
                ex.code[v1]);
    if (trial >= 0) IDMRG_HIP(hipEventRecord(c->tev[trial][1], s));
  }
  {
    Prof pr(c, lo + 2, ex.flops_mix);
    const MixList& mY = frag ? ex.plan.mixYf : ex.plan.mixY;
    launch_mix(tin, toutY, ex.mY, ex.sY, (int)mY.t.size(), mY.tiles, ex.bases, active, s);
    const MixList& mT = frag ? ex.plan.mixTf : ex.plan.mixT;
    launch_mix(tin, toutT, ex.mT, ex.sT, (int)mT.t.size(), mT.tiles, ex.bases, active, s);
  }
  {
    Prof pr(c, lo + 1, ex.flops_g2);
    if (trial >= 0) IDMRG_HIP(hipEventRecord(c->tev[trial][2], s));
    launch_gemm(ex.prec, 1, ex.gv[1][v2], (int)ex.plan.g2.t.size(), ex.tiles[1][v2], ex.var[1][v2].xmax, ex.bases,
                active, s,
                ex.code[v2]);
    if (trial >= 0) IDMRG_HIP(hipEventRecord(c->tev[trial][3], s));
  }
  if (ex.prec != Prec::F64) {
    Prof pr(c, 3, 0.0);
    for (int p = 0; p < ex.P; ++p) {
      if (ex.has_shift[p])
        launch_convert_add((const float*)ex.ylow[p], x[p], ex.sig, p, y[p], ex.npsi[p], s);
      else
        launch_convert(1, ex.ylow[p], y[p], ex.npsi[p], s);
    }
  }
  IDMRG_HIP(hipGetLastError());
}

// Record what body(stream) launches into a HIP graph and instantiate it.  The
// launches go to the context's capture stream (the library's launchers read
// c->stream, which points there for the duration), so nothing runs now; the
// instance is replayed on the context stream.  Default priority, like every
// stream of the library.
template <typename F>
hipGraphExec_t capture_graph(idmrg_ctx* c, F&& body) {
  if (!c->cap) IDMRG_HIP(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  const hipStream_t keep = c->stream;
  IDMRG_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  c->stream = c->cap;
  hipGraph_t g = nullptr;
  try {
    body(c->cap);
  } catch (...) {
    c->stream = keep;
    (void)hipStreamEndCapture(c->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  c->stream = keep;
  IDMRG_HIP(hipStreamEndCapture(c->cap, &g));
  hipGraphExec_t e = nullptr;
  const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (r != hipSuccess) throw HipFailure(std::string("hipGraphInstantiate: ") + hipGetErrorString(r));
  return e;
}

// Instantiated graphs of one call; released after the stream has drained.
struct GraphSet {
  hipStream_t s;
  hipGraphExec_t ex[4] = {};
  explicit GraphSet(hipStream_t st) : s(st) {}
  ~GraphSet() {
    bool any = false;
    for (auto e : ex) any = any || e;
    if (!any) return;
    (void)hipStreamSynchronize(s);
    for (auto e : ex)
      if (e) (void)hipGraphExecDestroy(e);
  }
};

// ------------------------------------------------------------------ plans of the five calls

struct HeffCall : CallPlan {
  HeffExec ex;
};

std::shared_ptr<HeffCall> heff_call(idmrg_ctx* c, int P, const idmrg_heff* H, int prec) {
  Hash h;
  h.val(prec);
  hash_heff(h, P, H);
  return plan_of<HeffCall>(c, IDMRG_OP_HEFF, h.h, [&](HeffCall& k) { heff_plan(c, k.ex, P, H, prec, k.lay); });
}

struct LanczosCall : CallPlan {
  bool mixed = false;
  int kmax = 0;
  std::vector<int64_t> N, kcap, ld, qoff, woff, voff, soff;
  size_t oV = 0, oSmall = 0, oProbs = 0;
  HeffExec ex64, exlo;
};

std::shared_ptr<LanczosCall> lanczos_call(idmrg_ctx* c, int P, const idmrg_heff* H, const idmrg_lanczos_opts* o) {
  Hash h;
  h.val(o->k_max);
  h.val(o->prec);
  hash_heff(h, P, H);
  return plan_of<LanczosCall>(c, IDMRG_OP_LANCZOS, h.h, [&](LanczosCall& k) {
    if (o->k_max < 1 || o->k_max > kLzMaxK) throw InvalidArg("k_max must be 1..1024");
    if (o->prec < 0 || o->prec > 2) throw InvalidArg("unknown precision policy");
    k.mixed = o->prec != IDMRG_PREC_F64;
    k.kmax = o->k_max;
    k.N.assign(P, 0);
    for (int p = 0; p < P; ++p) {
      if (!H[p].w1) throw InvalidArg("null field in idmrg_heff");
      k.N[p] = psi_layout(make_leg(H[p].left, "left"), make_leg(H[p].right, "right"),
                          make_mpo(H[p].w1, "w1").qp).size;
      if (k.N[p] == 0) throw InvalidArg("empty two-site space");
    }
    // vectors: Q [kcap x N], w, v (and, mixed precision, the normalised start
    // vector s0: the fidelity of Eq. (12) is taken against the refined state);
    // every piece is a multiple of kLzAlign elements, so all rows start 2 KiB-aligned
    k.kcap.assign(P, 0);
    k.ld.assign(P, 0);
    k.qoff.assign(P, 0);
    k.woff.assign(P, 0);
    k.voff.assign(P, 0);
    k.soff.assign(P, 0);
    int64_t tot = 0;
    for (int p = 0; p < P; ++p) {
      k.kcap[p] = std::min<int64_t>(k.kmax, k.N[p]);
      k.ld[p] = (k.N[p] + kLzAlign - 1) / kLzAlign * kLzAlign;
      k.qoff[p] = tot;
      tot += k.kcap[p] * k.ld[p];
      k.woff[p] = tot;
      tot += k.ld[p];
      k.voff[p] = tot;
      tot += k.ld[p];
      k.soff[p] = tot;
      if (k.mixed) tot += k.ld[p];
    }
    k.oV = k.lay.add(tot * 8);
    const size_t nsm = (size_t)P * k.kmax;
    k.oSmall = k.lay.add((size_t)P * (k.kmax + 1) * kLzBlocks * 8 + 4 * nsm * 8 + P * sizeof(LzCtrl) + P * 4 + 4096);
    k.oProbs = k.lay.add((size_t)P * sizeof(LzProblem));
    heff_plan(c, k.ex64, P, H, IDMRG_PREC_F64, k.lay);
    if (k.mixed) heff_plan(c, k.exlo, P, H, o->prec, k.lay);
  });
}

struct TruncSec {
  int q = 0, r = 0, c = 0;
  std::vector<std::tuple<int, int, int>> rows, cols;
  int64_t m = 0, x = 0, g = 0, u = 0, v = 0, sv = 0;
};

struct TruncCall : CallPlan {
  std::vector<int> qp;
  std::vector<std::vector<TruncSec>> secs;
  std::vector<Leg> A, B;
  std::vector<PsiLayout> X;
  int64_t nM = 0, nX = 0, nG = 0, nU = 0, nV = 0, nS = 0;
  MixList gather;
  std::vector<SvdTask> svd;
  std::vector<SelTask> sel;
  std::vector<SelSector> ssec;
  int ncand_tot = 0;
  int pmax = 1;
  BjPlan bj;
  Packer pk;
  size_t a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0;
  size_t oSvd = 0, oSel = 0, oFlag = 0, oPlan = 0, oBjPlan = 0, oBjWork = 0, oOut = 0, outBytes = 0;
};

std::shared_ptr<TruncCall> trunc_call(idmrg_ctx* c, int P, int d, const int32_t* qp_in, int32_t m_max,
                                      const idmrg_trunc* t) {
  Hash h;
  h.val(P);
  h.arr(qp_in, d);
  h.val(m_max);
  for (int p = 0; p < P; ++p) {
    h.leg(t[p].left);
    h.leg(t[p].right);
  }
  return plan_of<TruncCall>(c, IDMRG_OP_TRUNCATE, h.h, [&](TruncCall& k) {
    if (m_max < 1) throw InvalidArg("bad truncation arguments");
    k.qp = make_qp(d, qp_in);
    k.secs.assign(P, {});
    k.A.assign(P, Leg{});
    k.B.assign(P, Leg{});
    k.X.assign(P, PsiLayout{});
    for (int p = 0; p < P; ++p) {
      k.A[p] = make_leg(t[p].left, "trunc.left");
      k.B[p] = make_leg(t[p].right, "trunc.right");
      k.X[p] = psi_layout(k.A[p], k.B[p], k.qp);
      std::map<int, TruncSec> byq;
      for (int a = 0; a < k.A[p].n(); ++a)
        for (int s1 = 0; s1 < d; ++s1) {
          TruncSec& S = byq[k.A[p].q[a] + k.qp[s1]];
          S.rows.emplace_back(a, s1, S.r);
          S.r += k.A[p].dim[a];
        }
      for (int s2 = 0; s2 < d; ++s2)
        for (int b = 0; b < k.B[p].n(); ++b) {
          TruncSec& S = byq[k.B[p].q[b] - k.qp[s2]];
          S.cols.emplace_back(s2, b, S.c);
          S.c += k.B[p].dim[b];
        }
      SelTask st{};
      st.sec0 = (int)k.ssec.size();
      st.cand0 = k.ncand_tot;
      st.m_max = m_max;
      st.prob = p;
      for (auto& kv : byq) {
        TruncSec S = kv.second;
        S.q = kv.first;
        if (S.r == 0 || S.c == 0) continue;
        const int n = std::min(S.r, S.c), pp = std::max(S.r, S.c);
        if (n > 4096 || pp > 8192)
          throw InvalidArg("centre sector larger than 4096 x 8192 states is not supported");
        S.m = k.nM; k.nM += (int64_t)S.r * S.c;
        S.x = k.nX; k.nX += bj_x_elems(n, pp);
        S.g = k.nG; k.nG += (int64_t)n * n;
        S.u = k.nU; k.nU += (int64_t)S.r * n;
        S.v = k.nV; k.nV += (int64_t)S.c * n;
        S.sv = k.nS; k.nS += n;
        k.pmax = std::max(k.pmax, pp);
        for (auto& rw : S.rows)
          for (auto& cl : S.cols) {
            const int a = std::get<0>(rw), s1 = std::get<1>(rw), ro = std::get<2>(rw);
            const int s2 = std::get<0>(cl), b = std::get<1>(cl), co = std::get<2>(cl);
            const int xi = k.X[p].find(a, s1, s2);
            if (xi < 0 || k.X[p].blk[xi].b != b) throw InvalidArg("internal: truncation block bookkeeping");
            MixTask m{};
            m.rows = k.A[p].dim[a]; m.cols = k.B[p].dim[b]; m.ldd = S.c; m.prob = p; m.dbase = 1;
            m.doff = S.m + (int64_t)ro * S.c + co;
            MixSrc sr{};
            sr.coef = 1.0; sr.base = 0; sr.off = k.X[p].blk[xi].off; sr.ld = k.B[p].dim[b];
            k.gather.add(m, {sr});
          }
        SvdTask sv{};
        sv.r = S.r; sv.c = S.c; sv.prob = p;
        sv.m_off = S.m; sv.x_off = S.x; sv.g_off = S.g; sv.u_off = S.u; sv.v_off = S.v; sv.s_off = S.sv;
        sv.f_off = S.x + bj_f_rel(n, pp);
        k.svd.push_back(sv);
        SelSector se{};
        se.charge = S.q; se.n = n; se.cand0 = k.ncand_tot; se.s_off = S.sv;
        k.ssec.push_back(se);
        k.ncand_tot += n;
        st.ncand += n;
        st.nsec += 1;
        k.secs[p].push_back(S);
      }
      if (st.ncand > 8192) throw InvalidArg("more than 8192 singular values per problem is not supported");
      if (st.ncand == 0) throw InvalidArg("two-site state has no centre sector");
      k.sel.push_back(st);
    }
    {
      std::vector<int64_t> sz((size_t)P * kNumBases, -1);
      for (int p = 0; p < P; ++p) {
        sz[(size_t)p * kNumBases + 0] = k.X[p].size;
        sz[(size_t)p * kNumBases + 1] = k.nM;
      }
      check_mix(k.gather, sz, "truncation gather");
    }
    // SVD scratch: M, X, G, U, V, S (each padded by 64 elements)
    k.oSvd = k.lay.add((k.nM + k.nX + k.nG + k.nU + k.nV + k.nS + 6 * 64) * 8);
    k.oSel = k.lay.add((size_t)k.ncand_tot * (4 + 8) + k.ssec.size() * 4 + P * 32 + 4096);
    k.oFlag = k.lay.add(4);
    k.a1 = k.pk.add(k.gather.t);
    k.a2 = k.pk.add(k.gather.src);
    k.a3 = k.pk.add(k.svd);
    k.a4 = k.pk.add(k.sel);
    k.a5 = k.pk.add(k.ssec);
    k.a6 = k.pk.reserve((size_t)P * kNumBases * sizeof(void*));
    k.oPlan = k.lay.add(k.pk.host.size());
    bj_prepare(k.svd, k.bj);
    k.oBjPlan = k.lay.add(k.bj.host.size());
    k.oBjWork = k.lay.add(k.bj.scratch);
    // the output scatter: at most three tasks (U, V, lambda) per sector, and a pointer table
    Packer most;
    most.add(std::vector<ScaleTask>(3 * k.ssec.size()));
    most.reserve((size_t)P * kNumBases * sizeof(void*));
    k.outBytes = most.host.size();
    k.oOut = k.lay.add(k.outBytes);
  });
}

struct EnvCall : CallPlan {
  EnvPlan plan;
  std::vector<int64_t> sz, o1, o2;
  size_t oT = 0, oPlan = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
  int64_t n1 = 0;
  Packer pk;
};

std::shared_ptr<EnvCall> env_call(idmrg_ctx* c, int P, int side, const idmrg_env_update* u) {
  Hash h;
  h.val(P);
  for (int p = 0; p < P; ++p) {
    h.leg(u[p].old_leg);
    h.leg(u[p].new_leg);
    h.mpo(u[p].w);
  }
  const int op = side == IDMRG_LEFT ? IDMRG_OP_ENV_LEFT : IDMRG_OP_ENV_RIGHT;
  return plan_of<EnvCall>(c, op, h.h, [&](EnvCall& k) {
    k.sz.assign((size_t)P * kNumBases, -1);
    for (int p = 0; p < P; ++p) {
      const Leg O = make_leg(u[p].old_leg, "env.old_leg"), C = make_leg(u[p].new_leg, "env.new_leg");
      const Mpo W = make_mpo(u[p].w, "env.w");
      int64_t* z = &k.sz[(size_t)p * kNumBases];
      if (side == IDMRG_LEFT) {
        build_envL(k.plan, p, O, C, W);
        z[0] = envL_layout(O, W.ql).size; z[1] = U_layout(O, W.qp, C).size; z[2] = envL_layout(C, W.qr).size;
      } else {
        build_envR(k.plan, p, O, C, W);
        z[0] = envR_layout(O, W.qr).size; z[1] = V_layout(O, W.qp, C).size; z[2] = envR_layout(C, W.ql).size;
      }
      z[3] = k.plan.n_T1[p]; z[4] = k.plan.n_T2[p];
    }
    check_gemm(k.plan.ga, side == IDMRG_LEFT ? 0 : 2, k.sz, "env stage a");
    check_mix(k.plan.mix, k.sz, "env mix");
    check_gemm(k.plan.gc, side == IDMRG_LEFT ? 2 : 0, k.sz, "env stage c");
    int64_t n1 = 0, n2 = 0;
    k.o1.assign(P, 0);
    k.o2.assign(P, 0);
    for (int p = 0; p < P; ++p) {
      k.o1[p] = n1; n1 += k.plan.n_T1[p] + 64;
      k.o2[p] = n2; n2 += k.plan.n_T2[p] + 64;
    }
    k.n1 = n1;
    k.oT = k.lay.add((n1 + n2) * 8);
    k.a1 = k.pk.add(k.plan.ga.upload());
    k.a2 = k.pk.add(k.plan.mix.t);
    k.a3 = k.pk.add(k.plan.mix.src);
    k.a4 = k.pk.add(k.plan.gc.upload());
    k.a5 = k.pk.reserve((size_t)P * kNumBases * sizeof(void*));
    k.oPlan = k.lay.add(k.pk.host.size());
  });
}

struct PredictCall : CallPlan {
  PredictPlan plan;
  std::vector<int64_t> sz, ov, ou;
  size_t oW = 0, oPlan = 0, a1 = 0, a2 = 0, a3 = 0;
  Packer pk;
};

std::shared_ptr<PredictCall> predict_call(idmrg_ctx* c, int P, int d, const int32_t* qp_in, const idmrg_predict* pr) {
  Hash h;
  h.val(P);
  h.arr(qp_in, d);
  for (int p = 0; p < P; ++p) {
    h.leg(pr[p].leg_a);
    h.leg(pr[p].leg_beta);
    h.leg(pr[p].leg_b);
  }
  return plan_of<PredictCall>(c, IDMRG_OP_PREDICT, h.h, [&](PredictCall& k) {
    const std::vector<int> qp = make_qp(d, qp_in);
    k.sz.assign((size_t)P * kNumBases, -1);
    for (int p = 0; p < P; ++p) {
      const Leg Aa = make_leg(pr[p].leg_a, "leg_a"), Bt = make_leg(pr[p].leg_beta, "leg_beta"),
                Bb = make_leg(pr[p].leg_b, "leg_b");
      build_predict(k.plan, p, Aa, Bt, Bb, qp);
      int64_t* z = &k.sz[(size_t)p * kNumBases];
      z[0] = Aa.total(); z[1] = z[6] = V_layout(Bt, qp, Aa).size; z[2] = Bt.total();
      z[3] = z[7] = U_layout(Bt, qp, Bb).size; z[4] = Bb.total(); z[5] = psi_layout(Aa, Bb, qp).size;
    }
    check_scale(k.plan.scale, k.sz, "predict scale", 0);
    check_gemm(k.plan.g, 2, k.sz, "predict gemm");
    int64_t n = 0;
    k.ov.assign(P, 0);
    k.ou.assign(P, 0);
    for (int p = 0; p < P; ++p) {
      k.ov[p] = n; n += k.plan.n_Vs[p] + 64;
      k.ou[p] = n; n += k.plan.n_Us[p] + 64;
    }
    k.oW = k.lay.add(n * 8);
    k.a1 = k.pk.add(k.plan.scale.t);
    k.a2 = k.pk.add(k.plan.g.upload());
    k.a3 = k.pk.reserve((size_t)P * kNumBases * sizeof(void*));
    k.oPlan = k.lay.add(k.pk.host.size());
  });
}

// ---- uniform MPS (Eq. (11)): a two-site piece as the fused site's right
// isometry, and overlaps of left and right environments

struct TwositeCall : CallPlan {
  MixList mix;
  std::vector<int64_t> sz;
  size_t oPlan = 0, a1 = 0, a2 = 0, a3 = 0;
  Packer pk;
};

std::shared_ptr<TwositeCall> twosite_call(idmrg_ctx* c, int P, int d, const int32_t* qp_in,
                                          const idmrg_twosite_item* it) {
  Hash h;
  h.val(P);
  h.arr(qp_in, d);
  for (int p = 0; p < P; ++p) {
    h.leg(it[p].left);
    h.leg(it[p].right);
  }
  return plan_of<TwositeCall>(c, IDMRG_OP_TWOSITE_V, h.h, [&](TwositeCall& k) {
    const std::vector<int> qp = make_qp(d, qp_in);
    k.sz.assign((size_t)P * kNumBases, -1);
    for (int p = 0; p < P; ++p) {
      const Leg A = make_leg(it[p].left, "twosite.left"), B = make_leg(it[p].right, "twosite.right");
      build_twosite_V(k.mix, p, A, B, qp);
      k.sz[(size_t)p * kNumBases + 0] = psi_layout(A, B, qp).size;
      k.sz[(size_t)p * kNumBases + 1] = V_layout(B, fused_qp(qp), A).size;
    }
    check_mix(k.mix, k.sz, "twosite_to_right_iso");
    k.a1 = k.pk.add(k.mix.t);
    k.a2 = k.pk.add(k.mix.src);
    k.a3 = k.pk.reserve((size_t)P * kNumBases * sizeof(void*));
    k.oPlan = k.lay.add(k.pk.host.size());
  });
}

struct OverlapCall : CallPlan {
  std::vector<OverlapSeg> segs;
  std::vector<int32_t> seg0;
  std::vector<int64_t> sz;
  size_t oPartial = 0, oOut = 0, oPlan = 0, a1 = 0, a2 = 0, a3 = 0;
  Packer pk;
};

std::shared_ptr<OverlapCall> overlap_call(idmrg_ctx* c, int P, const idmrg_overlap_item* it) {
  Hash h;
  h.val(P);
  for (int p = 0; p < P; ++p) {
    h.leg(it[p].leg);
    h.arr(it[p].ql, it[p].nl);
    h.arr(it[p].qr, it[p].nr);
    h.val(it[p].wl);
    h.val(it[p].wr);
  }
  return plan_of<OverlapCall>(c, IDMRG_OP_OVERLAP, h.h, [&](OverlapCall& k) {
    k.sz.assign((size_t)P * kNumBases, -1);
    k.seg0.assign(P + 1, 0);
    for (int p = 0; p < P; ++p) {
      const idmrg_overlap_item& o = it[p];
      if (!o.ql || !o.qr || o.nl < 2 || o.nr < 2 || o.nl > 4096 || o.nr > 4096)
        throw InvalidArg("overlap: bad channel lists");
      const Leg leg = make_leg(o.leg, "overlap.leg");
      const std::vector<int> ql(o.ql, o.ql + o.nl), qr(o.qr, o.qr + o.nr);
      k.seg0[p] = (int32_t)k.segs.size();
      build_overlap(k.segs, p, leg, ql, qr, o.wl, o.wr);
      k.sz[(size_t)p * kNumBases + 0] = envL_layout(leg, ql).size;
      k.sz[(size_t)p * kNumBases + 1] = envR_layout(leg, qr).size;
    }
    k.seg0[P] = (int32_t)k.segs.size();
    for (const OverlapSeg& g : k.segs) {
      const int64_t* z = &k.sz[(size_t)g.item * kNumBases];
      if (g.aoff < 0 || g.aoff + (int64_t)(g.rows - 1) * g.lda + g.cols > z[0] || g.boff < 0 ||
          g.boff + (int64_t)(g.rows - 1) * g.ldb + g.cols > z[1])
        throw InvalidArg("internal: overlap segment out of bounds");
    }
    k.oPartial = k.lay.add(std::max<size_t>(k.segs.size(), 1) * 8);
    k.oOut = k.lay.add((size_t)P * 8);
    k.a1 = k.pk.add(k.segs);
    k.a2 = k.pk.add(k.seg0);
    k.a3 = k.pk.reserve((size_t)P * kNumBases * sizeof(void*));
    k.oPlan = k.lay.add(k.pk.host.size());
  });
}

}  // namespace

// ------------------------------------------------------------------ context API

extern "C" int idmrg_create(idmrg_ctx** ctx, int device, void* hip_stream) {
  if (!ctx) return IDMRG_EINVAL;
  *ctx = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return IDMRG_EHIP;
  if (hipSetDevice(device) != hipSuccess) return IDMRG_EHIP;
  auto* c = new (std::nothrow) idmrg_ctx();
  if (!c) return IDMRG_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipHostMalloc((void**)&c->ring, kRingBytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return IDMRG_ENOMEM;
  }
  for (size_t i = 0; i < kRingSlotsMax + 1; ++i) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      idmrg_destroy(c);
      return IDMRG_EHIP;
    }
    c->ring_events.push_back(e);
  }
  // this device's address of the static scratch array, once per device
  if (device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        idmrg_destroy(c);
        return IDMRG_EHIP;
      }
      g_scratch_ptr[device] = p;
    }
    c->static_scratch = g_scratch_ptr[device];
  }
  *ctx = c;
  return IDMRG_OK;
}

extern "C" int idmrg_destroy(idmrg_ctx* c) {
  if (!c) return IDMRG_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& row : c->cache)
    for (auto& p : row) p.reset();
  if (c->own.p) (void)hipFree(c->own.p);
  if (c->ring) (void)hipHostFree(c->ring);
  for (auto& r : c->ring_busy) (void)hipEventDestroy(r.ev);
  for (auto e : c->ring_events) (void)hipEventDestroy(e);
  for (auto& r : c->pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (auto& row : c->tev)
    for (auto e : row)
      if (e) (void)hipEventDestroy(e);
  delete c;
  return IDMRG_OK;
}

extern "C" int idmrg_set_stream(idmrg_ctx* c, void* hip_stream) {
  if (!c) return IDMRG_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  c->stream = (hipStream_t)hip_stream;
  return IDMRG_OK;
}

extern "C" int idmrg_set_workspace(idmrg_ctx* c, void* ptr, size_t bytes) {
  return guarded(c, [&]() {
    if (!ptr) {
      c->user_ws = nullptr;
      c->user_ws_n = 0;
      return IDMRG_OK;
    }
    if (((uintptr_t)ptr & 255) != 0) throw InvalidArg("workspace must be 256-byte aligned");
    check_dev(ptr, (int64_t)bytes, 1, "workspace");
    if (c->own.p) {   // the library's own block is no longer needed
      sync(c);
      IDMRG_HIP(hipFree(c->own.p));
      c->own = DevBuf{};
    }
    c->user_ws = (char*)ptr;
    c->user_ws_n = bytes;
    return IDMRG_OK;
  });
}

extern "C" int idmrg_tune_get(idmrg_ctx* c, idmrg_tune_entry* out, int cap, int* n) {
  if (!c || !n || (cap > 0 && !out)) return IDMRG_EINVAL;
  int k = 0;
  for (const auto& kv : c->tune) {
    if (k < cap) {
      idmrg_tune_entry& e = out[k];
      e = idmrg_tune_entry{};
      e.prec = std::get<0>(kv.first);
      e.stage = std::get<1>(kv.first);
      e.log2_flops = std::get<2>(kv.first);
      e.log2_n = std::get<3>(kv.first);
      e.log2_k = std::get<4>(kv.first);
      e.tiling = kv.second;
      auto it = c->tune_ms.find(kv.first);
      for (int v = 0; v < IDMRG_TUNE_VARIANTS; ++v) e.trial_ms[v] = it != c->tune_ms.end() ? it->second[v] : -1.f;
    }
    ++k;
  }
  *n = k;
  return IDMRG_OK;
}

extern "C" int idmrg_tune_set(idmrg_ctx* c, const idmrg_tune_entry* in, int n) {
  if (!c || n < 0 || (n > 0 && !in)) return IDMRG_EINVAL;
  for (int k = 0; k < n; ++k) {
    const idmrg_tune_entry& e = in[k];
    if (e.prec < 0 || e.prec > 2 || e.stage < 0 || e.stage > 1 || e.tiling < 0 || e.tiling >= kTilings ||
        (e.tiling >= 4 && e.prec != IDMRG_PREC_BF16X3))
      return IDMRG_EINVAL;
  }
  for (int k = 0; k < n; ++k) {
    const idmrg_tune_entry& e = in[k];
    const auto key = std::make_tuple(e.prec, e.stage, e.log2_flops, e.log2_n, e.log2_k);
    c->tune[key] = e.tiling;
    c->tune_ms[key] = std::vector<float>(e.trial_ms, e.trial_ms + IDMRG_TUNE_VARIANTS);
  }
  return IDMRG_OK;
}

extern "C" int idmrg_get_stats(idmrg_ctx* c, idmrg_stats* out) {
  if (!c || !out) return IDMRG_EINVAL;
  *out = c->stats;
  return IDMRG_OK;
}

extern "C" int idmrg_profile(idmrg_ctx* c, int enable) {
  return guarded(c, [&]() {
    prof_collect(c);
    c->prof = enable != 0;
    if (enable)
      for (int k = 0; k < IDMRG_PROF_CLASSES; ++k) c->prof_n[k] = 0, c->prof_ms[k] = 0, c->prof_flops[k] = 0;
    return IDMRG_OK;
  });
}

extern "C" int idmrg_profile_get(idmrg_ctx* c, int cls, int64_t* launches, double* ms, double* flops) {
  return guarded(c, [&]() {
    if (cls < 0 || cls >= IDMRG_PROF_CLASSES || !launches || !ms || !flops) throw InvalidArg("bad profile query");
    prof_collect(c);
    *launches = c->prof_n[cls];
    *ms = c->prof_ms[cls];
    *flops = c->prof_flops[cls];
    return IDMRG_OK;
  });
}

extern "C" const char* idmrg_last_error(const idmrg_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" int64_t idmrg_psi_size(idmrg_leg A, idmrg_leg B, int32_t d, const int32_t* qp) {
  try {
    return psi_layout(make_leg(A, "A"), make_leg(B, "B"), make_qp(d, qp)).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int64_t idmrg_envL_size(idmrg_leg A, int32_t dl, const int32_t* ql) {
  try {
    if (dl < 2 || !ql) return -1;
    return envL_layout(make_leg(A, "A"), std::vector<int>(ql, ql + dl)).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int64_t idmrg_envR_size(idmrg_leg B, int32_t dr, const int32_t* qr) {
  try {
    if (dr < 2 || !qr) return -1;
    return envR_layout(make_leg(B, "B"), std::vector<int>(qr, qr + dr)).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int64_t idmrg_U_size(idmrg_leg A, int32_t d, const int32_t* qp, idmrg_leg C) {
  try {
    return U_layout(make_leg(A, "A"), make_qp(d, qp), make_leg(C, "C")).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int64_t idmrg_V_size(idmrg_leg B, int32_t d, const int32_t* qp, idmrg_leg C) {
  try {
    return V_layout(make_leg(B, "B"), make_qp(d, qp), make_leg(C, "C")).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int idmrg_heff_work(const idmrg_heff* H, double* flops, double* bytes) {
  if (!H || !flops || !bytes) return IDMRG_EINVAL;
  try {
    const Mpo W1 = make_mpo(H->w1, "w1"), W2 = make_mpo(H->w2, "w2");
    heff_work(make_leg(H->left, "left"), make_leg(H->right, "right"), W1, W2, *flops, *bytes);
    return IDMRG_OK;
  } catch (...) {
    return IDMRG_EINVAL;
  }
}

extern "C" int idmrg_workspace_size(idmrg_ctx* ctx, int op, int nprob, const void* desc, const idmrg_ws_query* q,
                                    size_t* bytes) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!desc || !q || !bytes) throw InvalidArg("null argument");
    size_t n = 0;
    switch (op) {
      case IDMRG_OP_HEFF:
        n = heff_call(ctx, nprob, (const idmrg_heff*)desc, q->prec)->lay.total;
        break;
      case IDMRG_OP_LANCZOS:
        if (!q->opts) throw InvalidArg("IDMRG_OP_LANCZOS needs the Lanczos options");
        n = lanczos_call(ctx, nprob, (const idmrg_heff*)desc, q->opts)->lay.total;
        break;
      case IDMRG_OP_TRUNCATE:
        n = trunc_call(ctx, nprob, q->d, q->qp, q->m_max, (const idmrg_trunc*)desc)->lay.total;
        break;
      case IDMRG_OP_ENV_LEFT:
      case IDMRG_OP_ENV_RIGHT:
        n = env_call(ctx, nprob, op == IDMRG_OP_ENV_LEFT ? IDMRG_LEFT : IDMRG_RIGHT,
                     (const idmrg_env_update*)desc)->lay.total;
        break;
      case IDMRG_OP_PREDICT:
        n = predict_call(ctx, nprob, q->d, q->qp, (const idmrg_predict*)desc)->lay.total;
        break;
      case IDMRG_OP_TWOSITE_V:
        n = twosite_call(ctx, nprob, q->d, q->qp, (const idmrg_twosite_item*)desc)->lay.total;
        break;
      case IDMRG_OP_OVERLAP:
        n = overlap_call(ctx, nprob, (const idmrg_overlap_item*)desc)->lay.total;
        break;
      default:
        throw InvalidArg("unknown operation");
    }
    *bytes = std::max<size_t>(n, 256);
    return IDMRG_OK;
  });
}

// ------------------------------------------------------------------ heff_apply

extern "C" int heff_apply(idmrg_ctx* ctx, int nprob, const idmrg_heff* H, const double* const* x, double* const* y,
                          int prec) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!H || !x || !y) throw InvalidArg("null argument");
    std::vector<double*> xs(nprob), ys(nprob);
    for (int p = 0; p < nprob; ++p) {
      if (!x[p] || !y[p] || x[p] == y[p]) throw InvalidArg("x and y must be distinct device pointers");
      xs[p] = const_cast<double*>(x[p]);
      ys[p] = y[p];
    }
    auto k = heff_call(ctx, nprob, H, prec);
    char* base = acquire(ctx, k->lay.total);
    heff_bind(ctx, k->ex, base, H, xs, ys);
    heff_run(ctx, k->ex, xs, ys, nullptr);
    return IDMRG_OK;
  });
}

extern "C" int heff_apply_static(idmrg_ctx* ctx, int nprob, const idmrg_heff* H, const double* const* x,
                                 double* const* y, int prec) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!H || !x || !y) throw InvalidArg("null argument");
    if (!ctx->static_scratch) throw InvalidArg("no static scratch on this device");
    std::vector<double*> xs(nprob), ys(nprob);
    for (int p = 0; p < nprob; ++p) {
      if (!x[p] || !y[p] || x[p] == y[p]) throw InvalidArg("x and y must be distinct device pointers");
      xs[p] = const_cast<double*>(x[p]);
      ys[p] = y[p];
    }
    auto k = heff_call(ctx, nprob, H, prec);
    if (k->lay.total > kStaticScratchBytes)
      throw InvalidArg("heff_apply_static: this call needs " + std::to_string(k->lay.total) +
                       " bytes of scratch; the static scratch holds " + std::to_string(kStaticScratchBytes) +
                       " (use heff_apply)");
    char* base = (char*)ctx->static_scratch;
    heff_bind(ctx, k->ex, base, H, xs, ys);
    heff_run(ctx, k->ex, xs, ys, nullptr);
    return IDMRG_OK;
  });
}

// ------------------------------------------------------------------ lanczos_solve_batch

extern "C" int lanczos_solve_batch(idmrg_ctx* ctx, int nprob, const idmrg_heff* H, double* const* psi,
                                   const idmrg_lanczos_opts* o, double* energy, idmrg_lanczos_info* info) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!H || !psi || !o || !energy || !info) throw InvalidArg("null argument");
    if (!(o->tol_E >= 0) || !(o->tol_res >= 0)) throw InvalidArg("tolerances must be >= 0");
    const int P = nprob;
    auto call = lanczos_call(ctx, P, H, o);
    LanczosCall& k = *call;
    const int kmax = k.kmax;
    const int chunk = std::max(1, o->chunk > 0 ? o->chunk : 8);
    const bool mixed = k.mixed;
    hipStream_t s = ctx->stream;
    for (int p = 0; p < P; ++p) {
      if (!psi[p]) throw InvalidArg("null psi");
      check_dev(psi[p], k.N[p], 8, "psi");
    }
    char* base = acquire(ctx, k.lay.total);
    double* V = (double*)(base + k.oV);
    const size_t nsm = (size_t)P * kmax;
    double* partial = (double*)(base + k.oSmall);
    double* alpha = partial + (size_t)P * kmax * kLzBlocks;
    double* beta = alpha + nsm;
    double* ritz = beta + nsm;
    double* coef = ritz + nsm;
    LzCtrl* ctrl = (LzCtrl*)(coef + nsm);
    double* pnorm = (double*)(ctrl + P);   // [P][kLzBlocks]
    int32_t* active = (int32_t*)(pnorm + (size_t)P * kLzBlocks);
    std::vector<double*> vv(P), ww(P);
    std::vector<LzProblem> probs(P);
    for (int p = 0; p < P; ++p) {
      vv[p] = V + k.voff[p];
      ww[p] = V + k.woff[p];
      // FP32 basis rows (first pass of a mixed solve) live in the FP64 rows' space after row 0: (kcap - 1) ld
      // floats fit in (kcap - 1) ld doubles
      float* qf = mixed && o->fp32_basis ? (float*)(V + k.qoff[p] + k.ld[p]) : nullptr;
      probs[p] = LzProblem{k.N[p], k.ld[p], V + k.qoff[p], ww[p], vv[p], psi[p], mixed ? V + k.soff[p] : nullptr, qf};
    }
    // The two plans use disjoint scratch regions, so binding the second never
    // touches what the first has uploaded.
    HeffExec& ex64 = k.ex64;
    HeffExec& exlo = k.exlo;
    heff_bind(ctx, ex64, base, H, vv, ww);
    if (mixed) heff_bind(ctx, exlo, base, H, vv, ww);
    LzProblem* dprobs = (LzProblem*)(base + k.oProbs);
    stage(ctx, dprobs, probs.data(), P * sizeof(LzProblem));

    // Mixed precision: every outer pass is a Lanczos run whose first matvec is
    // FP64 (so alpha_0 and beta_0 are the exact Rayleigh quotient and residual
    // norm of the current vector) and whose later matvecs use the low-precision
    // policy; the pass's Ritz vector starts the next pass.  A pass that stops
    // at its first step (beta_0 <= tol_res) has converged in FP64.
    // (split-bf16: swept on the YC8 m = 2048 workload with the energy-shifted
    // copies, least Lanczos time per step; three passes per solve)
    const double lowE = o->prec == IDMRG_PREC_F32 ? 1e-9 : 1e-6;
    const double lowR = o->prec == IDMRG_PREC_F32 ? 1e-5 : 5e-5;
    const int k_inner = o->prec == IDMRG_PREC_F32 ? 70 : 100;
    const int max_outer = mixed ? 16 : 1;
    // Tile autotuning: the first matvecs of the precision that does most of the
    // work try one tiling variant each (identical results), then the fastest
    // variant of each stage is kept and remembered for this shape bucket.
    HeffExec& bulk = mixed ? exlo : ex64;
    bool tuned = !(bulk.need_tune[0] || bulk.need_tune[1]);
    int trial_next = 0;
    if (!tuned)
      for (auto& row : ctx->tev)
        for (auto& e : row)
          if (!e) IDMRG_HIP(hipEventCreate(&e));
    std::vector<int32_t> going(P, 1);
    std::vector<int> iters(P, 0), fp64mv(P, 0), reorths(P, 0);
    std::vector<LzCtrl> fin(P), out(P);
    std::vector<double> ov0(P, 0.0);
    GraphSet graphs(s);
    for (int outer = 0; outer < max_outer; ++outer) {
      if (outer == 1 && mixed && o->fp32_basis) {
        // Refinement passes keep an FP64 basis: their Ritz correction must reach the final residual tolerance,
        // and rounding the basis to FP32 leaves a residual of about |H - theta| u_32 |correction|, which is near
        // 1e-8 after the first pass.  The first pass stops at a residual far above that.
        for (auto& pr : probs) pr.Qf = nullptr;
        stage(ctx, dprobs, probs.data(), P * sizeof(LzProblem));
      }
      std::vector<LzCtrl> hctrl(P);
      std::vector<int32_t> hact(P);
      int64_t maxk = 0;
      for (int p = 0; p < P; ++p) {
        LzCtrl z{};
        z.active = going[p];
        z.kcap = going[p] ? (int32_t)std::min<int64_t>(mixed && outer > 0 ? k_inner : kmax, k.kcap[p]) : 0;
        hctrl[p] = z;
        hact[p] = going[p];
        maxk = std::max<int64_t>(maxk, z.kcap);
      }
      stage(ctx, ctrl, hctrl.data(), P * sizeof(LzCtrl));
      stage(ctx, active, hact.data(), P * 4);
      lz_init(P, dprobs, ctrl, partial, kmax, s);
      if (outer == 0) {
        if (mixed)
          for (int p = 0; p < P; ++p)
            IDMRG_HIP(hipMemcpyAsync(probs[p].s0, vv[p], k.ld[p] * 8, hipMemcpyDeviceToDevice, s));
        std::vector<LzCtrl> chk(P);
        IDMRG_HIP(hipMemcpyAsync(chk.data(), ctrl, P * sizeof(LzCtrl), hipMemcpyDeviceToHost, s));
        sync(ctx);
        for (int p = 0; p < P; ++p)
          if (!(chk[p].norm0 > 0.0) || !std::isfinite(chk[p].norm0))
            throw InvalidArg("start vector has zero or non-finite norm (problem " + std::to_string(p) + ")");
      }
      const double tolE = mixed ? std::max(o->tol_E, lowE) : o->tol_E;
      const double tolR = mixed ? std::max(o->tol_res, lowR) : o->tol_res;
      const double tolF = mixed ? o->tol_res : 0.0;
      // refinement passes reduce the exact residual by a fixed factor each
      const double relF = (mixed && outer > 0) ? (o->prec == IDMRG_PREC_F32 ? 1e-4 : 2e-4) : 0.0;
      std::vector<int32_t> act(P);
      // one iteration: matvec (FP64 for the first of a mixed pass) and the vector work
      auto iteration = [&](int64_t i, int trial, hipStream_t st) {
        HeffExec& e = (!mixed || i == 0) ? ex64 : exlo;
        heff_run(ctx, e, vv, ww, active, trial);
        Prof pr(ctx, 4, 0.0);
        lz_iteration_tail(P, dprobs, ctrl, active, alpha, beta, ritz, coef, partial, pnorm, kmax, tolE, tolR, tolF,
                          relF, o->cgs2 ? 1 : 0, st);
      };
      for (int64_t it = 0; it < maxk;) {
        if (o->graph && tuned && !ctx->prof && it + chunk <= maxk) {
          // a full chunk as one graph launch; the launches depend only on whether the chunk
          // opens a mixed pass (FP64 first matvec) and on the pass's tolerances (outer > 0)
          const int key = (mixed && it == 0 ? 1 : 0) + (outer > 0 ? 2 : 0);
          if (!graphs.ex[key]) {
            const int64_t i0 = it;
            graphs.ex[key] = capture_graph(ctx, [&](hipStream_t cs) {
              for (int kk = 0; kk < chunk; ++kk) iteration(i0 + kk, -1, cs);
            });
          }
          IDMRG_HIP(hipGraphLaunch(graphs.ex[key], s));
          it += chunk;
        } else {
          for (int kk = 0; kk < chunk && it < maxk; ++kk, ++it) {
            HeffExec& e = (!mixed || it == 0) ? ex64 : exlo;
            const int trial = (!tuned && &e == &bulk && trial_next < bulk.nvar) ? trial_next++ : -1;
            iteration(it, trial, s);
          }
        }
        IDMRG_HIP(hipMemcpyAsync(act.data(), active, P * 4, hipMemcpyDeviceToHost, s));
        sync(ctx);
        if (!tuned && trial_next == bulk.nvar) {
          tune_resolve(ctx, bulk, trial_next);
          tuned = true;
        }
        if (std::all_of(act.begin(), act.end(), [](int32_t a) { return a == 0; })) break;
      }
      if (!tuned && trial_next > 0) {   // the pass ended before every variant was tried
        tune_resolve(ctx, bulk, trial_next);
        tuned = true;
      }
      lz_finish(P, dprobs, ctrl, ritz, partial, kmax, s);
      IDMRG_HIP(hipMemcpyAsync(out.data(), ctrl, P * sizeof(LzCtrl), hipMemcpyDeviceToHost, s));
      sync(ctx);
      for (int p = 0; p < P; ++p) {
        if (!going[p]) continue;
        iters[p] += out[p].iters;
        reorths[p] += out[p].reorths;
        fp64mv[p] += 1;
        if (outer == 0) ov0[p] = out[p].overlap0;
        fin[p] = out[p];
        if (!mixed || (out[p].iters == 1 && out[p].converged)) going[p] = 0;
      }
      if (std::all_of(going.begin(), going.end(), [](int32_t g) { return g == 0; })) break;
    }
    if (mixed) {
      // |<start, psi>| against the returned (refined) state
      lz_overlap(P, dprobs, ctrl, partial, kmax, s);
      IDMRG_HIP(hipMemcpyAsync(out.data(), ctrl, P * sizeof(LzCtrl), hipMemcpyDeviceToHost, s));
      sync(ctx);
      for (int p = 0; p < P; ++p) ov0[p] = out[p].overlap0;
    }
    if (!mixed) {
      // FP64 residual of the result: w = H psi (v holds psi after lz_finish)
      heff_run(ctx, ex64, vv, ww, nullptr);
      lz_residual(P, dprobs, ctrl, partial, kmax, s);
      IDMRG_HIP(hipMemcpyAsync(out.data(), ctrl, P * sizeof(LzCtrl), hipMemcpyDeviceToHost, s));
      sync(ctx);
      for (int p = 0; p < P; ++p) fin[p].residual = out[p].residual;
    }
    int rc = IDMRG_OK;
    for (int p = 0; p < P; ++p) {
      energy[p] = fin[p].theta;
      info[p].overlap0 = ov0[p];
      info[p].iters = iters[p];
      info[p].converged = mixed ? (going[p] ? 0 : 1) : fin[p].converged;
      info[p].fp64_matvecs = mixed ? fp64mv[p] : 0;
      info[p].flags = fin[p].flags;
      info[p].reorth_passes = reorths[p];
      info[p].reserved = 0;
      info[p].residual = fin[p].residual;
      if (!std::isfinite(fin[p].theta) || !std::isfinite(fin[p].residual)) {
        ctx->err = "non-finite energy or residual (problem " + std::to_string(p) + ")";
        return IDMRG_ENUMERIC;
      }
      if (!info[p].converged) rc = IDMRG_WARN_NOCONV;
    }
    return rc;
  });
}

// ------------------------------------------------------------------ truncate_twosite

extern "C" int truncate_twosite(idmrg_ctx* ctx, int nprob, int32_t d, const int32_t* qp_in, int32_t m_max,
                                double lam_floor, double deg_rel, idmrg_trunc* t) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!t || m_max < 1 || !(lam_floor >= 0) || !(deg_rel >= 0)) throw InvalidArg("bad truncation arguments");
    const int P = nprob;
    for (int p = 0; p < P; ++p)
      if (!t[p].psi) throw InvalidArg("null psi");
    auto call = trunc_call(ctx, P, d, qp_in, m_max, t);
    TruncCall& k = *call;
    hipStream_t s = ctx->stream;
    for (int p = 0; p < P; ++p) check_dev(t[p].psi, k.X[p].size, 8, "psi");
    std::vector<SelTask> sel = k.sel;   // the floor and the guard are arguments of the call, not of the plan
    for (auto& st : sel) {
      st.lam_floor = lam_floor;
      st.deg_rel = deg_rel;
    }
    k.pk.patch(k.a4, sel);
    char* base = acquire(ctx, k.lay.total);
    double* dM = (double*)(base + k.oSvd);
    double* dX = dM + k.nM + 64;
    double* dG = dX + k.nX + 64;
    double* dU = dG + k.nG + 64;
    double* dV = dU + k.nU + 64;
    double* dS = dV + k.nV + 64;
    const int64_t nS = k.nS;
    char* sw = base + k.oSel;
    int32_t* colmap = (int32_t*)sw;
    double* lam_sel = (double*)(sw + ((size_t)k.ncand_tot * 4 + 255) / 256 * 256);
    int32_t* kept = (int32_t*)((char*)lam_sel + ((size_t)k.ncand_tot * 8 + 255) / 256 * 256);
    double* scal = (double*)((char*)kept + (k.ssec.size() * 4 + 255) / 256 * 256);
    std::vector<void*> hb((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      void** b = &hb[(size_t)p * kNumBases];
      b[0] = (void*)t[p].psi; b[1] = dM; b[2] = dX; b[3] = dG; b[4] = dU; b[5] = dV; b[6] = dS;
    }
    k.pk.patch(k.a6, hb);
    char* dev = base + k.oPlan;
    stage(ctx, dev, k.pk.host.data(), k.pk.host.size());
    int svd_sweeps = 0, svd_conv = 1;
    std::vector<int32_t> completed(P, 1);
    int32_t* dflag = (int32_t*)(base + k.oFlag);
    {
      Prof pr(ctx, 6, 0.0);
      launch_mix(0, 0, (MixTask*)(dev + k.a1), (MixSrc*)(dev + k.a2), (int)k.gather.t.size(), k.gather.tiles,
                 (void**)(dev + k.a6), nullptr, s);
      // non-finite input is reported, not decomposed (the Jacobi norms would hide it)
      IDMRG_HIP(hipMemsetAsync(dflag, 0, 4, s));
      launch_check_finite(dM, k.nM, dflag, s);
    }
    {
      Prof pr(ctx, 5, 0.0);
      BjScratch scr;
      scr.tol = std::max(1e-15, 4.4e-16 * std::sqrt((double)k.pmax));
      // null rows: at most 1e-15 .. 1e-14 of their block's norm (rounding residue); never
      // above lam_floor, so that a null row never ranks as a nonzero value unless lam_floor
      // itself is below 1e-15
      scr.zero_rel = std::min(std::max(lam_floor, 1e-15), 1e-14);
      // Null rows (sigma <= zero_rel |M_q|_F) need a completed direction only if the
      // selection can keep one.  Zero-weight states are kept only when every candidate is
      // (m_max >= candidates); otherwise a null row is kept only if it ranks as a nonzero
      // value, which needs lam_floor < zero_rel.  "above" counts conservatively the rows
      // with sigma / |sigma| above zero_rel (1 + 1e-9), which no null row reaches: when all
      // of the kept states are among them, no completion is needed.
      scr.need_completion = [&](std::vector<int32_t>& complete) {
        std::vector<double> hS(nS);
        IDMRG_HIP(hipMemcpyAsync(hS.data(), dS, nS * 8, hipMemcpyDeviceToHost, s));
        sync(ctx);
        std::vector<double> tot(P, 0.0);
        std::vector<int64_t> cand(P, 0), above(P, 0);
        for (const auto& sv : k.svd) {
          const int n = std::min(sv.r, sv.c);
          cand[sv.prob] += n;
          for (int i = 0; i < n; ++i) tot[sv.prob] += hS[sv.s_off + i] * hS[sv.s_off + i];
        }
        const double thr = scr.zero_rel * (1.0 + 1e-9);
        for (const auto& sv : k.svd) {
          const int n = std::min(sv.r, sv.c);
          const double cut = thr * std::sqrt(tot[sv.prob]);
          for (int i = 0; i < n; ++i) above[sv.prob] += hS[sv.s_off + i] > cut;
        }
        for (int pr = 0; pr < P; ++pr) {
          const bool all_kept = m_max >= cand[pr];
          const bool null_may_rank = lam_floor < scr.zero_rel;
          completed[pr] = !(tot[pr] > 0.0 && (all_kept ? above[pr] >= cand[pr]
                                                       : (!null_may_rank || above[pr] >= m_max)));
        }
        for (size_t m = 0; m < k.svd.size(); ++m) complete[m] = completed[k.svd[m].prob];
      };
      char* bjdev = base + k.oBjPlan;
      stage(ctx, bjdev, k.bj.host.data(), k.bj.host.size());
      bj_svd(k.bj, (void**)(dev + k.a6), (SvdTask*)(dev + k.a3), scr, s, bjdev, base + k.oBjWork,
             [&]() { sync(ctx); });
      svd_sweeps = scr.sweeps;
      svd_conv = scr.converged;
    }
    {
      Prof pr(ctx, 6, 0.0);
      launch_select((SelTask*)(dev + k.a4), (int)sel.size(), (SelSector*)(dev + k.a5), dS, kept, colmap, lam_sel,
                    scal, s);
    }
    IDMRG_HIP(hipGetLastError());
    std::vector<int32_t> hkept(k.ssec.size());
    std::vector<double> hscal(4 * (size_t)P);
    int32_t hflag = 0;
    IDMRG_HIP(hipMemcpyAsync(hkept.data(), kept, hkept.size() * 4, hipMemcpyDeviceToHost, s));
    IDMRG_HIP(hipMemcpyAsync(hscal.data(), scal, hscal.size() * 8, hipMemcpyDeviceToHost, s));
    IDMRG_HIP(hipMemcpyAsync(&hflag, dflag, 4, hipMemcpyDeviceToHost, s));
    sync(ctx);
    if (hflag) {
      ctx->err = "the two-site state holds NaN or infinite values";
      return IDMRG_ENUMERIC;
    }
    // outputs
    ScaleList outl;
    std::vector<void*> ob((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      const SelTask& st = sel[p];
      Leg C;
      std::vector<int> which;
      for (int q = 0; q < st.nsec; ++q)
        if (hkept[st.sec0 + q] > 0) {
          C.q.push_back(k.ssec[st.sec0 + q].charge);
          C.dim.push_back(hkept[st.sec0 + q]);
          which.push_back(q);
        }
      if (C.n() > t[p].cap_sec || !t[p].q_out || !t[p].dim_out) throw InvalidArg("new-leg capacity too small");
      const IsoLayout U = U_layout(k.A[p], k.qp, C), Vl = V_layout(k.B[p], k.qp, C);
      if (U.size > t[p].cap_U || Vl.size > t[p].cap_V || C.total() > t[p].cap_lam)
        throw InvalidArg("output capacity too small (U, V or lambda)");
      if (!t[p].U || !t[p].V || !t[p].lambda) throw InvalidArg("null output buffer");
      void** b = &ob[(size_t)p * kNumBases];
      b[0] = dU; b[1] = dV; b[2] = lam_sel; b[3] = t[p].U; b[4] = t[p].V; b[5] = t[p].lambda;
      int64_t loff = 0;
      for (int ci = 0; ci < C.n(); ++ci) {
        const TruncSec& S = k.secs[p][which[ci]];
        const SelSector& se = k.ssec[st.sec0 + which[ci]];
        const int n = se.n, kk = C.dim[ci];
        if (U.rows[ci] != S.r || Vl.rows[ci] != S.c) throw InvalidArg("internal: isometry row mismatch");
        ScaleTask a{};
        a.rows = S.r; a.cols = kk; a.lds = n; a.ldd = kk; a.prob = p; a.sbase = 0; a.dbase = 3; a.rbase = -1;
        a.cbase = -1; a.colmap = se.cand0; a.soff = S.u; a.doff = U.off[ci];
        outl.add(a);
        ScaleTask v = a;
        v.rows = S.c; v.sbase = 1; v.dbase = 4; v.soff = S.v; v.doff = Vl.off[ci];
        outl.add(v);
        ScaleTask l{};
        l.rows = 1; l.cols = kk; l.lds = kk; l.ldd = kk; l.prob = p; l.sbase = 2; l.dbase = 5; l.rbase = -1;
        l.cbase = -1; l.colmap = -1; l.soff = se.cand0; l.doff = loff;
        outl.add(l);
        loff += kk;
        t[p].q_out[ci] = C.q[ci];
        t[p].dim_out[ci] = kk;
      }
      t[p].nsec_out = C.n();
      t[p].eps = hscal[4 * p + 0];
      t[p].eps_prime = hscal[4 * p + 1];
      t[p].cut_gap = hscal[4 * p + 2];
      t[p].m_kept = (int32_t)hscal[4 * p + 3];
      t[p].svd_sweeps = svd_sweeps;
      t[p].svd_converged = svd_conv;
      t[p].null_completed = completed[p];
      t[p].reserved = 0;
    }
    {
      std::vector<int64_t> sz((size_t)P * kNumBases, -1);
      for (int p = 0; p < P; ++p) {
        int64_t* z = &sz[(size_t)p * kNumBases];
        z[0] = k.nU; z[1] = k.nV; z[2] = k.ncand_tot; z[3] = t[p].cap_U; z[4] = t[p].cap_V; z[5] = t[p].cap_lam;
        check_dev(t[p].U, t[p].cap_U, 8, "U");
        check_dev(t[p].V, t[p].cap_V, 8, "V");
        check_dev(t[p].lambda, t[p].cap_lam, 8, "lambda");
      }
      check_scale(outl, sz, "truncation output", k.ncand_tot);
    }
    Packer pk2;
    const size_t b1 = pk2.add(outl.t), b2 = pk2.add(ob);
    if (pk2.host.size() > k.outBytes) throw InvalidArg("internal: output plan larger than reserved");
    char* dev2 = base + k.oOut;
    stage(ctx, dev2, pk2.host.data(), pk2.host.size());
    {
      Prof pr(ctx, 6, 0.0);
      launch_scale((ScaleTask*)(dev2 + b1), colmap, (int)outl.t.size(), outl.tiles, 0.0, (void**)(dev2 + b2), s);
    }
    IDMRG_HIP(hipGetLastError());
    sync(ctx);
    for (int p = 0; p < P; ++p)
      if (!std::isfinite(t[p].eps)) {
        ctx->err = "non-finite singular values";
        return IDMRG_ENUMERIC;
      }
    if (!svd_conv) {
      ctx->err = "Jacobi SVD did not converge in " + std::to_string(svd_sweeps) + " sweeps";
      return IDMRG_WARN_NOCONV;
    }
    return IDMRG_OK;
  });
}

// ------------------------------------------------------------------ update_env

extern "C" int update_env(idmrg_ctx* ctx, int nprob, int side, const idmrg_env_update* u) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!u || (side != IDMRG_LEFT && side != IDMRG_RIGHT)) throw InvalidArg("bad update_env arguments");
    const int P = nprob;
    for (int p = 0; p < P; ++p)
      if (!u[p].env_old || !u[p].iso || !u[p].env_new) throw InvalidArg("null buffer in idmrg_env_update");
    auto call = env_call(ctx, P, side, u);
    EnvCall& k = *call;
    for (int p = 0; p < P; ++p) {
      const int64_t* z = &k.sz[(size_t)p * kNumBases];
      check_dev(u[p].env_old, z[0], 8, "env_old");
      check_dev(u[p].iso, z[1], 8, "iso");
      check_dev(u[p].env_new, z[2], 8, "env_new");
    }
    char* base = acquire(ctx, k.lay.total);
    double* ws = (double*)(base + k.oT);
    std::vector<void*> hb((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      void** b = &hb[(size_t)p * kNumBases];
      b[0] = (void*)u[p].env_old; b[1] = (void*)u[p].iso; b[2] = u[p].env_new;
      b[3] = ws + k.o1[p]; b[4] = ws + k.n1 + k.o2[p];
    }
    k.pk.patch(k.a5, hb);
    char* dev = base + k.oPlan;
    stage(ctx, dev, k.pk.host.data(), k.pk.host.size());
    void** bases = (void**)(dev + k.a5);
    hipStream_t s = ctx->stream;
    Prof pr(ctx, 7, k.plan.ga.flops() + k.plan.gc.flops() + k.plan.mix.flops());
    launch_gemm(Prec::F64, side == IDMRG_LEFT ? 0 : 2, (GemmTask*)(dev + k.a1), (int)k.plan.ga.t.size(),
                k.plan.ga.tiles, k.plan.ga.xmax, bases, nullptr, s);
    launch_mix(0, 0, (MixTask*)(dev + k.a2), (MixSrc*)(dev + k.a3), (int)k.plan.mix.t.size(), k.plan.mix.tiles,
               bases, nullptr, s);
    launch_gemm(Prec::F64, side == IDMRG_LEFT ? 2 : 0, (GemmTask*)(dev + k.a4), (int)k.plan.gc.t.size(),
                k.plan.gc.tiles, k.plan.gc.xmax, bases, nullptr, s);
    IDMRG_HIP(hipGetLastError());
    return IDMRG_OK;
  });
}

// ------------------------------------------------------------------ predict_wavefunction

extern "C" int predict_wavefunction(idmrg_ctx* ctx, int nprob, int32_t d, const int32_t* qp_in, double lam_floor,
                                    const idmrg_predict* pr) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!pr || !(lam_floor >= 0)) throw InvalidArg("bad predict arguments");
    const int P = nprob;
    for (int p = 0; p < P; ++p)
      if (!pr[p].lam_i || !pr[p].V_i || !pr[p].lam_prev || !pr[p].U_ip1 || !pr[p].lam_ip1 || !pr[p].psi)
        throw InvalidArg("null buffer in idmrg_predict");
    auto call = predict_call(ctx, P, d, qp_in, pr);
    PredictCall& k = *call;
    for (int p = 0; p < P; ++p) {
      const int64_t* z = &k.sz[(size_t)p * kNumBases];
      check_dev(pr[p].lam_i, z[0], 8, "lam_i");
      check_dev(pr[p].V_i, z[1], 8, "V_i");
      check_dev(pr[p].lam_prev, z[2], 8, "lam_prev");
      check_dev(pr[p].U_ip1, z[3], 8, "U_ip1");
      check_dev(pr[p].lam_ip1, z[4], 8, "lam_ip1");
      check_dev(pr[p].psi, z[5], 8, "psi");
    }
    char* base = acquire(ctx, k.lay.total);
    double* ws = (double*)(base + k.oW);
    std::vector<void*> hb((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      void** b = &hb[(size_t)p * kNumBases];
      b[0] = (void*)pr[p].lam_i; b[1] = (void*)pr[p].V_i; b[2] = (void*)pr[p].lam_prev; b[3] = (void*)pr[p].U_ip1;
      b[4] = (void*)pr[p].lam_ip1; b[5] = pr[p].psi; b[6] = ws + k.ov[p]; b[7] = ws + k.ou[p];
    }
    k.pk.patch(k.a3, hb);
    char* dev = base + k.oPlan;
    stage(ctx, dev, k.pk.host.data(), k.pk.host.size());
    void** bases = (void**)(dev + k.a3);
    Prof prf(ctx, 8, k.plan.g.flops());
    launch_scale((ScaleTask*)(dev + k.a1), nullptr, (int)k.plan.scale.t.size(), k.plan.scale.tiles, lam_floor, bases,
                 ctx->stream);
    launch_gemm(Prec::F64, 2, (GemmTask*)(dev + k.a2), (int)k.plan.g.t.size(), k.plan.g.tiles, k.plan.g.xmax, bases,
                nullptr, ctx->stream);
    IDMRG_HIP(hipGetLastError());
    return IDMRG_OK;
  });
}

// ------------------------------------------------------------------ uniform MPS

extern "C" int twosite_to_right_iso(idmrg_ctx* ctx, int nitem, int32_t d, const int32_t* qp_in,
                                    const idmrg_twosite_item* items) {
  return guarded(ctx, [&]() {
    check_nprob(nitem);
    if (!items) throw InvalidArg("null items");
    for (int p = 0; p < nitem; ++p)
      if (!items[p].psi || !items[p].out || (const double*)items[p].out == items[p].psi)
        throw InvalidArg("twosite_to_right_iso: psi and out must be distinct device buffers");
    auto call = twosite_call(ctx, nitem, d, qp_in, items);
    TwositeCall& k = *call;
    for (int p = 0; p < nitem; ++p) {
      check_dev(items[p].psi, k.sz[(size_t)p * kNumBases + 0], 8, "psi");
      check_dev(items[p].out, k.sz[(size_t)p * kNumBases + 1], 8, "out");
    }
    char* base = acquire(ctx, k.lay.total);
    std::vector<void*> hb((size_t)nitem * kNumBases, nullptr);
    for (int p = 0; p < nitem; ++p) {
      hb[(size_t)p * kNumBases + 0] = (void*)items[p].psi;
      hb[(size_t)p * kNumBases + 1] = items[p].out;
    }
    k.pk.patch(k.a3, hb);
    char* dev = base + k.oPlan;
    stage(ctx, dev, k.pk.host.data(), k.pk.host.size());
    launch_mix(0, 0, (MixTask*)(dev + k.a1), (MixSrc*)(dev + k.a2), (int)k.mix.t.size(), k.mix.tiles,
               (void* const*)(dev + k.a3), nullptr, ctx->stream);
    IDMRG_HIP(hipGetLastError());
    return IDMRG_OK;
  });
}

extern "C" int env_overlap(idmrg_ctx* ctx, int nitem, const idmrg_overlap_item* items, double* out) {
  return guarded(ctx, [&]() {
    check_nprob(nitem);
    if (!items || !out) throw InvalidArg("null argument");
    for (int p = 0; p < nitem; ++p)
      if (!items[p].L || !items[p].R) throw InvalidArg("env_overlap: null environment");
    auto call = overlap_call(ctx, nitem, items);
    OverlapCall& k = *call;
    for (int p = 0; p < nitem; ++p) {
      check_dev(items[p].L, k.sz[(size_t)p * kNumBases + 0], 8, "L");
      check_dev(items[p].R, k.sz[(size_t)p * kNumBases + 1], 8, "R");
    }
    char* base = acquire(ctx, k.lay.total);
    std::vector<void*> hb((size_t)nitem * kNumBases, nullptr);
    for (int p = 0; p < nitem; ++p) {
      hb[(size_t)p * kNumBases + 0] = (void*)items[p].L;
      hb[(size_t)p * kNumBases + 1] = (void*)items[p].R;
    }
    k.pk.patch(k.a3, hb);
    char* dev = base + k.oPlan;
    stage(ctx, dev, k.pk.host.data(), k.pk.host.size());
    double* dout = (double*)(base + k.oOut);
    launch_overlap((const OverlapSeg*)(dev + k.a1), (int)k.segs.size(), (const int32_t*)(dev + k.a2), nitem,
                   (void* const*)(dev + k.a3), (double*)(base + k.oPartial), dout, ctx->stream);
    IDMRG_HIP(hipGetLastError());
    IDMRG_HIP(hipMemcpyAsync(out, dout, (size_t)nitem * 8, hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    for (int p = 0; p < nitem; ++p)
      if (!std::isfinite(out[p])) {
        ctx->err = "non-finite overlap (item " + std::to_string(p) + ")";
        return IDMRG_ENUMERIC;
      }
    return IDMRG_OK;
  });
}
