// libnmc runtime and C ABI: context, tables, Green-spectrum cache, workspace
// pool, the batched nested solve, and the continuous-batching serving loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/nmc.h"
#include "kernels.h"
#include "serve_core.hpp"

namespace {

using nmc::FieldDesc;
using nmc::FieldTable;
using nmc::PassGeom;

constexpr int kMinN = 4;
constexpr int kMaxL = 16;
constexpr int kMaxP = 512;         // level grids: N <= 256
constexpr int kMaxScaledP = 1024;  // doubled grids of N = 256, quadrupled grids of N = 128
constexpr size_t kAlign = 256;
constexpr int kServeStreams = 4;
constexpr int kMaxBatchRequests = 32;
constexpr int kMaxDevices = 64;

size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

int period_of(int N) {
  if (N < kMinN || N % 4 != 0) return 0;
  int P = 8;
  while (P < 2 * N) P *= 2;
  return P <= kMaxP ? P : 0;
}

size_t real_size(nmc_precision p) { return p == NMC_F64 ? 8 : 4; }

// Two ways to obtain the hole potentials of Sect. 4 on the stencil box:
//  * hole grids (kind 2): each level with its child region zeroed, carried by
//    a small cascade S_n = Prolong(S_{n-1}) + Phi^n_hole;
//  * child-region boxes (kind 1): the child region alone in an (N/2+2)^3 box,
//    Phi_hole = Phi - C, and S_l = Phi(Omega^l) - C_l left by the last pass of
//    level l.  Cheaper grids but one last-pass launch per level, which pays
//    from N = 128 up (measured).
bool use_boxes(int N) { return N >= 128; }

// The modified method (Sect. 7, Appendix B) convolves a doubled grid per
// level pair on twice the period; it uses the hole-grid formulation.
bool is_modified(unsigned flags) { return (flags & (NMC_MODIFIED | NMC_MODIFIED3)) != 0; }
// The three-level scheme of Appendix B adds a quadrupled grid (period 4P)
// per level with two finer levels.
bool is_modified3(unsigned flags, int L) { return (flags & NMC_MODIFIED3) != 0 && L >= 3; }
// Which method a request uses (requests of one group share every launch):
// original / modified / three-level, times two carry rules.
int method_of(unsigned flags) {
  const int m = (flags & NMC_MODIFIED3) ? 2 : (flags & NMC_MODIFIED) ? 1 : 0;
  return m + ((flags & NMC_PROLONG_TRILINEAR) ? 3 : 0);
}
// Largest period a solve with these flags needs.
int max_period(int N, int L, unsigned flags) {
  const int P = period_of(N);
  return is_modified3(flags, L) ? 4 * P : is_modified(flags) ? 2 * P : P;
}

// Workspace layout of one request (offsets from its base): per level l the
// full grid's A and B; per level l < L-1 the second grid (hole grid,
// child-region box, or with the modified method the doubled grid), the
// restriction data Rc (the block-mean pyramid of level l+1, or the cascaded
// restriction in its first (N/2)^3 values), the box potential (hole
// potential or C) and the carried potential S (hi, and lo for the FP32
// path).  With the modified method the "full" grids of levels l < L-1 are
// the hole grids with full output.
struct Layout {
  int N, L, P, NC;
  bool boxes, mod, mod3;
  size_t r, c;
  size_t a_full, b_full, a_sec, b_sec, rc_bytes, box_bytes, a_q, b_q;
  size_t total;
  size_t A(int l) const { return (size_t)l * (a_full + b_full); }
  size_t B(int l) const { return A(l) + a_full; }
  size_t full_end() const { return (size_t)L * (a_full + b_full); }
  size_t As(int l) const { return full_end() + (size_t)l * (a_sec + b_sec); }
  size_t Bs(int l) const { return As(l) + a_sec; }
  size_t sec_end() const { return full_end() + (size_t)(L - 1) * (a_sec + b_sec); }
  size_t Rc(int l) const { return sec_end() + (size_t)l * rc_bytes; }
  size_t Box(int l) const { return Rc(0) + (size_t)(L - 1) * rc_bytes + (size_t)l * box_bytes; }
  size_t Shi(int l) const { return Box(0) + (size_t)(L - 1) * box_bytes + (size_t)l * 2 * box_bytes; }
  size_t Slo(int l) const { return Shi(l) + box_bytes; }
  // quadrupled grids of the three-level scheme, levels l < L-2
  size_t Aq(int l) const { return Shi(0) + (size_t)(L - 1) * 2 * box_bytes + (size_t)l * (a_q + b_q); }
  size_t Bq(int l) const { return Aq(l) + a_q; }
};

Layout make_layout(int N, int L, nmc_precision p, unsigned flags) {
  Layout lo{};
  lo.N = N;
  lo.L = L;
  lo.P = period_of(N);
  lo.NC = N / 2 + 2;
  lo.mod = is_modified(flags);
  lo.mod3 = is_modified3(flags, L);
  lo.boxes = use_boxes(N) && !lo.mod;
  lo.r = real_size(p);
  lo.c = 2 * lo.r;
  const size_t P = lo.P, NC = lo.NC, ns = lo.boxes ? NC : (size_t)N;
  lo.a_full = align_up((size_t)N * N * (P / 2) * lo.c);
  lo.b_full = align_up((size_t)N * nmc::zrow_pitch((int)P, lo.c) * lo.c);
  if (lo.mod) {
    // doubled grid, period 2P: N x N rows of the x half spectrum (P values;
    // x-pass output and folded y-inverse output), N z rows (y-pass output,
    // folded z-pass output in place)
    const size_t PD = 2 * P;
    lo.a_sec = align_up((size_t)N * N * (PD / 2) * lo.c);
    lo.b_sec = align_up((size_t)N * nmc::zrow_pitch((int)PD, lo.c) * lo.c);
  } else {
    lo.a_sec = align_up(ns * ns * (P / 2) * lo.c);
    lo.b_sec = align_up(ns * nmc::zrow_pitch((int)P, lo.c) * lo.c);
  }
  lo.rc_bytes = align_up((size_t)nmc::pyramid_slab(N, L) * lo.r);
  lo.box_bytes = align_up(NC * NC * NC * lo.r);
  if (lo.mod3) {
    // quadrupled grid, period 4P: N x N rows of the x half spectrum (2P
    // values), N z rows
    const size_t PQ = 4 * P;
    lo.a_q = align_up((size_t)N * N * (PQ / 2) * lo.c);
    lo.b_q = align_up((size_t)N * nmc::zrow_pitch((int)PQ, lo.c) * lo.c);
  }
  lo.total = lo.Aq(0) + (lo.mod3 ? (size_t)(L - 2) * (lo.a_q + lo.b_q) : 0);
  lo.total = std::max(lo.total, kAlign);
  return lo;
}

struct Req {
  const void* rho;
  void* phi;
  int N, L;
  double h0, G;
  nmc_precision p;
  unsigned flags;
};

struct Block {
  void* ptr;
  size_t bytes;
};

struct Lease {
  std::vector<Block> blocks;
  hipEvent_t ev = nullptr;
  bool in_arena = false;  // a serving batch's region of the serving arena
};

struct PerP {
  void* tw64 = nullptr;  // double2[P]
  void* tw32 = nullptr;  // float2[P]
  double* g64 = nullptr;  // spectrum octant [kz][ky][kx]
  float* g32 = nullptr;
  double *gz64 = nullptr, *gn64 = nullptr;  // z-pass layouts
  float *gz32 = nullptr, *gn32 = nullptr;
  size_t bytes = 0;   // device bytes of the spectrum tables (0 while not built)
  uint64_t used = 0;  // last use (context clock), for the LRU eviction
};

// A serving request as the device side needs it: the solve and the event
// recorded on the submitting stream (its rho is written and its phi free once
// the event has completed).
struct ServeReq {
  Req r;
  hipEvent_t ready = nullptr;
};

// A repeated nmc_solve call, identified by every argument.
struct GraphKey {
  const void* rho;
  void* phi;
  int N, L;
  double h0, G;
  int p;
  unsigned flags;
  bool operator<(const GraphKey& o) const {
    return std::memcmp(this, &o, sizeof(GraphKey)) < 0;
  }
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  Block ws{};
  hipEvent_t last = nullptr;  // completion of the latest replay
  uint64_t used = 0;
};

constexpr size_t kMaxGraphs = 8;

}  // namespace

struct nmc_ctx {
  int device = 0;
  size_t budget = 0;
  std::string err = "no error";
  std::map<int, PerP> perp;
  size_t green_bytes = 0;  // Green tables held (counted against the budget)
  // workspace pool
  std::vector<Block> free_blocks;
  std::deque<Lease> leases;  // outstanding (event not yet observed complete)
  size_t allocated = 0;      // pool + leased
  // serving: the scheduler core (host logic) and the device side's records
  std::unique_ptr<nmc::ServeCore> serve;
  std::unordered_map<uint64_t, ServeReq> sreq;
  hipStream_t streams[kServeStreams] = {};
  int next_stream = 0;
  std::vector<hipEvent_t> ev_pool;  // reusable submit events
  char* arena_base = nullptr;        // serving workspace under a budget: one allocation
  nmc::RingArena arena;              // and its regions in use
  // second stream of a solve (hole grids and carry cascade) and its fork/join events
  hipStream_t aux_stream = nullptr;
  // this device's static scratch array (nmc_solve_noalloc)
  char* scratch = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // captured solves
  hipStream_t cap_stream = nullptr;
  std::map<GraphKey, GraphEntry> graphs;
  std::map<GraphKey, int> seen;
  uint64_t clock = 0;
  // per-pass profiling
  bool profiling = false;
  struct ProfRec {
    int pass;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<ProfRec> prof;
};

namespace {

int fail(nmc_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_fail(nmc_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, NMC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define NMC_HIP(ctx, call)                         \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

// --- tables ------------------------------------------------------------------

int ensure_twiddles(nmc_ctx* ctx, int P, PerP& pp) {
  if (pp.tw64) return NMC_OK;
  std::vector<double> t64(2 * P);
  std::vector<float> t32(2 * P);
  // exp(-2 pi i j / P), evaluated in long double and rounded once per type
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int j = 0; j < P; ++j) {
    const long double a = two_pi * (long double)j / (long double)P;
    const long double c = cosl(a), s = -sinl(a);
    t64[2 * j] = (double)c;
    t64[2 * j + 1] = (double)s;
    t32[2 * j] = (float)c;
    t32[2 * j + 1] = (float)s;
  }
  // the tables are published only when both are complete: a failed call
  // leaves none behind, and the next call builds them again
  void *d64 = nullptr, *d32 = nullptr;
  hipError_t e = hipMalloc(&d64, sizeof(double) * 2 * P);
  if (e == hipSuccess) e = hipMalloc(&d32, sizeof(float) * 2 * P);
  if (e == hipSuccess) e = hipMemcpy(d64, t64.data(), sizeof(double) * 2 * P, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d32, t32.data(), sizeof(float) * 2 * P, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d64);
    (void)hipFree(d32);
    return hip_fail(ctx, e, "twiddle tables");
  }
  pp.tw64 = d64;
  pp.tw32 = d32;
  return NMC_OK;
}

// Self-cell integral of 1/r over the unit cube (Eq. 13 of the paper):
// 3 ln(2 + sqrt 3) - pi / 2.
double self_cell_integral() {
  const long double pi = 3.141592653589793238462643383279502884L;
  return (double)(3.0L * logl(2.0L + sqrtl(3.0L)) - pi / 2.0L);
}

// Device bytes of the Green tables of period P: the FP64 and FP32 spectrum
// octants and their z-pass layouts (the twiddles are small and not counted).
size_t green_table_bytes(int P) {
  const size_t H = P / 2 + 1;
  return H * H * H * 12 + (nmc::green_layout_elems<double>(P) + H * H) * 8 +
         (nmc::green_layout_elems<float>(P) + H * H) * 4;
}

int ensure_green(nmc_ctx* ctx, int P, hipStream_t s) {
  PerP& pp = ctx->perp[P];
  int rc = ensure_twiddles(ctx, P, pp);
  if (rc) return rc;
  if (pp.g64) return NMC_OK;
  const size_t H = P / 2 + 1, n = H * H * H;
  double *t1 = nullptr, *t2 = nullptr;
  const size_t nz64 = nmc::green_layout_elems<double>(P), nz32 = nmc::green_layout_elems<float>(P);
  // pp.g64 marks the tables as built: on any failure below every table is
  // freed and its pointer cleared, so a later call builds the set again
  hipError_t e = hipSuccess;
  for (auto [ptr, bytes] : {std::pair<void**, size_t>{(void**)&pp.g64, n * sizeof(double)},
                            {(void**)&pp.g32, n * sizeof(float)},
                            {(void**)&t1, n * sizeof(double)},
                            {(void**)&t2, n * sizeof(double)},
                            {(void**)&pp.gz64, nz64 * sizeof(double)},
                            {(void**)&pp.gn64, H * H * sizeof(double)},
                            {(void**)&pp.gz32, nz32 * sizeof(float)},
                            {(void**)&pp.gn32, H * H * sizeof(float)}})
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  if (e == hipSuccess) e = nmc::launch_green(P, self_cell_integral(), (const double2*)pp.tw64, t1, t2, pp.g64, s);
  if (e == hipSuccess) e = nmc::launch_round_f32(pp.g64, pp.g32, n, s);
  if (e == hipSuccess) e = nmc::launch_green_layout<double>(P, pp.g64, pp.gz64, pp.gn64, s);
  if (e == hipSuccess) e = nmc::launch_green_layout<float>(P, pp.g64, pp.gz32, pp.gn32, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(t1);
  (void)hipFree(t2);
  if (e != hipSuccess) {
    for (void* q : {(void*)pp.g64, (void*)pp.g32, (void*)pp.gz64, (void*)pp.gn64, (void*)pp.gz32, (void*)pp.gn32})
      (void)hipFree(q);
    pp.g64 = nullptr;
    pp.g32 = nullptr;
    pp.gz64 = pp.gn64 = nullptr;
    pp.gz32 = pp.gn32 = nullptr;
    return hip_fail(ctx, e, "green spectrum build");
  }
  pp.bytes = green_table_bytes(P);
  ctx->green_bytes += pp.bytes;
  return NMC_OK;
}

void free_green(nmc_ctx* ctx, PerP& pp) {
  for (void* q : {(void*)pp.g64, (void*)pp.g32, (void*)pp.gz64, (void*)pp.gn64, (void*)pp.gz32, (void*)pp.gn32})
    (void)hipFree(q);
  pp.g64 = nullptr;
  pp.g32 = nullptr;
  pp.gz64 = pp.gn64 = nullptr;
  pp.gz32 = pp.gn32 = nullptr;
  ctx->green_bytes -= pp.bytes;
  pp.bytes = 0;
}

// --- workspace pool ------------------------------------------------------------

void reap_leases(nmc_ctx* ctx, bool wait_oldest) {
  while (!ctx->leases.empty()) {
    Lease& l = ctx->leases.front();
    hipError_t q = wait_oldest ? hipEventSynchronize(l.ev) : hipEventQuery(l.ev);
    if (q == hipErrorNotReady) break;
    for (auto& b : l.blocks) ctx->free_blocks.push_back(b);
    (void)hipEventDestroy(l.ev);
    ctx->leases.pop_front();
    wait_oldest = false;
  }
}

int pool_alloc(nmc_ctx* ctx, size_t bytes, Block* out) {
  bytes = align_up(bytes, 2u << 20);
  reap_leases(ctx, false);
  for (int attempt = 0; attempt < 2; ++attempt) {
    // best fit among cached blocks within 2x
    int best = -1;
    for (size_t i = 0; i < ctx->free_blocks.size(); ++i) {
      const Block& b = ctx->free_blocks[i];
      if (b.bytes >= bytes && b.bytes < 2 * bytes && (best < 0 || b.bytes < ctx->free_blocks[best].bytes))
        best = (int)i;
    }
    if (best >= 0) {
      *out = ctx->free_blocks[best];
      ctx->free_blocks.erase(ctx->free_blocks.begin() + best);
      return NMC_OK;
    }
    // release cached blocks while over budget (or before a fresh allocation fails)
    while (ctx->budget && ctx->allocated + ctx->green_bytes + bytes > ctx->budget && !ctx->free_blocks.empty()) {
      auto it = std::max_element(ctx->free_blocks.begin(), ctx->free_blocks.end(),
                                 [](const Block& a, const Block& b) { return a.bytes < b.bytes; });
      (void)hipFree(it->ptr);
      ctx->allocated -= it->bytes;
      ctx->free_blocks.erase(it);
    }
    if (!ctx->budget || ctx->allocated + ctx->green_bytes + bytes <= ctx->budget) {
      void* p = nullptr;
      hipError_t e = hipMalloc(&p, bytes);
      if (e == hipSuccess) {
        ctx->allocated += bytes;
        *out = Block{p, bytes};
        return NMC_OK;
      }
      (void)hipGetLastError();
      // free every cached block and retry once
      for (auto& b : ctx->free_blocks) {
        (void)hipFree(b.ptr);
        ctx->allocated -= b.bytes;
      }
      ctx->free_blocks.clear();
      e = hipMalloc(&p, bytes);
      if (e == hipSuccess) {
        ctx->allocated += bytes;
        *out = Block{p, bytes};
        return NMC_OK;
      }
      (void)hipGetLastError();
    }
    if (ctx->leases.empty()) break;
    reap_leases(ctx, true);  // wait for the oldest outstanding solve, then retry
  }
  return fail(ctx, NMC_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes does not fit (budget " +
                                   std::to_string(ctx->budget) + "; held: " + std::to_string(ctx->allocated) +
                                   " workspace, " + std::to_string(ctx->green_bytes) + " Green tables)");
}

// The lease's blocks return to the pool when the event recorded after the
// solve has completed; without an event, once the stream has drained.
int lease_close(nmc_ctx* ctx, Lease&& lease, hipStream_t s, std::deque<Lease>* into) {
  hipError_t e = hipEventCreateWithFlags(&lease.ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(lease.ev, s);
  if (e != hipSuccess) {
    if (lease.ev) (void)hipEventDestroy(lease.ev);
    (void)hipStreamSynchronize(s);
    for (auto& b : lease.blocks) ctx->free_blocks.push_back(b);
    return hip_fail(ctx, e, "solve completion event");
  }
  into->push_back(std::move(lease));
  return NMC_OK;
}

// --- validation ----------------------------------------------------------------

int validate(nmc_ctx* ctx, const Req& r, int refine) {
  if (!r.rho || !r.phi) return fail(ctx, NMC_EINVAL, "rho and phi must be non-null device pointers");
  if (r.N < kMinN || r.N % 4 != 0) return fail(ctx, NMC_EINVAL, "N must be a multiple of 4, >= 4");
  if (!period_of(r.N)) return fail(ctx, NMC_EUNSUPPORTED, "N above 256 (padded period above 512)");
  if (max_period(r.N, r.L, r.flags) > kMaxScaledP)
    return fail(ctx, NMC_EUNSUPPORTED, is_modified3(r.flags, r.L)
                                           ? "NMC_MODIFIED3: N above 128 (quadrupled-grid period above 1024)"
                                           : "NMC_MODIFIED: N above 256 (doubled-grid period above 1024)");
  if (r.L < 1 || r.L > kMaxL) return fail(ctx, NMC_EINVAL, "L must be in [1, 16]");
  if (!(r.h0 > 0) || !std::isfinite(r.h0)) return fail(ctx, NMC_EINVAL, "h0 must be positive and finite");
  if (!std::isfinite(r.G)) return fail(ctx, NMC_EINVAL, "G must be finite");
  if (refine != 2) return fail(ctx, NMC_EINVAL, "refinement factor must be 2");
  if (r.p != NMC_F64 && r.p != NMC_F32) return fail(ctx, NMC_EINVAL, "unknown precision");
  const size_t bytes = (size_t)r.L * r.N * r.N * r.N * real_size(r.p);
  const char* a = (const char*)r.rho;
  const char* b = (const char*)r.phi;
  if (a < b + bytes && b < a + bytes) return fail(ctx, NMC_EINVAL, "rho and phi overlap");
  return NMC_OK;
}

// --- profiling -------------------------------------------------------------------

struct ProfScope {
  // The kernel of the enclosed launcher call records event a when it starts
  // and b when it ends (nmc::set_next_launch_events), so the recorded time is
  // the kernel's own duration; if the launcher launched nothing, the events
  // are recorded on the stream around the call instead.
  nmc_ctx* ctx;
  hipStream_t s;
  int pass;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(nmc_ctx* c, hipStream_t st, int p, double by) : ctx(c), s(st), pass(p), bytes(by) {
    if (!ctx->profiling) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      a = b = nullptr;
      return;
    }
    nmc::set_next_launch_events(a, b);
  }
  ~ProfScope() {
    if (!a) return;
    if (nmc::take_next_launch_events()) {  // not consumed by a kernel launch
      (void)hipEventRecord(a, s);
      (void)hipEventRecord(b, s);
    }
    ctx->prof.push_back({pass, a, b, bytes});
  }
};

// Algorithmic HBM bytes of one grid in each pass (what the pruned method reads
// and writes with this layout; the zero padding is never touched).  nin is
// the grid's input extent per axis and nout its output rows (FieldDesc).
struct PassBytes {
  double r, c, N, nin, nout, P, H, NS;
  int kind;
  // kinds 3, 5 (scaled grids, P the scaled period): N output rows after the fold
  PassBytes(int N_, int P_, size_t rsz, int kind_)
      : r((double)rsz), c(2.0 * rsz), N(N_), nin(kind_ == 1 ? N_ / 2 + 2 : N_),
        nout(kind_ == 0 || kind_ == 4 || kind_ == 3 || kind_ == 5 ? N_ : N_ / 2 + 2), P(P_),
        H(P_ / 2 + 1), NS(N_ / 2 + 2), kind(kind_) {}
  double half() const { return P / 2; }
  double x() const {
    const double in = kind == 1 ? std::pow(N / 2, 3) : N * N * N;
    return in * r + nin * nin * half() * c;
  }
  double y() const { return nin * nin * half() * c + nin * P * half() * c; }
  // the spectrum octant is shared by every grid of a launch: spectrum() is
  // added once per launch
  double z() const { return (nin + nout) * P * half() * c; }
  double spectrum() const { return H * H * H * r; }
  double iy() const {
    return nout * P * half() * c + nout * nout * half() * c;
  }
  // fused plane passes: the x-transformed plane stays on chip
  double xy() const {
    const double in = kind == 1 ? std::pow(N / 2, 3) : N * N * N;
    return in * r + nin * P * half() * c;
  }
  double iyx(bool carry, bool next) const { return nout * P * half() * c + ix(carry, next) - nout * nout * half() * c; }
  double ix(bool carry, bool next) const {
    // the carried box S is read once per level; C is read and S_l written
    // (kind 4: the hole potential's box written)
    return nout * nout * half() * c + nout * nout * nout * r + (carry ? NS * NS * NS * r : 0.0) +
           (next ? (kind == 4 ? 1 : 2) * NS * NS * NS * r : 0.0);
  }
  // a scaled grid's folded last pass: N^2 half spectra read, the potential
  // so far read and Phi(Omega^l) written on N^3 cells, the carry read
  double ix_doubled(bool carry) const {
    return N * N * half() * c + 2 * N * N * N * r + (carry ? NS * NS * NS * r : 0.0);
  }
};

// --- the solve -------------------------------------------------------------------

template <class R>
int run_group(nmc_ctx* ctx, const Req* reqs, int count, char* ws, hipStream_t s, hipStream_t aux) {
  const int N = reqs[0].N;
  const int P = period_of(N);
  const int NC = N / 2 + 2;
  const bool mod = is_modified(reqs[0].flags);
  const bool boxes = use_boxes(N) && !mod;
  const int PD = 2 * P;  // period of the doubled grids (modified method)
  auto tables = [&](int Pc) {
    PerP& pp = ctx->perp[Pc];
    nmc::Tables<R> t;
    if constexpr (sizeof(R) == 8) {
      t.tw = (const double2*)pp.tw64;
      t.gz = pp.gz64;
      t.gn = pp.gn64;
    } else {
      t.tw = (const float2*)pp.tw32;
      t.gz = pp.gz32;
      t.gn = pp.gn32;
    }
    return t;
  };
  const nmc::Tables<R> tb = tables(P);
  const nmc::Tables<R> tbd = mod ? tables(PD) : tb;
  const int PQ = 4 * P;  // period of the quadrupled grids (three-level scheme)
  const bool any_mod3 = mod && (reqs[0].flags & NMC_MODIFIED3) && PQ <= kMaxScaledP;
  const nmc::Tables<R> tbq = any_mod3 ? tables(PQ) : tb;
  std::vector<FieldDesc> quads;  // quadrupled grids
  const size_t lvl = (size_t)N * N * N;
  std::vector<FieldDesc> fulls, secs;  // full grids; hole grids or child-region boxes
  std::vector<int> full_level;
  struct RestrictStep {
    const R* fine;
    const R* fine_rc;
    R* out;
  };
  std::vector<RestrictStep> restricts;  // cascaded restriction (N not a multiple of 2^L)
  std::vector<nmc::PyramidDesc> pyramids;
  int pyr_maxL = 0;
  std::vector<nmc::CarryDesc> carries;  // hole pipeline: S_n, n = 1 .. L-2
  std::vector<int> carry_levels;
  int maxL = 0;
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    const Req& q = reqs[i];
    const Layout lo = make_layout(N, q.L, q.p, q.flags);
    char* base = ws + off;
    off += lo.total;
    maxL = std::max(maxL, q.L);
    const R* rho = (const R*)q.rho;
    R* phi = (R*)q.phi;
    const bool restrict_on = !(q.flags & NMC_NO_RESTRICT);
    const bool comp = sizeof(R) == 4 && !(q.flags & NMC_F32_UNCOMPENSATED);
    const bool pyramid = nmc::pyramid_exact(N, q.L);
    const long long rslab = (long long)(lo.rc_bytes / sizeof(R));
    if (restrict_on && q.L >= 2) {
      if (pyramid) {
        pyramids.push_back({rho, base + lo.Rc(0), rslab, q.L});
        pyr_maxL = std::max(pyr_maxL, q.L);
      } else {
        for (int l = q.L - 2; l >= 0; --l) {
          const R* fine_rc = (l + 1 <= q.L - 2) ? (const R*)(base + lo.Rc(l + 1)) : nullptr;
          restricts.push_back({rho + (size_t)(l + 1) * lvl, fine_rc, (R*)(base + lo.Rc(l))});
        }
      }
    }
    if (!boxes && q.L >= 3) {
      carries.push_back({base + lo.Box(0), base + lo.Shi(0), (long long)(lo.box_bytes / sizeof(R)), comp ? 1 : 0});
      carry_levels.push_back(q.L - 2);
    }
    const double P3 = (double)P * P * P;
    for (int l = 0; l < q.L; ++l) {
      const double h = std::ldexp(q.h0, -l);
      const bool finer = l < q.L - 1;  // a finer level exists
      const bool hole_full = mod && finer;  // modified method: hole grid with full output
      FieldDesc f{};
      f.rho = rho + (size_t)l * lvl;
      f.rc = (restrict_on && finer && !mod) ? (const void*)(base + lo.Rc(l)) : nullptr;
      f.rslab = rslab;
      f.rdepth = pyramid ? q.L - 1 - l : 1;
      f.A = base + lo.A(l);
      f.B = base + lo.B(l);
      f.out = phi + (size_t)l * lvl;
      const void* carry_in = nullptr;  // S_{l-1}
      const void* carry_lo = nullptr;
      if (l >= 1) {
        // hole grids: S_0 is the hole potential itself; boxes: S_0 lives in Shi(0)
        carry_in = (!boxes && l == 1) ? base + lo.Box(0) : base + lo.Shi(l - 1);
        carry_lo = (comp && (boxes || l >= 2)) ? (const void*)(base + lo.Slo(l - 1)) : nullptr;
      }
      if (!hole_full) {  // the modified method adds the carry in the doubled grid's last pass
        f.S = carry_in;
        f.Slo = carry_lo;
      }
      if (boxes && finer) {
        f.Sout = base + lo.Shi(l);
        f.Slo_out = comp ? (void*)(base + lo.Slo(l)) : nullptr;
        f.C = base + lo.Box(l);
      }
      if (hole_full) f.Sout = base + lo.Box(l);  // the hole potential's box, for the carry
      f.scale = -q.G * h * h / P3;
      f.kind = hole_full ? 4 : 0;
      f.comp = comp ? 1 : 0;
      f.tri = (q.flags & NMC_PROLONG_TRILINEAR) ? 1 : 0;
      fulls.push_back(f);
      full_level.push_back(l);
      // three-level scheme (Appendix B): a level with two finer levels takes
      // level l+1's hole density on the doubled grid and level l+2's density
      // on a quadrupled grid
      const bool triple = lo.mod3 && l < q.L - 2;
      if (triple) {
        const double hq = std::ldexp(q.h0, -(l + 2));
        const double PQ3 = (double)PQ * PQ * PQ;
        FieldDesc c{};
        c.rho = rho + (size_t)(l + 2) * lvl;
        c.rc = (restrict_on && l + 2 < q.L - 1) ? (const void*)(base + lo.Rc(l + 2)) : nullptr;
        c.rslab = rslab;
        c.rdepth = pyramid ? q.L - 3 - l : 1;
        c.A = base + lo.Aq(l);
        c.B = base + lo.Bq(l);
        c.out = phi + (size_t)l * lvl;  // added after the doubled grid's pass
        c.scale = -q.G * hq * hq / PQ3;
        c.kind = 3;
        c.comp = f.comp;
        c.tri = f.tri;
        quads.push_back(c);
      }
      if (finer && mod) {
        // doubled grid of the pair (l, l+1): level l+1's density (its own
        // child region restricted, or zeroed in the three-level scheme) on
        // the grid of level l+1's spacing
        const double hf = std::ldexp(q.h0, -(l + 1));
        const double PD3 = (double)PD * PD * PD;
        FieldDesc c{};
        c.rho = rho + (size_t)(l + 1) * lvl;
        c.rc = (restrict_on && l + 1 < q.L - 1 && !triple) ? (const void*)(base + lo.Rc(l + 1)) : nullptr;
        c.rslab = rslab;
        c.rdepth = pyramid ? q.L - 2 - l : 1;
        c.A = base + lo.As(l);
        c.B = base + lo.Bs(l);
        c.out = phi + (size_t)l * lvl;
        c.S = carry_in;
        c.Slo = carry_lo;
        c.scale = -q.G * hf * hf / PD3;
        c.kind = triple ? 5 : 3;
        c.comp = f.comp;
        c.tri = f.tri;
        secs.push_back(c);
      } else if (finer) {
        FieldDesc c{};
        c.rho = f.rho;
        c.rc = boxes ? f.rc : nullptr;
        c.rslab = f.rslab;
        c.rdepth = f.rdepth;
        c.A = base + lo.As(l);
        c.B = base + lo.Bs(l);
        c.out = base + lo.Box(l);
        c.scale = f.scale;
        c.kind = boxes ? 1 : 2;
        c.comp = f.comp;
        c.tri = f.tri;
        secs.push_back(c);
      }
    }
  }
  auto for_chunks_p = [&](const std::vector<FieldDesc>& fs, int n, auto launch, int pass, hipStream_t st,
                          int Pc, const nmc::Tables<R>& tbc) -> hipError_t {
    for (size_t a = 0; a < fs.size(); a += nmc::kMaxFieldsPerLaunch) {
      FieldTable ft{};
      const int cnt = (int)std::min<size_t>(nmc::kMaxFieldsPerLaunch, fs.size() - a);
      double bytes = 0;
      for (int k = 0; k < cnt; ++k) {
        ft.f[k] = fs[a + k];
        const PassBytes pb(N, Pc, sizeof(R), ft.f[k].kind);
        switch (pass) {
          case NMC_PASS_X: bytes += pb.x(); break;
          case NMC_PASS_Y: bytes += pb.y(); break;
          case NMC_PASS_Z: bytes += pb.z(); break;
          case NMC_PASS_IY: bytes += pb.iy(); break;
          case NMC_PASS_XY: bytes += pb.xy(); break;
          case NMC_PASS_IYX_SECOND:
          case NMC_PASS_IYX_FULL: bytes += pb.iyx(ft.f[k].S != nullptr, ft.f[k].Sout != nullptr); break;
          case NMC_PASS_IX_DOUBLED: bytes += pb.ix_doubled(ft.f[k].S != nullptr); break;
          default: bytes += pb.ix(ft.f[k].S != nullptr, ft.f[k].Sout != nullptr); break;
        }
      }
      if (pass == NMC_PASS_Z) bytes += PassBytes(N, Pc, sizeof(R), 0).spectrum();
      PassGeom g{N, Pc, n, cnt, Pc / P};
      ProfScope ps(ctx, st, pass, bytes);
      hipError_t e = launch(ft, g, tbc, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  auto for_chunks = [&](const std::vector<FieldDesc>& fs, int n, auto launch, int pass,
                        hipStream_t st) -> hipError_t { return for_chunks_p(fs, n, launch, pass, st, P, tb); };
  auto restrict_cascade = [&](hipStream_t st) -> int {
    const double nn = (double)N * N * N;
    for (size_t a = 0; a < pyramids.size(); a += nmc::kMaxPyramidsPerLaunch) {
      nmc::PyramidTable tab{};
      const int cnt = (int)std::min<size_t>(nmc::kMaxPyramidsPerLaunch, pyramids.size() - a);
      double bytes = 0;
      for (int k = 0; k < cnt; ++k) {
        tab.r[k] = pyramids[a + k];
        bytes += (double)(tab.r[k].L - 1) * (nn + (double)nmc::pyramid_slab(N, tab.r[k].L)) * sizeof(R);
      }
      ProfScope ps(ctx, st, NMC_PASS_RESTRICT, bytes);
      NMC_HIP(ctx, nmc::launch_pyramid<R>(tab, cnt, N, pyr_maxL, st));
    }
    for (const auto& r : restricts) {
      ProfScope ps(ctx, st, NMC_PASS_RESTRICT, (nn + nn / 8) * sizeof(R));
      NMC_HIP(ctx, nmc::launch_restrict<R>(r.fine, r.fine_rc, r.out, N, st));
    }
    return NMC_OK;
  };
  const bool tri = (reqs[0].flags & NMC_PROLONG_TRILINEAR) != 0;  // shared by the group (method_of)
  auto carry_cascade = [&](hipStream_t st) -> int {
    const double ns3 = std::pow((double)NC, 3);
    // one launch sequence per kind of sum (compensated or plain)
    std::vector<size_t> order;
    for (int c = 1; c >= 0; --c)
      for (size_t k = 0; k < carries.size(); ++k)
        if (carries[k].comp == c) order.push_back(k);
    for (size_t a = 0; a < order.size();) {
      int cnt = 0;
      while (a + cnt < order.size() && cnt < nmc::kMaxCarriesPerLaunch &&
             carries[order[a + cnt]].comp == carries[order[a]].comp)
        ++cnt;
      if (tri) {
        // tensor-product rule: one launch per level
        nmc::CarryTable tab{};
        int maxlev = 0;
        for (int k = 0; k < cnt; ++k) {
          tab.r[k] = carries[order[a + k]];
          tab.nlev[k] = carry_levels[order[a + k]];
          maxlev = std::max(maxlev, tab.nlev[k]);
        }
        for (int n = 1; n <= maxlev; ++n) {
          double bytes = 0;
          for (int k = 0; k < cnt; ++k)
            if (n <= tab.nlev[k]) bytes += ns3 * sizeof(R) * (tab.r[k].comp ? 5 : 3);  // S_{n-1}, hole read; S_n written
          ProfScope ps(ctx, st, NMC_PASS_CARRY, bytes);
          NMC_HIP(ctx, nmc::launch_carry_tri<R>(tab, cnt, N, n, st));
        }
        a += cnt;
        continue;
      }
      for (int n0 = 1;; n0 += nmc::kMaxCarryDepth) {
        nmc::CarryTable tab{};
        int any = 0;
        double bytes = 0;
        for (int k = 0; k < cnt; ++k) {
          tab.r[k] = carries[order[a + k]];
          const int left = carry_levels[order[a + k]] - (n0 - 1);
          tab.nlev[k] = std::max(0, std::min(nmc::kMaxCarryDepth, left));
          any += tab.nlev[k];
          // per level: the hole potential read, S written (hi, lo)
          bytes += tab.nlev[k] * ns3 * sizeof(R) * (tab.r[k].comp ? 3 : 2);
        }
        if (!any) break;
        ProfScope ps(ctx, st, NMC_PASS_CARRY, bytes);
        NMC_HIP(ctx, nmc::launch_carry<R>(tab, cnt, N, n0, st));
      }
      a += cnt;
    }
    return NMC_OK;
  };
  auto forward_to_iy = [&](const std::vector<FieldDesc>& fs, int nin, int nout, hipStream_t st) -> int {
    if (fs.empty()) return NMC_OK;
    NMC_HIP(ctx, for_chunks(fs, nin, nmc::launch_fwd_x<R>, NMC_PASS_X, st));
    NMC_HIP(ctx, for_chunks(fs, nin, nmc::launch_fwd_y<R>, NMC_PASS_Y, st));
    NMC_HIP(ctx, for_chunks(fs, nin, nmc::launch_z<R>, NMC_PASS_Z, st));
    NMC_HIP(ctx, for_chunks(fs, nout, nmc::launch_inv_y<R>, NMC_PASS_IY, st));
    return NMC_OK;
  };
  int rc;
  const bool one_stream = (reqs[0].flags & NMC_ONE_STREAM) != 0;
  const bool fused = nmc::plane_passes_fit<R>(P) && !(reqs[0].flags & NMC_NO_FUSED_PLANES);
  if (mod) {
    // Modified method: hole grids with full output (kind 4) and the finest
    // full grid on period P, as in the hole pipeline; the scaled grids
    // (doubled on period 2P, quadrupled on 4P) independent of them until
    // their last passes, which add their means to the hole potential in phi
    // (the doubled grids' pass also the carry).
    if ((rc = restrict_cascade(s))) return rc;
    std::vector<FieldDesc> holes, finest;
    for (const auto& f : fulls) (f.kind == 4 ? holes : finest).push_back(f);
    auto scaled_to_iy = [&](const std::vector<FieldDesc>& fs, int Pc, const nmc::Tables<R>& tbc,
                            hipStream_t st) -> int {
      if (fs.empty()) return NMC_OK;
      NMC_HIP(ctx, for_chunks_p(fs, N, nmc::launch_fwd_x<R>, NMC_PASS_X, st, Pc, tbc));
      NMC_HIP(ctx, for_chunks_p(fs, N, nmc::launch_fwd_y<R>, NMC_PASS_Y, st, Pc, tbc));
      NMC_HIP(ctx, for_chunks_p(fs, N, nmc::launch_z<R>, NMC_PASS_Z, st, Pc, tbc));
      NMC_HIP(ctx, for_chunks_p(fs, N, nmc::launch_inv_y_fold<R>, NMC_PASS_IY, st, Pc, tbc));
      return NMC_OK;
    };
    auto scaled_grids_to_iy = [&](hipStream_t st) -> int {
      int r = scaled_to_iy(secs, PD, tbd, st);
      return r ? r : scaled_to_iy(quads, PQ, tbq, st);
    };
    // the scaled grids' passes on the second stream: measured faster from
    // N = 64 and with quadrupled grids; at N = 32 with doubled grids only
    // the join costs more than the overlap gains (FP32 14.2k against 11.3k
    // solves/s at 32^3 x 3)
    const bool fork = aux && aux != s && !secs.empty() && !ctx->profiling && !one_stream &&
                      (N >= 64 || !quads.empty());
    if (fork) {
      NMC_HIP(ctx, hipEventRecord(ctx->ev_fork, s));
      NMC_HIP(ctx, hipStreamWaitEvent(aux, ctx->ev_fork, 0));
      if ((rc = scaled_grids_to_iy(aux))) return rc;
      NMC_HIP(ctx, hipEventRecord(ctx->ev_join, aux));
    }
    if (fused) {
      NMC_HIP(ctx, for_chunks(fulls, N, nmc::launch_fwd_xy<R>, NMC_PASS_XY, s));
      NMC_HIP(ctx, for_chunks(fulls, N, nmc::launch_z<R>, NMC_PASS_Z, s));
      if (!holes.empty()) NMC_HIP(ctx, for_chunks(holes, N, nmc::launch_inv_yx<R>, NMC_PASS_IYX_SECOND, s));
      if ((rc = carry_cascade(s))) return rc;
      NMC_HIP(ctx, for_chunks(finest, N, nmc::launch_inv_yx<R>, NMC_PASS_IYX_FULL, s));
    } else {
      if ((rc = forward_to_iy(fulls, N, N, s))) return rc;
      if (!holes.empty()) NMC_HIP(ctx, for_chunks(holes, N, nmc::launch_inv_x<R>, NMC_PASS_IX_SECOND, s));
      if ((rc = carry_cascade(s))) return rc;
      NMC_HIP(ctx, for_chunks(finest, N, nmc::launch_inv_x<R>, NMC_PASS_IX_FULL, s));
    }
    if (fork) {
      NMC_HIP(ctx, hipStreamWaitEvent(s, ctx->ev_join, 0));
    } else if ((rc = scaled_grids_to_iy(s))) {
      return rc;
    }
    if (!secs.empty())
      NMC_HIP(ctx, for_chunks_p(secs, N, nmc::launch_inv_x_fold<R>, NMC_PASS_IX_DOUBLED, s, PD, tbd));
    if (!quads.empty())
      NMC_HIP(ctx, for_chunks_p(quads, N, nmc::launch_inv_x_fold<R>, NMC_PASS_IX_DOUBLED, s, PQ, tbq));
    return NMC_OK;
  }
  if (!boxes) {
    // hole grids: one stream, full and hole grids share every launch
    if ((rc = restrict_cascade(s))) return rc;
    std::vector<FieldDesc> all(fulls);
    all.insert(all.end(), secs.begin(), secs.end());
    if (fused) {
      NMC_HIP(ctx, for_chunks(all, N, nmc::launch_fwd_xy<R>, NMC_PASS_XY, s));
      NMC_HIP(ctx, for_chunks(all, N, nmc::launch_z<R>, NMC_PASS_Z, s));
      if (!secs.empty()) NMC_HIP(ctx, for_chunks(secs, NC, nmc::launch_inv_yx<R>, NMC_PASS_IYX_SECOND, s));
      if ((rc = carry_cascade(s))) return rc;
      NMC_HIP(ctx, for_chunks(fulls, N, nmc::launch_inv_yx<R>, NMC_PASS_IYX_FULL, s));
      return NMC_OK;
    }
    if ((rc = forward_to_iy(all, N, N, s))) return rc;
    if (!secs.empty()) NMC_HIP(ctx, for_chunks(secs, NC, nmc::launch_inv_x<R>, NMC_PASS_IX_SECOND, s));
    if ((rc = carry_cascade(s))) return rc;
    NMC_HIP(ctx, for_chunks(fulls, N, nmc::launch_inv_x<R>, NMC_PASS_IX_FULL, s));
    return NMC_OK;
  }
  // child-region boxes: they need the restriction, then the boxes and the
  // full grids are independent until the last pass and may use two streams
  if ((rc = restrict_cascade(s))) return rc;
  if (aux && aux != s && !secs.empty() && !ctx->profiling && !one_stream) {
    NMC_HIP(ctx, hipEventRecord(ctx->ev_fork, s));
    NMC_HIP(ctx, hipStreamWaitEvent(aux, ctx->ev_fork, 0));
    if ((rc = forward_to_iy(secs, NC, NC, aux))) return rc;
    NMC_HIP(ctx, for_chunks(secs, NC, nmc::launch_inv_x<R>, NMC_PASS_IX_SECOND, aux));
    if ((rc = forward_to_iy(fulls, N, N, s))) return rc;
    NMC_HIP(ctx, hipEventRecord(ctx->ev_join, aux));
    NMC_HIP(ctx, hipStreamWaitEvent(s, ctx->ev_join, 0));
  } else {
    std::vector<FieldDesc> all(fulls);
    all.insert(all.end(), secs.begin(), secs.end());
    if ((rc = forward_to_iy(all, N, N, s))) return rc;
    if (!secs.empty()) NMC_HIP(ctx, for_chunks(secs, NC, nmc::launch_inv_x<R>, NMC_PASS_IX_SECOND, s));
  }
  // Last pass of the full grids, coarsest level first: level l adds the carry
  // S_{l-1} left by level l-1 and leaves S_l for level l+1.
  for (int l = 0; l < maxL; ++l) {
    std::vector<FieldDesc> fl;
    for (size_t k = 0; k < fulls.size(); ++k)
      if (full_level[k] == l) fl.push_back(fulls[k]);
    NMC_HIP(ctx, for_chunks(fl, N, nmc::launch_inv_x<R>, NMC_PASS_IX_FULL, s));
  }
  return NMC_OK;
}

void drop_graph(nmc_ctx* ctx, std::map<GraphKey, GraphEntry>::iterator it);

// The serving arena's allocation (hipFree waits for the device).
void release_arena(nmc_ctx* ctx) {
  if (!ctx->arena_base) return;
  (void)hipFree(ctx->arena_base);
  ctx->allocated -= ctx->arena.size();
  ctx->arena_base = nullptr;
  ctx->arena = nmc::RingArena{};
}

// Under a budget, until `need` more bytes fit: release cached workspace
// blocks, then the captured graphs (they hold workspace and the tables'
// addresses), then the least recently used Green tables whose period is not
// in `keep` (after the device has finished every use).  What still does not
// fit is reported by the allocation that follows.
void make_room(nmc_ctx* ctx, size_t need, const std::vector<int>& keep) {
  if (!ctx->budget) return;
  auto over = [&] { return ctx->allocated + ctx->green_bytes + need > ctx->budget; };
  bool synced = false;
  reap_leases(ctx, false);
  while (over()) {
    if (!ctx->free_blocks.empty()) {
      auto it = std::max_element(ctx->free_blocks.begin(), ctx->free_blocks.end(),
                                 [](const Block& a, const Block& b) { return a.bytes < b.bytes; });
      (void)hipFree(it->ptr);
      ctx->allocated -= it->bytes;
      ctx->free_blocks.erase(it);
      continue;
    }
    if (ctx->arena_base && ctx->arena.empty() && (!ctx->serve || ctx->serve->idle())) {
      release_arena(ctx);  // the serving arena, while no batch uses it
      continue;
    }
    if (!synced) {
      (void)hipDeviceSynchronize();
      reap_leases(ctx, false);
      while (!ctx->graphs.empty()) drop_graph(ctx, ctx->graphs.begin());
      synced = true;
      continue;  // completed leases and the dropped graphs' workspace are free now
    }
    PerP* lru = nullptr;
    for (auto& kv : ctx->perp)
      if (kv.second.bytes && std::find(keep.begin(), keep.end(), kv.first) == keep.end() &&
          (!lru || kv.second.used < lru->used))
        lru = &kv.second;
    if (!lru) return;
    free_green(ctx, *lru);
  }
}

// Green tables (and twiddles) of every period a group needs, and room for
// its workspace of ws_bytes, under the budget.
std::vector<int> periods_of(int N, unsigned flags) {
  const int P = period_of(N);
  std::vector<int> keep{P};
  if (is_modified(flags)) keep.push_back(2 * P);
  if ((flags & NMC_MODIFIED3) && 4 * P <= kMaxScaledP) keep.push_back(4 * P);
  return keep;
}

// The Green tables (and twiddles) of every period a group needs.
int prepare_tables(nmc_ctx* ctx, int N, unsigned flags, hipStream_t s) {
  const std::vector<int> keep = periods_of(N, flags);
  size_t need = 0;
  for (int q : keep)
    if (!ctx->perp[q].bytes) need += green_table_bytes(q);
  if (need) make_room(ctx, need, keep);
  for (int q : keep) {
    int rc = ensure_green(ctx, q, s);
    if (rc) return rc;
    ctx->perp[q].used = ++ctx->clock;
  }
  return NMC_OK;
}

int prepare(nmc_ctx* ctx, int N, unsigned flags, hipStream_t s, size_t ws_bytes) {
  int rc = prepare_tables(ctx, N, flags, s);
  if (rc) return rc;
  const std::vector<int> keep = periods_of(N, flags);
  // a cached block the pool will reuse for the workspace needs no room
  const size_t ws = align_up(ws_bytes, 2u << 20);
  reap_leases(ctx, false);
  const bool reusable = std::any_of(ctx->free_blocks.begin(), ctx->free_blocks.end(),
                                    [&](const Block& b) { return b.bytes >= ws && b.bytes < 2 * ws; });
  if (!reusable) make_room(ctx, ws, keep);
  return NMC_OK;
}

// Launch requests that share N and precision, on one workspace block.
int launch_group(nmc_ctx* ctx, const Req* reqs, int count, hipStream_t s, Lease* lease, hipStream_t aux) {
  size_t total = 0;
  for (int i = 0; i < count; ++i) total += make_layout(reqs[i].N, reqs[i].L, reqs[i].p, reqs[i].flags).total;
  int rc = prepare(ctx, reqs[0].N, reqs[0].flags, s, total);
  if (rc) return rc;
  Block b{};
  rc = pool_alloc(ctx, total, &b);
  if (rc) return rc;
  lease->blocks.push_back(b);
  if (reqs[0].p == NMC_F64) return run_group<double>(ctx, reqs, count, (char*)b.ptr, s, aux);
  return run_group<float>(ctx, reqs, count, (char*)b.ptr, s, aux);
}

int solve_many(nmc_ctx* ctx, const Req* reqs, int count, hipStream_t s, Lease* lease) {
  // group by (N, precision, method), preserving order inside a group
  std::map<std::tuple<int, int, int>, std::vector<Req>> groups;
  for (int i = 0; i < count; ++i)
    groups[std::make_tuple(reqs[i].N, (int)reqs[i].p, method_of(reqs[i].flags))].push_back(reqs[i]);
  for (auto& kv : groups) {
    auto& v = kv.second;
    for (size_t a = 0; a < v.size(); a += kMaxBatchRequests) {
      const int n = (int)std::min<size_t>(kMaxBatchRequests, v.size() - a);
      int rc = launch_group(ctx, v.data() + a, n, s, lease, ctx->aux_stream);
      if (rc) return rc;
    }
  }
  return NMC_OK;
}

// --- captured (graph) solves ------------------------------------------------------

void drop_graph(nmc_ctx* ctx, std::map<GraphKey, GraphEntry>::iterator it) {
  GraphEntry& e = it->second;
  if (e.last) {
    (void)hipEventSynchronize(e.last);
    (void)hipEventDestroy(e.last);
  }
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.ws.ptr) ctx->free_blocks.push_back(e.ws);
  ctx->graphs.erase(it);
}

int build_graph(nmc_ctx* ctx, const Req& r, const GraphKey& key, hipStream_t s) {
  int rc = prepare(ctx, r.N, r.flags, s, make_layout(r.N, r.L, r.p, r.flags).total);
  if (rc) return rc;
  if (!ctx->cap_stream) NMC_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  while (ctx->graphs.size() >= kMaxGraphs) {
    auto lru = ctx->graphs.begin();
    for (auto it = ctx->graphs.begin(); it != ctx->graphs.end(); ++it)
      if (it->second.used < lru->second.used) lru = it;
    drop_graph(ctx, lru);
  }
  GraphEntry e;
  rc = pool_alloc(ctx, make_layout(r.N, r.L, r.p, r.flags).total, &e.ws);
  if (rc) return rc;
  NMC_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
  rc = r.p == NMC_F64 ? run_group<double>(ctx, &r, 1, (char*)e.ws.ptr, ctx->cap_stream, ctx->aux_stream)
                      : run_group<float>(ctx, &r, 1, (char*)e.ws.ptr, ctx->cap_stream, ctx->aux_stream);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &g);
  if (rc == NMC_OK && ee != hipSuccess) rc = hip_fail(ctx, ee, "hipStreamEndCapture");
  if (rc == NMC_OK) {
    ee = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
    if (ee != hipSuccess) rc = hip_fail(ctx, ee, "hipGraphInstantiate");
  }
  if (g) (void)hipGraphDestroy(g);
  if (rc == NMC_OK) {
    ee = hipEventCreateWithFlags(&e.last, hipEventDisableTiming);
    if (ee != hipSuccess) rc = hip_fail(ctx, ee, "hipEventCreate");
  }
  if (rc) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    ctx->free_blocks.push_back(e.ws);
    return rc;
  }
  ctx->graphs[key] = e;
  return NMC_OK;
}

int launch_graph(nmc_ctx* ctx, GraphEntry& e, hipStream_t s) {
  NMC_HIP(ctx, hipStreamWaitEvent(s, e.last, 0));  // a replay on another stream may still run
  NMC_HIP(ctx, hipGraphLaunch(e.exec, s));
  NMC_HIP(ctx, hipEventRecord(e.last, s));
  e.used = ++ctx->clock;
  return NMC_OK;
}

int set_device(nmc_ctx* ctx) {
  NMC_HIP(ctx, hipSetDevice(ctx->device));
  return NMC_OK;
}

// --- static scratch (nmc_solve_noalloc) -------------------------------------------

}  // namespace

// Workspace of nmc_solve_noalloc: a fixed array in the library's device code,
// one copy per GPU the library runs on, held until the process ends.  Host
// code never passes `scratch` itself to a kernel (on the host it names a
// stand-in, not device memory): it uses the address hipGetSymbolAddress gives
// for the current device.
__device__ __align__(256) char scratch[NMC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of this device's `scratch`, looked up once per device (the
// device must be current).
int scratch_address(nmc_ctx* ctx, int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ctx, NMC_EINVAL, "device index above the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return NMC_OK;
}

// --- serving ------------------------------------------------------------------

// The serving scheduler's device side: each batch is one batched solve on
// the next serving stream, ordered after the events recorded at submission,
// and completes with an event recorded after it.
// The serving arena of a context with a budget: created at the first
// serving launch from what the budget leaves beside the Green tables, the
// workspace of solves in flight and room for the tables of other periods
// (a sixteenth of the budget, at most 1 GiB); cached solve workspace blocks
// are released first.  make_room frees it again while no batch uses it.
int ensure_arena(nmc_ctx* ctx) {
  if (ctx->arena_base) return NMC_OK;
  reap_leases(ctx, false);
  for (auto& b : ctx->free_blocks) {
    (void)hipFree(b.ptr);
    ctx->allocated -= b.bytes;
  }
  ctx->free_blocks.clear();
  const size_t headroom = std::min<size_t>(ctx->budget / 16, size_t(1) << 30);
  const size_t held = ctx->allocated + ctx->green_bytes + headroom;
  if (held >= ctx->budget) return fail(ctx, NMC_ENOMEM, "serving: the budget leaves no room for serving workspace");
  const size_t size = (ctx->budget - held) / (2u << 20) * (2u << 20);
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, size);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, NMC_ENOMEM, "serving: workspace arena of " + std::to_string(size) + " bytes: " +
                                     hipGetErrorString(e));
  }
  ctx->arena_base = static_cast<char*>(p);
  ctx->arena = nmc::RingArena(size);
  ctx->allocated += size;
  return NMC_OK;
}

class HipServeDevice final : public nmc::ServeDevice {
 public:
  explicit HipServeDevice(nmc_ctx* c) : ctx_(c) {}
  int poll(const nmc::ServeBatch& b) override {
    const hipError_t q = hipEventQuery(static_cast<const Lease*>(b.dev)->ev);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) return hip_fail(ctx_, q, "serving batch");
    return 1;
  }
  int launch(nmc::ServeBatch& b) override {
    auto lease = std::make_unique<Lease>();
    std::vector<Req> rs;
    for (uint64_t t : b.tickets) rs.push_back(ctx_->sreq.at(t).r);
    hipStream_t s = ctx_->streams[ctx_->next_stream];
    int rc = NMC_OK;
    // under a budget the batch's workspace is a region of the serving arena;
    // NMC_ENOMEM (nothing enqueued) when it does not fit beside the batches
    // in flight, and the scheduler retries after some retire
    size_t arena_bytes = 0, arena_off = 0;
    if (ctx_->budget) {
      for (const Req& r : rs) arena_bytes += make_layout(r.N, r.L, r.p, r.flags).total;
      arena_bytes = align_up(arena_bytes, size_t(64) << 10);
      if ((rc = prepare_tables(ctx_, rs[0].N, rs[0].flags, s))) return rc;
      if ((rc = ensure_arena(ctx_))) return rc == NMC_ENOMEM ? NMC_EDEVICE : rc;
      if (ctx_->arena.alloc(arena_bytes, &arena_off)) {
        lease->in_arena = true;
      } else if (!ctx_->arena.empty() || arena_bytes <= ctx_->arena.size()) {
        return NMC_ENOMEM;  // fits once batches in flight retire
      } else {
        // larger than the whole ring, nothing in flight: release it and take
        // workspace of its own (the pool can also evict other periods' tables)
        release_arena(ctx_);
        arena_bytes = 0;
      }
    }
    // order the batch after the callers' work on its inputs and outputs
    for (uint64_t t : b.tickets) {
      hipError_t e = hipStreamWaitEvent(s, ctx_->sreq.at(t).ready, 0);
      if (e != hipSuccess) {
        rc = hip_fail(ctx_, e, "serving: wait for the submitting stream");
        break;
      }
    }
    if (rc == NMC_OK) {
      if (lease->in_arena) {
        char* ws = ctx_->arena_base + arena_off;
        rc = rs[0].p == NMC_F64 ? run_group<double>(ctx_, rs.data(), (int)rs.size(), ws, s, nullptr)
                                : run_group<float>(ctx_, rs.data(), (int)rs.size(), ws, s, nullptr);
      } else {
        rc = launch_group(ctx_, rs.data(), (int)rs.size(), s, lease.get(), nullptr);
      }
    }
    if (rc == NMC_OK) {
      hipError_t e = hipEventCreateWithFlags(&lease->ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(lease->ev, s);
      if (e != hipSuccess) {
        if (lease->ev) (void)hipEventDestroy(lease->ev);
        lease->ev = nullptr;
        rc = hip_fail(ctx_, e, "serving batch event");
      }
    }
    if (rc) {
      // a failed launch may have enqueued part of the group: its workspace is
      // free once the stream has drained.  ENOMEM: the pool could not place
      // it next to the work in flight (block sizes differ from footprints);
      // nothing was enqueued, and a later tick retries
      if (rc != NMC_ENOMEM) (void)hipStreamSynchronize(s);
      for (auto& blk : lease->blocks) ctx_->free_blocks.push_back(blk);
      if (lease->in_arena) ctx_->arena.release_newest();
      return rc;
    }
    ctx_->next_stream = (ctx_->next_stream + 1) % kServeStreams;
    b.bytes = arena_bytes;
    for (auto& blk : lease->blocks) b.bytes += blk.bytes;  // what the device really holds
    b.dev = lease.release();
    return NMC_OK;
  }
  void release(nmc::ServeBatch& b) override {
    Lease* l = static_cast<Lease*>(b.dev);
    for (uint64_t t : b.tickets) {  // the batch waited for these events: complete
      ServeReq& q = ctx_->sreq.at(t);
      if (q.ready) ctx_->ev_pool.push_back(q.ready);
      q.ready = nullptr;
    }
    for (auto& blk : l->blocks) ctx_->free_blocks.push_back(blk);
    if (l->in_arena) ctx_->arena.release_oldest();  // batches retire in launch order
    (void)hipEventDestroy(l->ev);
    delete l;
    b.dev = nullptr;
  }

 private:
  nmc_ctx* ctx_;
};

int serve_tick(nmc_ctx* ctx, int* launched) {
  HipServeDevice dev(ctx);
  const int rc = ctx->serve->tick(dev, launched);
  if (rc == NMC_ENOMEM) return fail(ctx, NMC_ENOMEM, "serving: a batch does not fit the budget with nothing in flight");
  return rc;
}

}  // namespace

// ================================ C ABI ======================================

extern "C" {

int nmc_period(int N) { return period_of(N); }

int nmc_footprint_bytes_flags(int N, int L, nmc_precision p, unsigned flags, size_t* bytes) {
  if (!bytes || N < kMinN || N % 4 != 0 || L < 1 || L > kMaxL || (p != NMC_F64 && p != NMC_F32))
    return NMC_EINVAL;
  if (!period_of(N)) return NMC_EUNSUPPORTED;
  if (max_period(N, L, flags) > kMaxScaledP) return NMC_EUNSUPPORTED;
  *bytes = make_layout(N, L, p, flags).total;
  return NMC_OK;
}

int nmc_footprint_bytes(int N, int L, nmc_precision p, size_t* bytes) {
  return nmc_footprint_bytes_flags(N, L, p, 0u, bytes);
}

int nmc_create(nmc_ctx** out, int hip_device, size_t hbm_budget_bytes) {
  if (!out) return NMC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return NMC_EINVAL;
  auto* ctx = new nmc_ctx();
  ctx->device = hip_device;
  ctx->budget = hbm_budget_bytes;
  ctx->serve = std::make_unique<nmc::ServeCore>(hbm_budget_bytes, kMaxBatchRequests);
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete ctx;
    return NMC_EDEVICE;
  }
  for (auto& s : ctx->streams) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return NMC_EDEVICE;
    }
  }
  if (hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
    delete ctx;
    return NMC_EDEVICE;
  }
  // set-up of nmc_solve_noalloc: this device's scratch address (device current)
  if (scratch_address(ctx, hip_device, &ctx->scratch) != NMC_OK) {
    nmc_destroy(ctx);
    return NMC_EDEVICE;
  }
  *out = ctx;
  return NMC_OK;
}

void nmc_destroy(nmc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  reap_leases(ctx, false);
  while (!ctx->graphs.empty()) drop_graph(ctx, ctx->graphs.begin());
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->serve) {
    for (const auto& b : ctx->serve->inflight()) {
      Lease* l = static_cast<Lease*>(b.dev);
      if (!l) continue;
      for (auto& blk : l->blocks) (void)hipFree(blk.ptr);
      if (l->ev) (void)hipEventDestroy(l->ev);
      delete l;
    }
  }
  for (auto& l : ctx->leases)
    for (auto& blk : l.blocks) (void)hipFree(blk.ptr);
  for (auto& b : ctx->free_blocks) (void)hipFree(b.ptr);
  if (ctx->arena_base) (void)hipFree(ctx->arena_base);
  for (auto& kv : ctx->perp) {
    (void)hipFree(kv.second.tw64);
    (void)hipFree(kv.second.tw32);
    (void)hipFree(kv.second.g64);
    (void)hipFree(kv.second.g32);
    (void)hipFree(kv.second.gz64);
    (void)hipFree(kv.second.gn64);
    (void)hipFree(kv.second.gz32);
    (void)hipFree(kv.second.gn32);
  }
  for (auto& kv : ctx->sreq)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& s : ctx->streams) (void)hipStreamDestroy(s);
  if (ctx->aux_stream) (void)hipStreamDestroy(ctx->aux_stream);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  delete ctx;
}

const char* nmc_last_error(const nmc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int nmc_solve(nmc_ctx* ctx, const void* rho, void* phi, int N, int L, double h0, int refine, double G,
              nmc_precision p, unsigned flags, void* hip_stream) {
  if (!ctx) return NMC_EINVAL;
  Req r{rho, phi, N, L, h0, G, p, flags};
  int rc = validate(ctx, r, refine);
  if (rc) return rc;
  if ((rc = set_device(ctx))) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  if (!ctx->profiling && !(flags & NMC_NO_GRAPH)) {
    GraphKey key{};
    std::memset(&key, 0, sizeof(key));
    key.rho = rho;
    key.phi = phi;
    key.N = N;
    key.L = L;
    key.h0 = h0;
    key.G = G;
    key.p = (int)p;
    key.flags = flags;
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
      if (ctx->seen.size() > 4096) ctx->seen.clear();
      if (++ctx->seen[key] >= 2) {
        rc = build_graph(ctx, r, key, s);
        if (rc) return rc;
        it = ctx->graphs.find(key);
      }
    }
    if (it != ctx->graphs.end()) return launch_graph(ctx, it->second, s);
  }
  Lease lease;
  rc = solve_many(ctx, &r, 1, s, &lease);
  if (rc) {
    (void)hipStreamSynchronize(s);  // nothing enqueued before the failure may still use the workspace
    for (auto& b : lease.blocks) ctx->free_blocks.push_back(b);
    return rc;
  }
  return lease_close(ctx, std::move(lease), s, &ctx->leases);
}

int nmc_solve_noalloc(nmc_ctx* ctx, const void* rho, void* phi, int N, int L, double h0, int refine,
                      double G, nmc_precision p, unsigned flags, void* hip_stream) {
  if (!ctx) return NMC_EINVAL;
  Req r{rho, phi, N, L, h0, G, p, flags};
  int rc = validate(ctx, r, refine);
  if (rc) return rc;
  const size_t need = make_layout(N, L, p, flags).total;
  if (need > NMC_SCRATCH_BYTES)
    return fail(ctx, NMC_ENOMEM, "nmc_solve_noalloc: workspace of " + std::to_string(need) +
                                     " bytes exceeds the static scratch of " + std::to_string(NMC_SCRATCH_BYTES) +
                                     " bytes");
  // every table the solve reads must already be resident: building one allocates
  const int P = period_of(N);
  int periods[3] = {P, 0, 0};
  if (is_modified(flags)) periods[1] = 2 * P;
  if (is_modified3(flags, L)) periods[2] = 4 * P;
  for (int q : periods) {
    if (!q) continue;
    auto it = ctx->perp.find(q);
    if (it == ctx->perp.end() || !it->second.g64 || !it->second.tw64)
      return fail(ctx, NMC_ENOMEM, "nmc_solve_noalloc: the Green tables of period " + std::to_string(q) +
                                       " are not resident (build them first with nmc_solve or "
                                       "nmc_green_spectrum of this N and method)");
  }
  if ((rc = set_device(ctx))) return rc;
  if (!ctx->scratch) return fail(ctx, NMC_EDEVICE, "nmc_solve_noalloc: no scratch address for this device");
  for (int q : periods)
    if (q) ctx->perp.find(q)->second.used = ++ctx->clock;
  hipStream_t s = (hipStream_t)hip_stream;
  // every grid on the caller's stream; the kernels write every workspace
  // value before reading it, so nothing needs clearing between calls
  return p == NMC_F64 ? run_group<double>(ctx, &r, 1, ctx->scratch, s, s)
                      : run_group<float>(ctx, &r, 1, ctx->scratch, s, s);
}

int nmc_acceleration(nmc_ctx* ctx, const void* phi, void* g, int N, int L, double h0, nmc_precision p,
                     void* hip_stream) {
  if (!ctx) return NMC_EINVAL;
  // same checks as a solve, with g (three components per cell) as output
  Req r{phi, g, N, L, h0, 1.0, p, 0};
  int rc = validate(ctx, r, 2);
  if (rc) return rc;
  const size_t in = (size_t)L * N * N * N * real_size(p);
  const char* a = (const char*)phi;
  const char* b = (const char*)g;
  if (a < b + 3 * in && b < a + in) return fail(ctx, NMC_EINVAL, "phi and g overlap");
  if ((rc = set_device(ctx))) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  {
    // algorithmic bytes: the level's potential read once, three components written
    ProfScope ps(ctx, s, NMC_PASS_ACCEL, 4.0 * in);
    if (p == NMC_F64)
      NMC_HIP(ctx, nmc::launch_accel<double>((const double*)phi, (double*)g, N, L, h0, s));
    else
      NMC_HIP(ctx, nmc::launch_accel<float>((const float*)phi, (float*)g, N, L, h0, s));
  }
  return NMC_OK;
}

int nmc_solve_batch(nmc_ctx* ctx, const nmc_request* reqs, int count, void* hip_stream) {
  if (!ctx) return NMC_EINVAL;
  if (count < 0 || (count > 0 && !reqs)) return fail(ctx, NMC_EINVAL, "bad request array");
  std::vector<Req> rs;
  for (int i = 0; i < count; ++i) {
    Req r{reqs[i].rho, reqs[i].phi, reqs[i].N, reqs[i].L, reqs[i].h0, reqs[i].G, reqs[i].p, reqs[i].flags};
    int rc = validate(ctx, r, 2);
    if (rc) return fail(ctx, rc, "request " + std::to_string(i) + ": " + ctx->err);
    rs.push_back(r);
  }
  if (count == 0) return NMC_OK;
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  Lease lease;
  rc = solve_many(ctx, rs.data(), count, s, &lease);
  if (rc) {
    (void)hipStreamSynchronize(s);
    for (auto& b : lease.blocks) ctx->free_blocks.push_back(b);
    return rc;
  }
  return lease_close(ctx, std::move(lease), s, &ctx->leases);
}

int nmc_serve_submit(nmc_ctx* ctx, const nmc_request* req, void* hip_stream, uint64_t* ticket) {
  if (!ctx) return NMC_EINVAL;
  if (!req || !ticket) return fail(ctx, NMC_EINVAL, "null request or ticket");
  Req r{req->rho, req->phi, req->N, req->L, req->h0, req->G, req->p, req->flags};
  int rc = validate(ctx, r, 2);
  if (rc) return rc;
  const size_t bytes = align_up(make_layout(r.N, r.L, r.p, r.flags).total, 2u << 20);
  if (ctx->budget && bytes > ctx->budget)
    return fail(ctx, NMC_ENOMEM, "request footprint " + std::to_string(bytes) + " exceeds the budget");
  if ((rc = set_device(ctx))) return rc;
  hipEvent_t ev = nullptr;
  if (!ctx->ev_pool.empty()) {
    ev = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
  } else {
    NMC_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  hipError_t e = hipEventRecord(ev, (hipStream_t)hip_stream);
  if (e != hipSuccess) {
    ctx->ev_pool.push_back(ev);
    return hip_fail(ctx, e, "serving: record on the submitting stream");
  }
  const uint64_t t = ctx->serve->submit(nmc::ServeKey{r.N, (int)r.p, method_of(r.flags)}, bytes);
  ctx->sreq[t] = ServeReq{r, ev};
  *ticket = t;
  return NMC_OK;
}

int nmc_serve_tick(nmc_ctx* ctx, int* launched) {
  if (!ctx) return NMC_EINVAL;
  int rc = set_device(ctx);
  if (rc) return rc;
  return serve_tick(ctx, launched);
}

int nmc_serve_poll(nmc_ctx* ctx, uint64_t ticket, int* done) {
  if (!ctx || !done) return NMC_EINVAL;
  const nmc::ServeCore::Item* it = ctx->serve->find(ticket);
  if (!it) return fail(ctx, NMC_EINVAL, "unknown ticket");
  if (it->state != nmc::ServeCore::kDone) {
    int rc = nmc_serve_tick(ctx, nullptr);
    if (rc) return rc;
  }
  *done = ctx->serve->find(ticket)->state == nmc::ServeCore::kDone ? 1 : 0;
  return NMC_OK;
}

int nmc_serve_take_completed(nmc_ctx* ctx, uint64_t* out, int cap, int* n) {
  if (!ctx || !n || cap < 0 || (cap > 0 && !out)) return NMC_EINVAL;
  int rc = nmc_serve_tick(ctx, nullptr);
  if (rc) return rc;
  const int k = ctx->serve->take_completed(out, cap);
  for (int i = 0; i < k; ++i) ctx->sreq.erase(out[i]);
  *n = k;
  return NMC_OK;
}

int nmc_serve_stats_get(nmc_ctx* ctx, nmc_serve_stats* out) {
  if (!ctx || !out) return NMC_EINVAL;
  *out = ctx->serve->stats();
  out->budget_bytes = ctx->budget;
  out->green_cache_bytes = ctx->green_bytes;
  out->arena_bytes = ctx->arena_base ? ctx->arena.size() : 0;
  return NMC_OK;
}

int nmc_serve_drain(nmc_ctx* ctx) {
  if (!ctx) return NMC_EINVAL;
  int rc = set_device(ctx);
  if (rc) return rc;
  while (!ctx->serve->idle()) {
    if ((rc = serve_tick(ctx, nullptr))) return rc;
    if (const nmc::ServeBatch* b = ctx->serve->oldest_inflight())
      NMC_HIP(ctx, hipEventSynchronize(static_cast<const Lease*>(b->dev)->ev));
  }
  return serve_tick(ctx, nullptr);
}

int nmc_green_spectrum(nmc_ctx* ctx, int N, nmc_precision p, void* out, void* hip_stream) {
  if (!ctx) return NMC_EINVAL;
  if (!out) return fail(ctx, NMC_EINVAL, "null output");
  const int P = period_of(N);
  if (!P) return fail(ctx, N < kMinN || N % 4 ? NMC_EINVAL : NMC_EUNSUPPORTED, "bad N");
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  // the tables count against the budget like those of a solve
  if (!ctx->perp[P].bytes) make_room(ctx, green_table_bytes(P), {P});
  if ((rc = ensure_green(ctx, P, s))) return rc;
  const size_t H = P / 2 + 1, n = H * H * H;
  PerP& pp = ctx->perp[P];
  pp.used = ++ctx->clock;
  if (p == NMC_F64)
    NMC_HIP(ctx, hipMemcpyAsync(out, pp.g64, n * 8, hipMemcpyDeviceToDevice, s));
  else
    NMC_HIP(ctx, hipMemcpyAsync(out, pp.g32, n * 4, hipMemcpyDeviceToDevice, s));
  return NMC_OK;
}

int nmc_fft_lines(nmc_ctx* ctx, const void* in, void* out, int P, int nlines, int dir, nmc_precision p,
                  void* hip_stream) {
  if (!ctx) return NMC_EINVAL;
  if (!in || !out || nlines < 0 || (dir != -1 && dir != 1) || P < 8 || P > kMaxP || (P & (P - 1)))
    return fail(ctx, NMC_EINVAL, "bad fft_lines arguments");
  if (nlines == 0) return NMC_OK;
  int rc = set_device(ctx);
  if (rc) return rc;
  PerP& pp = ctx->perp[P];
  if ((rc = ensure_twiddles(ctx, P, pp))) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  if (p == NMC_F64)
    NMC_HIP(ctx, nmc::launch_fft_lines<double>(in, out, P, nlines, dir, pp.tw64, s));
  else
    NMC_HIP(ctx, nmc::launch_fft_lines<float>(in, out, P, nlines, dir, pp.tw32, s));
  return NMC_OK;
}

int nmc_profile_enable(nmc_ctx* ctx, int on) {
  if (!ctx) return NMC_EINVAL;
  for (auto& r : ctx->prof) {
    (void)hipEventSynchronize(r.b);
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  ctx->prof.clear();
  ctx->profiling = on != 0;
  return NMC_OK;
}

int nmc_profile_read(nmc_ctx* ctx, nmc_pass_stat* out) {
  if (!ctx || !out) return NMC_EINVAL;
  for (int i = 0; i < NMC_NUM_PASSES; ++i) out[i] = nmc_pass_stat{0, 0.0, 0.0};
  int rc = NMC_OK;
  for (auto& r : ctx->prof) {
    float ms = 0;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && rc == NMC_OK) rc = hip_fail(ctx, e, "profile events");
    if (r.pass >= 0 && r.pass < NMC_NUM_PASSES) {
      out[r.pass].launches++;
      out[r.pass].total_ms += ms;
      out[r.pass].bytes += r.bytes;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  ctx->prof.clear();
  return rc;
}

const char* nmc_pass_name(int pass) {
  static const char* names[NMC_NUM_PASSES] = {"restrict", "x",     "y",  "z", "inv_y", "inv_x_second", "carry",
                                              "inv_x_full", "xy", "inv_yx_second", "inv_yx_full", "acceleration",
                                              "inv_x_doubled"};
  return (pass >= 0 && pass < NMC_NUM_PASSES) ? names[pass] : "?";
}

}  // extern "C"
