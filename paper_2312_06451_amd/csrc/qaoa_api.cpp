// Host runtime behind the C ABI of include/qaoa.h: handles, buffer management, the pass
// planner of the transverse-field path, scale bookkeeping and result assembly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <array>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>
#include <mutex>
#include <functional>
#include <atomic>

#include "../../include/qaoa.h"
#include "qaoa_internal.h"
#include "qaoa_clique.h"

using namespace qaoa;
using cd = std::complex<double>;

// ---------------------------------------------------------------- errors

static thread_local std::string g_last_error;

namespace {
struct Err {
  int code;
  std::string msg;
};
Err fail(int code, const std::string &m) { return Err{code, m}; }
#define HIPCHK(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw Err{QAOA_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)};             \
  } while (0)
#define REQUIRE(cond, msg)                                                                    \
  do {                                                                                        \
    if (!(cond)) throw Err{QAOA_ERR_INVALID_ARG, msg};                                        \
  } while (0)

}  // namespace

// Lets the angle-finding loop (its own translation unit) report through qaoa_last_error.
namespace qaoa {
void set_last_error(const char *msg) { g_last_error = msg ? msg : ""; }
}  // namespace qaoa

namespace {
template <typename F>
int guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return QAOA_OK;
  } catch (const Err &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const qaoa::CliqueError &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return QAOA_ERR_OUT_OF_MEMORY;
  } catch (...) {
    g_last_error = "unexpected exception";
    return QAOA_ERR_HIP;
  }
}

// Device buffer that grows on demand (never shrinks while its owner lives).
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  void *get(size_t bytes) {
    if (bytes <= cap && p) return p;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (bytes == 0) return nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Err{QAOA_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    cap = bytes;
    return p;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct HostBuf {
  void *p = nullptr;
  size_t cap = 0;
  void *get(size_t bytes) {
    if (bytes <= cap && p) return p;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipHostMalloc(&p, bytes < 4096 ? 4096 : bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Err{QAOA_ERR_OUT_OF_MEMORY, "hipHostMalloc failed"};
    }
    cap = bytes < 4096 ? 4096 : bytes;
    return p;
  }
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
};

// Host memory the device writes directly (fine-grained, coherent, mapped): small result
// arrays that the host reads after synchronising the stream, with no device-to-host copy.
struct MappedBuf {
  void *h = nullptr, *d = nullptr;
  size_t cap = 0;
  void get(size_t bytes) {
    if (bytes <= cap && h) return;
    if (h) (void)hipHostFree(h);
    h = d = nullptr;
    cap = 0;
    const size_t want = bytes < 4096 ? 4096 : bytes;
    if (hipHostMalloc(&h, want, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      h = nullptr;
      (void)hipGetLastError();
      throw Err{QAOA_ERR_OUT_OF_MEMORY, "hipHostMalloc (mapped) failed"};
    }
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
      (void)hipHostFree(h);
      h = d = nullptr;
      (void)hipGetLastError();
      throw Err{QAOA_ERR_HIP, "hipHostGetDevicePointer failed"};
    }
    cap = want;
  }
  ~MappedBuf() {
    if (h) (void)hipHostFree(h);
  }
};

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    HIPCHK(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int64_t binom64(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return r;
}

}  // namespace

// ---------------------------------------------------------------- handles

struct KTotals {
  int64_t launches = 0;
  double ms = 0, bytes = 0, flops = 0;
};

// Choices of the tile-pass plan that leave the results exact up to rounding: the run-time
// tuner (plan_for) searches them, the defaults are the fixed rule.
struct PlanOpts {
  uint8_t narrow = 1;      // strided tiles take runs down to 64 B when that saves a tile
  uint8_t narrow_top = 1;  // with uneven widths (narrow covers; the odd bit of two evenly
                           // split strided tiles), the top tile takes the narrowest runs
  uint8_t lowbits = 1;     // the register-group rules of make_tiles
  uint8_t swap = 0;        // three tiles: the top tile in the middle of a round (single-block
                           // passes) instead of at its end (the round-boundary passes)
  uint8_t down = 0;        // the first round visits the tiles from the top one down
  uint8_t xcd = 1;         // XCD-aware workgroup order (consecutive tiles on one XCD)
  int8_t ckpt = -1;        // reverse sweep: -1 the context's memory rule, 0 in place, 1 checkpoints
  uint8_t swz = 1;         // narrow covers: the swizzled state layout, cached accesses for the
                           // tiles with runs under 128 bytes
};

// Element shift of the swizzled layout's target bits (bits [S, S + 10) of the element index,
// byte address bits [9, 19)), measured best over shifts 3..12 for the top tile of the n = 32
// narrow cover.
inline int swz_shift(int prec) { return prec == QAOA_FP32 ? 6 : 5; }

struct qaoa_ctx {
  int device = 0;
  int64_t live = 0;          // problems and mixers created on this context and not yet destroyed
  int checkpoint_mode = -1;  // -1: when memory allows, 0: never, 1: always
  int xprod_tiles = 1;       // X-product mixers on Hadamard tile passes when they apply
  // tile-pass plans: QAOA_AUTOTUNE / qaoa_ctx_set_autotune; chosen plans per (n, precision,
  // gradient, mixer, checkpoints fit), measured or loaded from a file
  int autotune = 0;
  std::map<std::array<int, 5>, PlanOpts> plans;
  DevBuf phi, lam, ckpt, partials, params, luts, luts2, results, cnt, items, gitems, gamps;
  HostBuf hparams, hresults;
  MappedBuf small_out;  // results of the whole-state kernels
  MappedBuf small_params;  // items and angles of the whole-state kernels, read by them in place
  unsigned char *scratch = nullptr;  // this device's copy of the allocation-free entry point's array
  // batched calls: pinned staging per tile-path instance, and the HIP graphs of their device
  // work (one per problem set, mixers, p, angle-set count, precision and gradient flag)
  int batch_graphs = 1;  // QAOA_BATCH_GRAPH = "0": enqueue every call's work eagerly
  std::vector<std::unique_ptr<HostBuf>> bstage, brstage;
  struct BGraph {
    std::vector<uint64_t> key;
    std::vector<int> ckpt;                // per instance: reverse-sweep mode the work was planned with
    std::vector<uint64_t> fps;            // per unit of work: fingerprint of the captured work
    std::vector<hipGraphExec_t> execs;    // per unit of work: its graph
    int calls = 0;                        // eager calls with this key so far
  };
  std::vector<BGraph> bgraphs;
  hipStream_t gstream = nullptr;  // capture stream when the caller passes the null stream
  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<Pending> pending;
  KTotals totals[QAOA_KC_COUNT];
  ~qaoa_ctx() {
    for (auto &g : bgraphs)
      for (auto ex : g.execs)
        if (ex) (void)hipGraphExecDestroy(ex);
    if (gstream) (void)hipStreamDestroy(gstream);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (auto &p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
  }
  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
};

// Brackets one launch with events when the context profiles (no-op otherwise).
struct KTimer {
  qaoa_ctx *ctx;
  hipStream_t st;
  int cls;
  double bytes, flops;
  hipEvent_t a = nullptr;
  KTimer(qaoa_ctx *c, hipStream_t s, int k, double by, double fl) : ctx(c), st(s), cls(k), bytes(by), flops(fl) {
    if (ctx->profiling) {
      a = ctx->take_event();
      HIPCHK(hipEventRecord(a, st));
    }
  }
  void done() {
    if (!a) return;
    hipEvent_t b = ctx->take_event();
    HIPCHK(hipEventRecord(b, st));
    ctx->pending.push_back({cls, a, b, bytes, flops});
    a = nullptr;
  }
};

// Timing hooks handed to the constrained path (same event pairs as KTimer).
static hipEvent_t g_pending_start = nullptr;
static void hook_begin(void *c, hipStream_t st) {
  qaoa_ctx *ctx = (qaoa_ctx *)c;
  if (!ctx->profiling) return;
  g_pending_start = ctx->take_event();
  HIPCHK(hipEventRecord(g_pending_start, st));
}
static void hook_end(void *c, hipStream_t st, int cls, double bytes, double flops) {
  qaoa_ctx *ctx = (qaoa_ctx *)c;
  if (!ctx->profiling || !g_pending_start) return;
  hipEvent_t b = ctx->take_event();
  HIPCHK(hipEventRecord(b, st));
  ctx->pending.push_back({cls, g_pending_start, b, bytes, flops});
  g_pending_start = nullptr;
}

// After the stream synchronised: fold recorded event pairs into the totals.
static void profile_collect(qaoa_ctx *ctx) {
  for (auto &p : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      KTotals &t = ctx->totals[p.cls];
      t.launches++;
      t.ms += ms;
      t.bytes += p.bytes;
      t.flops += p.flops;
    }
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

// The device table holds, per feasible state, an index into the problem's distinct cost
// values (increasing order); for a graph table the index is the cost itself (values 0..max).
static uint64_t next_handle_id() {
  static std::atomic<uint64_t> c{1};
  return c++;
}

struct qaoa_problem {
  uint64_t id = next_handle_id();  // unique for the process (keys of cached graphs)
  qaoa_ctx *ctx = nullptr;
  int n = 0, k = -1;
  uint64_t N = 0;
  int tbytes = 1;
  int64_t max_value = 0;              // largest table index
  int64_t total_weight = 0;
  double mean = 0.0;  // mean of C over the feasible set (centre of the adjoint vector)
  bool sym = true;    // C(~x) = C(x) for every x (full space only)
  std::vector<double> hvals;          // cost value of each index
  double *dvals = nullptr;            // the same, device FP64 and FP32
  float *dvals_f = nullptr;
  std::vector<double> hcounts;        // degeneracy of each index (Grover mixer; filled on first use)
  double *dcounts = nullptr;
  void *table = nullptr;
  void *table_rev = nullptr;          // reversed natural table (C(~x)), when !sym
  std::map<std::tuple<int, int, int>, void *> layouts;      // (T, c, h0) -> tile-major copy
  std::map<std::tuple<int, int, int>, void *> layouts_rev;  // reversed tile-major copies
  ~qaoa_problem() {
    if (table) (void)hipFree(table);
    if (table_rev) (void)hipFree(table_rev);
    if (dvals) (void)hipFree(dvals);
    if (dvals_f) (void)hipFree(dvals_f);
    if (dcounts) (void)hipFree(dcounts);
    for (auto &kv : layouts)
      if (kv.second) (void)hipFree(kv.second);
    for (auto &kv : layouts_rev)
      if (kv.second) (void)hipFree(kv.second);
  }
};

namespace {
// Upload the index -> value map (FP64 and FP32) of a problem.
void upload_values(qaoa_problem *prob, hipStream_t st) {
  const size_t L = prob->hvals.size();
  if (hipMalloc(&prob->dvals, L * sizeof(double)) != hipSuccess ||
      hipMalloc(&prob->dvals_f, L * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    throw fail(QAOA_ERR_OUT_OF_MEMORY, "value table allocation failed");
  }
  std::vector<float> hf(L);
  for (size_t i = 0; i < L; i++) hf[i] = (float)prob->hvals[i];
  HIPCHK(hipMemcpyAsync(prob->dvals, prob->hvals.data(), L * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(prob->dvals_f, hf.data(), L * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
}
}  // namespace

struct qaoa_mixer {
  uint64_t id = next_handle_id();
  qaoa_ctx *ctx = nullptr;
  int kind = 0;  // 0: transverse field, 1: clique, 2: Grover, 3: X products, 4: per-qubit angles
  int n = 0, k = -1;
  std::unique_ptr<CliqueMixer, CliqueMixerDeleter> clique;
  // kinds 3 and 4: the mixer's diagonal after the Walsh-Hadamard transform
  XDiag xd{};
  double *xvals = nullptr;  // kind 3: diagonal value of each index (xlen entries, device)
  float *xvals_f = nullptr;  // the same in FP32
  int xlen = 0;
  ~qaoa_mixer() {
    if (xvals) (void)hipFree(xvals);
    if (xvals_f) (void)hipFree(xvals_f);
  }
};

namespace {
// angles per set: [beta_1..beta_p, gamma_1..gamma_p], or with per-qubit angles
// [beta_{1,0..n-1}, ..., beta_{p,0..n-1}, gamma_1..gamma_p]
size_t set_len(const qaoa_mixer *mix, int p) { return (size_t)p * (mix->kind == 4 ? mix->n + 1 : 2); }
}  // namespace

// ---------------------------------------------------------------- plan of the X path

namespace {

struct TileGeo {
  int c, h0;
  uint32_t rot;  // tile bits rotated by this tile
};

// Tile cover of n address bits: tile 0 holds bits [0, T); each further tile holds c contiguous
// low bits and T - c bits above the previous tile's. Fewest tiles first, runs of at least 2^cmin
// amplitudes (widest-first, as wide as allowed; two strided tiles share their bits evenly);
// when runs down to 2^cnarrow save a tile, the strided bits are spread as evenly as possible
// over the tiles instead.
std::vector<TileGeo> make_tiles(int n, int T, int cmin, int cnarrow, const PlanOpts &o) {
  std::vector<TileGeo> t;
  t.push_back({T, T, (1u << T) - 1});
  auto ntiles = [&](int c) { return n <= T ? 1 : 1 + (n - T + (T - c) - 1) / (T - c); };
  std::vector<int> widths;
  if (o.narrow && ntiles(cnarrow) < ntiles(cmin)) {
    const int ns = ntiles(cnarrow) - 1, S = n - T;
    widths.assign(ns, S / ns);
    for (int i = 0; i < S % ns; i++) widths[o.narrow_top ? ns - 1 - i : i]++;
  } else {
    for (int next = T; next < n;) {
      widths.push_back(std::min(n - next, T - cmin));
      next += widths.back();
    }
    // Two strided tiles split the strided bits evenly, the odd bit to the top tile (option
    // narrow_top) or to the middle one: measured (X mixer, fwd+grad, FP32) faster than
    // widest-first for n = 22..27 by 0.5-4.7 %, and at n = 28 (7 + 8 against 8 + 7 bits) by 1 %.
    if (widths.size() == 2) {
      const int S = widths[0] + widths[1];
      widths[0] = o.narrow_top ? S / 2 : (S + 1) / 2;
      widths[1] = S - widths[0];
    }
  }
  int next = T;
  for (int width : widths) {
    int c = T - width;
    t.push_back({c, next, ((1u << T) - 1) & ~((1u << c) - 1)});
    next += width;
  }
  // Rounds visit the tiles in vector order (alternating direction), so the middle tile runs as
  // a single-block pass and the first and last share the round boundaries (two-block passes).
  if (o.swap && t.size() == 3) std::swap(t[1], t[2]);
  if (!o.lowbits) return t;
  // Balance the rotation work between passes. The lowest T - 8 address bits (the L register
  // group) are contiguous bits of every tile, so any tile may rotate them. With three or more
  // tiles, the middle tile of a layer runs as a single-block pass (memory-bound, with spare
  // ALU time), while the first tile runs as a two-block pass; moving those bits from the
  // first tile to the second cuts the largest pass from 2T to 2(T - (T - 8)) rotations.
  if (t.size() >= 3 && t[1].c >= T - 8) {
    const uint32_t L = (1u << (T - 8)) - 1;
    t[0].rot &= ~L;
    t[1].rot |= L;
  }
  // With two tiles every pass is a two-block pass. When the second tile's contiguous bits
  // include the M register group (tile bits [T-8, 8)), it takes those qubits: the first tile
  // then rotates its H and L groups only (2 x (2T - 16) rotations per pass instead of 2T)
  // and the second tile the M and H groups.
  if (t.size() == 2 && t[1].c >= 8) {
    const uint32_t M = ((1u << 8) - 1) & ~((1u << (T - 8)) - 1);
    t[0].rot &= ~M;
    t[1].rot |= M;
  }
  return t;
}

// Whether the cover of n bits under options o uses runs narrower than 2^cmin amplitudes, and
// the swizzled layout applies to it.
bool swz_applies(int n, int T, int cmin, int cnarrow, int prec, const PlanOpts &o) {
  if (n - 10 < swz_shift(prec) + 10) return false;
  for (const TileGeo &g : make_tiles(n, T, cmin, cnarrow, o))
    if (g.c < cmin) return true;
  return false;
}

// Whether option `which` of PlanOpts changes the plan of n bits at all (the tuner skips the
// others).
bool plan_knob_applies(int which, int n, int T, int cmin, int cnarrow, const PlanOpts &o) {
  PlanOpts a = o, b = o;
  switch (which) {
    case 0: a.narrow = 1; b.narrow = 0; break;
    case 1: a.narrow_top = 1; b.narrow_top = 0; break;
    case 2: a.lowbits = 1; b.lowbits = 0; break;
    case 3: a.swap = 1; b.swap = 0; break;
    default: return false;
  }
  auto ta = make_tiles(n, T, cmin, cnarrow, a), tb = make_tiles(n, T, cmin, cnarrow, b);
  if (ta.size() != tb.size()) return true;
  for (size_t i = 0; i < ta.size(); i++)
    if (ta[i].c != tb[i].c || ta[i].h0 != tb[i].h0 || ta[i].rot != tb[i].rot) return true;
  return false;
}

// One forward pass: [rotate tile bits for layer pre] [phase of layer ph] [rotate for layer post]
struct FwdPass {
  int tile;
  int pre = -1, ph = -1, post = -1;
};

std::vector<FwdPass> make_forward(int K, int p, bool down = false) {
  std::vector<std::pair<int, int>> seq;  // (tile, layer): layers alternate tile order
  for (int k = 0; k < p; k++)
    for (int i = 0; i < K; i++) seq.push_back({((k % 2 == 0) != down) ? i : K - 1 - i, k});
  std::vector<FwdPass> out;
  out.push_back(FwdPass{seq[0].first, -1, 0, 0});
  size_t i = 1;
  while (i < seq.size()) {
    if (i + 1 < seq.size() && seq[i + 1].first == seq[i].first) {
      out.push_back(FwdPass{seq[i].first, seq[i].second, seq[i + 1].second, seq[i + 1].second});
      i += 2;
    } else {
      out.push_back(FwdPass{seq[i].first, seq[i].second, -1, -1});
      i += 1;
    }
  }
  return out;
}

// Rotation parameters of e^{-i beta X} (see the kernel file header): tau for the kernel,
// flip = 1 when the applied operator omits an X (tau = -cot beta), f = dropped scalar of the
// forward rotation, finv = of the inverse rotation.
template <typename R>
void rot_params(double beta, R &tau, int &flip, cd &f, cd &finv) {
  double sb = std::sin(beta), cb = std::cos(beta);
  if (std::fabs(sb) <= std::fabs(cb)) {
    tau = (R)(sb / cb);
    flip = 0;
    double t = (double)tau, nrm = 1.0 / std::sqrt(1.0 + t * t);
    f = cd(cb < 0 ? -nrm : nrm, 0.0);
    finv = f;
  } else {
    tau = (R)(-cb / sb);
    flip = 1;
    double t = (double)tau, s = (sb < 0 ? -1.0 : 1.0) / std::sqrt(1.0 + t * t);
    f = cd(0.0, -s);
    finv = cd(0.0, s);
  }
}

cd cpow_int(cd z, int m) {
  cd r(1.0, 0.0);
  for (int i = 0; i < m; i++) r *= z;
  return r;
}

struct OutMap {
  int nout, p;
  int m = 1;  // outputs per beta layer: 1, or with per-qubit angles 1 + n (the total, then per qubit)
  int E() const { return 0; }
  int Nr() const { return 1; }
  int gb(int k) const { return 2 + k * m; }
  int gbq(int k, int q) const { return 2 + k * m + 1 + q; }
  int gg(int k) const { return 2 + p * m + k; }
};

// Tile-major copy of the cost table for tile geometry (T, c, h0), built once per problem and
// geometry (the natural table for a contiguous tile).
const void *tile_table(qaoa_problem *prob, int T, int c, int h0, hipStream_t st) {
  if (c == T) return prob->table;
  auto key = std::make_tuple(T, c, h0);
  auto it = prob->layouts.find(key);
  if (it != prob->layouts.end()) return it->second;
  void *d = nullptr;
  if (hipMalloc(&d, prob->N * prob->tbytes) != hipSuccess) {
    (void)hipGetLastError();
    throw fail(QAOA_ERR_OUT_OF_MEMORY, "table layout allocation failed");
  }
  hipError_t e = launch_table_relayout(prob->table, d, prob->tbytes, prob->n, T, c, h0, st);
  if (e != hipSuccess) {
    (void)hipFree(d);
    throw fail(QAOA_ERR_HIP, std::string("table relayout: ") + hipGetErrorString(e));
  }
  prob->layouts[key] = d;
  return d;
}

// The tile-pass path. xm == nullptr: transverse-field mixer, layer k = phase, then a rotation
// e^{-i beta_k X} of every qubit. xm = a single-angle X-product mixer:
// 2p half-layers, each a diagonal (even: the cost phase of layer h / 2, odd: the mixer diagonal
// of layer (h - 1) / 2) followed by the basis change V^dag (even) or V (odd), V = R_y(pi/2) on
// every qubit, applied as Y rotations with tau = -1 or +1 (scalar cos(pi/4) per qubit); no
// X-pair terms, the beta gradient is taken at the mixer diagonal like the gamma gradient at
// the phase.
// Deferred evaluation (batched calls): the device work of several instances is enqueued
// back to back (or captured once as a HIP graph and replayed) and the host reads every
// result after one synchronisation. Each instance stages its parameters and results in its
// own pinned buffers.
struct XDefer {
  HostBuf *hstage;   // pinned parameter staging of this instance
  HostBuf *rstage;   // pinned result rows of this instance
  bool launch;       // false: only write the staging (the device work is a replayed graph)
  int *ckpt;         // checkpointed reverse sweep: -1 decide and record, else use the record
  std::vector<std::function<void()>> *finish;  // host work to run after the synchronisation
  uint64_t *fp;      // fingerprint of every launch and copy the instance makes (FNV-1a)
};

// FNV-1a over raw bytes (fingerprints of enqueued work: kernel arguments, sizes, pointers).
inline void fnv(uint64_t *h, const void *p, size_t n) {
  if (!h) return;
  const unsigned char *b = (const unsigned char *)p;
  for (size_t i = 0; i < n; i++) *h = (*h ^ b[i]) * 1099511628211ull;
}
template <typename T>
inline void fnv_v(uint64_t *h, const T &v) {
  fnv(h, &v, sizeof(T));
}

// Checkpointed reverse sweep: the forward passes' outputs (need bytes) are kept when they and
// one more vector fit in half of the free device memory (the context's own checkpoint buffer
// counts as free), or always when the context says so and they fit at all.
bool ckpt_fits(qaoa_ctx *ctx, size_t need, size_t vbytes) {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const size_t have = fr + ctx->ckpt.cap;
  if (need > have) return false;
  return ctx->checkpoint_mode == 1 || need + vbytes <= have / 2;
}

template <typename R>
void run_x_path(qaoa_problem *prob, int p, const double *angles, int nsets, const void *d_psi0,
                int grad, double *out_expect, double *out_grad, void *d_state_out, hipStream_t st,
                const qaoa_mixer *xm = nullptr, const XDefer *df = nullptr, const PlanOpts *force = nullptr);

// Plan options of one evaluation shape: the context's tuned choice for (n, precision, gradient,
// mixer, whether checkpoints fit), measured on first use when the context tunes, else the
// fixed rule. The angle-set count is not part of the key, so a batched call and a single
// evaluation of the same problem follow the same plan and give bit-identical results.
template <typename R>
PlanOpts plan_for(qaoa_problem *prob, int p, const double *angles, int nsets, int grad, const qaoa_mixer *xm,
                  hipStream_t st, bool may_tune);

template <typename R>
void run_x_path(qaoa_problem *prob, int p, const double *angles, int nsets, const void *d_psi0,
                int grad, double *out_expect, double *out_grad, void *d_state_out, hipStream_t st,
                const qaoa_mixer *xm, const XDefer *df, const PlanOpts *force) {
  const bool dev = !df || df->launch;  // enqueue device work
  qaoa_ctx *ctx = prob->ctx;
  const int prec = sizeof(R) == 4 ? QAOA_FP32 : QAOA_FP64;
  const int T = prec == QAOA_FP32 ? TILE_BITS_F32 : TILE_BITS_F64;
  const int cmin = prec == QAOA_FP32 ? MIN_CONTIG_F32 : MIN_CONTIG_F64;
  const int cnarrow = prec == QAOA_FP32 ? MIN_CONTIG_NARROW_F32 : MIN_CONTIG_NARROW_F64;
  const int n = prob->n;
  const PlanOpts po = force ? *force : plan_for<R>(prob, p, angles, nsets, grad, xm, st, !df);
  const std::vector<TileGeo> tiles = make_tiles(n, T, cmin, cnarrow, po);
  const int K = (int)tiles.size();
  // the swizzled layout on narrow covers of the transverse-field mixer (each of their tiles
  // rotates bits of all three register groups, the one stage set built for that layout); not
  // when the initial state comes from the caller or the final vector goes to the caller (both
  // in natural order)
  bool swz = po.swz && swz_applies(n, T, cmin, cnarrow, prec, po) && !d_psi0 && !d_state_out && !xm;
  for (const TileGeo &g : tiles) {
    const uint32_t H = ((1u << T) - 1) & ~((1u << 8) - 1), M = ((1u << 8) - 1) & ~((1u << (T - 8)) - 1),
                   Lg = (1u << (T - 8)) - 1;
    swz = swz && (g.rot & H) && (g.rot & M) && (g.rot & Lg);
  }
  const int L = xm ? 2 * p : p;  // layers of the pass plan
  const bool ma = xm && xm->kind == 4;      // per-qubit angles
  const int SL = ma ? p * (n + 1) : 2 * p;  // angles per set
  const std::vector<FwdPass> fwd = make_forward(K, L, po.down != 0);
  const uint32_t nwg = 1u << (n - T);
  const uint64_t N = 1ull << n;
  const size_t esz = 2 * sizeof(R);
  const int lut_len = (int)prob->max_value + 1;
  if (lut_len > MAX_LUT) throw fail(QAOA_ERR_UNSUPPORTED, "largest cost value exceeds the LUT limit");
  const int lut_mix = xm ? xm->xlen : 0;
  if (lut_mix > MAX_LUT) throw fail(QAOA_ERR_UNSUPPORTED, "mixer diagonal exceeds the LUT limit");

  // tile-major table copies for every geometry that reads the table
  auto table_for = [&](int tile) -> const void * { return tile_table(prob, T, tiles[tile].c, tiles[tile].h0, st); };
  // the same layouts for C(~x): the whole array reversed (complementing x complements the
  // tile index and the element index); the table itself when C(~x) = C(x)
  auto table_rev_for = [&](int tile) -> const void * {
    if (prob->sym) return table_for(tile);
    const void *src = table_for(tile);
    const TileGeo &g = tiles[tile];
    void **slot;
    if (g.c == T) slot = &prob->table_rev;
    else slot = &prob->layouts_rev[std::make_tuple(T, g.c, g.h0)];
    if (*slot) return *slot;
    void *d = nullptr;
    if (hipMalloc(&d, N * prob->tbytes) != hipSuccess) {
      (void)hipGetLastError();
      throw fail(QAOA_ERR_OUT_OF_MEMORY, "reversed table allocation failed");
    }
    hipError_t e = launch_table_reverse(src, d, prob->tbytes, N, st);
    if (e != hipSuccess) {
      (void)hipFree(d);
      throw fail(QAOA_ERR_HIP, std::string("table reverse: ") + hipGetErrorString(e));
    }
    *slot = d;
    return d;
  };

  // buffers. With enough free memory the gradient keeps every forward pass's output
  // (checkpoints) and the reverse sweep reads the state from them instead of undoing and
  // rewriting it: 24 instead of 32 bytes per amplitude in each reverse pass.
  const size_t vbytes = (size_t)nsets * N * esz;
  const int npf_est = 1 + L * ((int)tiles.size() - 1);
  bool ckpt = false;
  if (df && *df->ckpt >= 0) {
    ckpt = *df->ckpt != 0;  // the decision the captured work was planned with
  } else if (grad && ctx->checkpoint_mode != 0 && po.ckpt != 0) {
    ckpt = ckpt_fits(ctx, (size_t)npf_est * vbytes, vbytes);
  }
  if (df) *df->ckpt = ckpt ? 1 : 0;
  void *dphi = ckpt ? nullptr : ctx->phi.get(vbytes);
  unsigned char *dck = ckpt ? (unsigned char *)ctx->ckpt.get((size_t)npf_est * vbytes) : nullptr;
  // forward pass j writes checkpoint j (or the single in-place buffer)
  auto fwd_out = [&](int j) -> void * { return ckpt ? (void *)(dck + (size_t)j * vbytes) : dphi; };
  auto fwd_in = [&](int j) -> void * { return j == 0 ? nullptr : fwd_out(j - 1); };
  void *dlam = grad ? ctx->lam.get(vbytes) : nullptr;
  OutMap om{2 + p * (ma ? n + 1 : 1) + p, p, ma ? n + 1 : 1};
  const int nout = om.nout;
  const int maxc = K + 1;
  const size_t part_elems = (size_t)nout * maxc * nsets * nwg;
  double *dpart = (double *)ctx->partials.get(part_elems * sizeof(double));

  // angle-derived parameters per set and layer
  std::vector<R> tau((size_t)nsets * L);
  std::vector<int> swp((size_t)nsets * L);
  std::vector<cd> ff((size_t)nsets * L), fi((size_t)nsets * L);
  for (int s = 0; s < nsets; s++)
    for (int k = 0; k < L; k++) {
      if (xm) {  // V^dag after an even half-layer's diagonal, V after an odd one's
        tau[s * L + k] = (R)((k % 2 == 0) ? -1.0 : 1.0);
        swp[s * L + k] = 0;
        ff[s * L + k] = fi[s * L + k] = cd(std::sqrt(0.5), 0.0);
        continue;
      }
      double beta = angles[(size_t)s * SL + k];
      rot_params<R>(beta, tau[s * L + k], swp[s * L + k], ff[s * L + k], fi[s * L + k]);
    }
  // flip state of set s's stored vector after `layers` complete rounds (all bits or none):
  // 1 when an odd number of them used the tau = -cot form; only an asymmetric table cares
  auto tflip = [&](int s, int layers) {
    if (prob->sym) return 0;
    int f = 0;
    for (int k = 0; k < layers; k++) f ^= swp[s * L + k];
    return f;
  };
  // angle of the diagonal of layer k: gamma_k; with X products gamma_{k/2} (even k) or
  // beta_{(k-1)/2} (odd k, the mixer diagonal)
  auto gam = [&](int s, int k) {
    if (!xm) return angles[(size_t)s * SL + p + k];
    return (k % 2 == 0) ? angles[(size_t)s * SL + (ma ? p * n : p) + k / 2] : angles[(size_t)s * SL + (k - 1) / 2];
  };
  auto is_mix = [&](int k) { return xm != nullptr && k % 2 == 1; };
  // output slot of the derivative taken at the diagonal of layer k
  auto diag_out = [&](int k) { return !xm ? om.gg(k) : (k % 2 == 0 ? om.gg(k / 2) : om.gb((k - 1) / 2)); };

  std::vector<PassArgs<R>> passes;
  std::vector<int> nvs;     // kernel kind: 1 forward, 2 reverse, 3 fused
  std::vector<int> shapes;  // 0: part 1 only, 1: both parts, 2: part 2 only
  std::vector<int> sxs;     // register stages holding the tile's rotated bits
  std::vector<int> mixlut;  // XD_POPCOUNT / XD_TERMS: the pass's diagonal is the mixer's (LUTs in jobs_m)
  std::vector<SetParams<R>> sps;
  std::vector<LutJob> jobs, jobs_m;
  auto push_job = [&](int k, const LutJob &jb) -> int {
    std::vector<LutJob> &J = is_mix(k) ? jobs_m : jobs;
    J.push_back(jb);
    return (int)J.size() - 1;
  };
  // a pass whose diagonal is the mixer's: the mixer's values, indexed by the Hamming weight of
  // y, or by its parities against the term masks (then the register parts' indices in the
  // middle's register assignment go with the pass: register j holds tile element j << sh)
  // per-qubit angles: for pass i and set s, the register parts' factors (RN complex, staged as
  // the pass's LUT) and the constant and per-qubit factors (33 complex doubles, read by each
  // thread once); filled per pass as the plan is built, uploaded with the parameters
  const int RBq = T - 8, RNq = 1 << RBq;
  std::vector<std::complex<R>> ma_lut;
  std::vector<cd> ma_bf;
  std::vector<int> ma_block;                 // per pass: block index into the tables, or -1
  std::vector<std::array<uint64_t, 32>> ma_yreg;  // per block: the address bits of register j
  // register assignment of the middle (after part 1's stages H, M, L in order)
  auto middle_shift = [&](int tile) {
    const uint32_t rot = tiles[tile].rot;
    const bool Lg = rot & ((1u << RBq) - 1), Mg = rot & (((1u << 8) - 1) & ~((1u << RBq) - 1));
    return Lg ? 0 : (Mg ? T - 2 * RBq : 8);
  };
  auto ma_fill = [&](int block, int s, int layer, cd scale, double sgn) {
    // D(y) = e^{-i sum_q b_q} prod_{q in y} e^{2i b_q} (forward, sgn = 1); the inverse with sgn = -1
    const double *b = angles + (size_t)s * SL + (size_t)layer * n;
    double B = 0.0;
    for (int qq = 0; qq < n; qq++) B += b[qq];
    cd *bf = &ma_bf[((size_t)block * nsets + s) * 33];
    bf[0] = scale * std::polar(1.0, -sgn * B);
    for (int qq = 0; qq < 32; qq++) bf[1 + qq] = qq < n ? std::polar(1.0, 2.0 * sgn * b[qq]) : cd(1.0, 0.0);
    std::complex<R> *L = &ma_lut[((size_t)block * nsets + s) * RNq];
    for (int jj = 0; jj < RNq; jj++) {
      cd v(1.0, 0.0);
      for (int qq = 0; qq < n; qq++)
        if ((ma_yreg[block][jj] >> qq) & 1) v *= bf[1 + qq];
      L[jj] = std::complex<R>((R)v.real(), (R)v.imag());
    }
  };
  auto ma_new_block = [&](PassArgs<R> &a, int tile) -> int {
    const int block = (int)ma_yreg.size();
    std::array<uint64_t, 32> yr{};
    const int sh = middle_shift(tile);
    const uint64_t cmask = (1ull << a.c) - 1;
    for (int jj = 0; jj < RNq; jj++) {
      const uint64_t e = (uint64_t)jj << sh;
      yr[jj] = (e & cmask) | ((e >> a.c) << a.h0);
    }
    ma_yreg.push_back(yr);
    ma_lut.resize((size_t)(block + 1) * nsets * RNq);
    ma_bf.resize((size_t)(block + 1) * nsets * 33);
    // where each qubit sits in the middle's register assignment
    const int MLO = T - 2 * RBq;
    for (int qq = 0; qq < 32; qq++) {
      int tb = -1;
      if (qq < a.c) tb = qq;
      else if (qq >= a.h0 && qq < a.h0 + T - a.c) tb = a.c + (qq - a.h0);
      int src = 16;
      if (tb >= 0) {
        if (sh == 8) src = tb >= 8 ? tb - 8 : 8 + tb;
        else if (sh == 0) src = tb < RBq ? tb : 8 + (tb - RBq);
        else src = (tb >= MLO && tb < MLO + RBq) ? tb - MLO : (tb < MLO ? 8 + tb : 8 + (tb - RBq));
      }
      a.ma_src[qq] = (int8_t)(qq < n ? src : 16);
    }
    a.lut_len = RNq;
    return block;
  };
  auto mix_diag = [&](PassArgs<R> &a, int tile) {
    a.vals = sizeof(R) == 4 ? (const void *)xm->xvals_f : (const void *)xm->xvals;
    a.lut_len = lut_mix;
    a.lam_c0 = (R)0;
    if (ma) return;
    if (xm->xd.mode != XD_TERMS) return;
    a.xnterms = xm->xd.nterms;
    for (int k = 0; k < XD_MAX_TERMS; k++) a.xmasks[k] = k < xm->xd.nterms ? xm->xd.masks[k] : 0;
    const uint32_t rot = tiles[tile].rot;
    const int RB = T - 8, MLO = T - 2 * RB;
    const bool Lg = rot & ((1u << RB) - 1), Mg = rot & (((1u << 8) - 1) & ~((1u << RB) - 1));
    const int sh = Lg ? 0 : (Mg ? MLO : 8);  // assignment after part 1 (stages H, M, L in order)
    const uint64_t cmask = (1ull << a.c) - 1;
    for (int j = 0; j < 32; j++) {
      if (j >= (1 << RB)) {
        a.xreg[j] = 0;
        continue;
      }
      const uint64_t e = (uint64_t)j << sh, y = (e & cmask) | ((e >> a.c) << a.h0);
      uint32_t idx = 0;
      for (int k = 0; k < xm->xd.nterms; k++) idx |= (uint32_t)(__builtin_popcountll(y & xm->xd.masks[k]) & 1) << k;
      a.xreg[j] = (uint16_t)idx;
    }
  };
  std::vector<int> cnt(nout, 0);
  auto slot_for = [&](int o) -> int64_t {
    int c = cnt[o]++;
    if (c >= maxc) throw fail(QAOA_ERR_HIP, "internal: too many contributions");
    return ((int64_t)o * maxc + c) * nsets * (int64_t)nwg;
  };
  auto base_args = [&](int tile) {
    PassArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.c = tiles[tile].c;
    a.h0 = tiles[tile].h0;
    a.nwg = nwg;
    a.xcd_remap = (nwg >= 8 && po.xcd) ? 1 : 0;
    a.nsets = nsets;
    a.vstride = N;
    a.phi = dphi;
    a.phi_out = dphi;
    a.lam = dlam;
    a.psi0 = d_psi0;
    a.table = nullptr;
    a.table_rev = nullptr;
    a.vals = sizeof(R) == 4 ? (const void *)prob->dvals_f : (const void *)prob->dvals;
    a.luts = nullptr;  // patched after upload
    a.lut_len = lut_len;
    a.u0 = (R)(1.0 / std::sqrt((double)N));
    a.lam_c0 = (R)prob->mean;
    a.partials = dpart;
    for (int s = 0; s < NSLOT; s++) a.slot_off[s] = -1;
    if (swz) {
      a.swz = swz_shift(prec);
      a.swz_src = n - 10;
      a.swz_add = tiles[tile].h0 + (T - tiles[tile].c) <= a.swz_src ? 1 : 0;
      // runs under a 128-byte line: the two workgroups that share each line meet in L2
      a.cached = ((size_t)1 << tiles[tile].c) * esz < 128 ? 1 : 0;
    }
    return a;
  };

  std::vector<cd> sig(nsets, cd(1.0, 0.0));
  std::vector<cd> sig_fwd;  // [pass][set]: scalar of forward pass j's output
  auto rotbits = [&](int tile) { return __builtin_popcount(tiles[tile].rot); };
  // register groups of the pass kernels: H = tile bits [8,T), M = [T-8, 8), L = [0, T-8)
  auto stage_set = [&](int tile) {
    const uint32_t rot = tiles[tile].rot, RB = T - 8;
    const uint32_t H = ((1u << T) - 1) & ~((1u << 8) - 1), M = ((1u << 8) - 1) & ~((1u << RB) - 1),
                   L = (1u << RB) - 1;
    int sx = ((rot & H) ? 1 : 0) | ((rot & M) ? 2 : 0) | ((rot & L) ? 4 : 0);
    if (sx != 7 && sx != 5 && sx != 3 && sx != 1) throw fail(QAOA_ERR_HIP, "internal: unsupported tile stage set");
    return sx;
  };
  auto add_pass = [&](const PassArgs<R> &a, int kind, int shape, int tile, int mixd = 0, int mblock = -1) {
    passes.push_back(a);
    nvs.push_back(kind);
    shapes.push_back(shape);
    sxs.push_back(stage_set(tile));
    mixlut.push_back(mixd);
    ma_block.push_back(mblock);
  };
  const int npf = (int)fwd.size();

  // ---------------- forward passes (all but the last)
  if (npf != npf_est) throw fail(QAOA_ERR_HIP, "internal: pass count");
  for (int j = 0; j < npf - 1; j++) {
    const FwdPass &fp = fwd[j];
    PassArgs<R> a = base_args(fp.tile);
    a.phi = fwd_in(j);
    a.phi_out = fwd_out(j);
    uint32_t f = 0;
    if (j == 0) f |= d_psi0 ? PF_LOAD_PSI0 : PF_GEN_PHI;
    else f |= PF_LOAD_PHI;
    f |= PF_STORE_PHI;
    if (fp.pre >= 0) a.mask1 = tiles[fp.tile].rot;
    int mblock = -1;
    if (fp.ph >= 0) {
      f |= PF_PHASE;
      if (is_mix(fp.ph)) {
        mix_diag(a, fp.tile);
        if (ma) mblock = ma_new_block(a, fp.tile);
      } else {
        a.table = table_for(fp.tile);
        a.table_rev = xm ? a.table : table_rev_for(fp.tile);
      }
    }
    if (fp.post >= 0) a.mask2 = tiles[fp.tile].rot;
    a.flags = f;
    for (int s = 0; s < nsets; s++) {
      SetParams<R> q;
      std::memset(&q, 0, sizeof(q));
      q.lut = -1;
      q.w1 = q.w2 = 1.0;
      q.lam_rho = (R)1;
      if (fp.pre >= 0) {
        q.tau1 = tau[s * L + fp.pre];
        sig[s] *= cpow_int(ff[s * L + fp.pre], rotbits(fp.tile));
      }
      if (fp.ph >= 0) {
        q.tflip = tflip(s, fp.ph);
        if (mblock >= 0) {
          ma_fill(mblock, s, (fp.ph - 1) / 2, sig[s], 1.0);
          q.lut = s;
        } else {
          q.lut = push_job(fp.ph, LutJob{gam(s, fp.ph), sig[s].real(), sig[s].imag(), -1.0});
        }
        sig[s] = cd(1.0, 0.0);
      }
      if (fp.post >= 0) {
        q.tau2 = tau[s * L + fp.post];
        sig[s] *= cpow_int(ff[s * L + fp.post], rotbits(fp.tile));
      }
      sps.push_back(q);
    }
    add_pass(a, 1, fp.pre < 0 ? 2 : (fp.post >= 0 ? 1 : 0), fp.tile, fp.ph >= 0 && is_mix(fp.ph) ? xm->xd.mode : 0,
             mblock);
    sig_fwd.insert(sig_fwd.end(), sig.begin(), sig.end());
  }

  // ---------------- last forward pass (alone, or fused with the start of the reverse sweep)
  const FwdPass &lp = fwd[npf - 1];
  std::vector<cd> sig_pre_last = sig;
  std::vector<cd> sig_p(nsets);
  std::vector<double> rho(nsets);
  {
    PassArgs<R> a = base_args(lp.tile);
    a.phi = fwd_in(npf - 1);
    a.phi_out = fwd_out(npf - 1);
    uint32_t f = (npf == 1) ? (d_psi0 ? PF_LOAD_PSI0 : PF_GEN_PHI) : PF_LOAD_PHI;
    // a single-pass plan would need the phase too; K >= 2 always gives >= 2 passes
    a.mask1 = tiles[lp.tile].rot;
    a.table = table_for(lp.tile);
    a.table_rev = xm ? a.table : table_rev_for(lp.tile);
    f |= PF_EXPECT;
    a.slot_off[SL_A] = slot_for(om.E());
    a.slot_off[SL_B] = slot_for(om.Nr());
    if (d_state_out) f |= PF_STORE_PHI;
    if (grad) {
      f |= PF_LAMBDA | PF_XT2 | PF_ROT2_BOTH | PF_STORE_LAM;
      a.mask2 = tiles[lp.tile].rot;
      if (!xm) a.slot_off[SL_C] = slot_for(om.gb(lp.pre));
    }
    a.flags = f;
    for (int s = 0; s < nsets; s++) {
      SetParams<R> q;
      std::memset(&q, 0, sizeof(q));
      q.lut = -1;
      q.tflip = tflip(s, L);
      q.tau1 = tau[s * L + lp.pre];
      sig[s] *= cpow_int(ff[s * L + lp.pre], rotbits(lp.tile));
      sig_p[s] = sig[s];
      double t = (double)q.tau1;
      rho[s] = std::pow(1.0 / (1.0 + t * t), rotbits(lp.tile));
      q.lam_rho = (R)rho[s];
      q.w1 = 1.0;
      q.w2 = std::norm(sig_p[s]) / (double)q.lam_rho;
      q.tau2 = -q.tau1;
      sps.push_back(q);
    }
    if (grad) add_pass(a, 3, 1, lp.tile);
    else add_pass(a, 1, 3, lp.tile);
  }

  // ---------------- reverse sweep
  if (grad) {
    // after the fused pass: phi (memory) and lam share the scalar sig_pre_last
    std::vector<cd> sb = sig_pre_last;
    for (int j = npf - 2; j >= 0; j--) {
      const FwdPass &fp = fwd[j];
      PassArgs<R> a = base_args(fp.tile);
      // the state after forward pass j: its checkpoint, or the vector undone in place
      a.phi = ckpt ? fwd_out(j) : dphi;
      a.phi_out = a.phi;
      // A checkpoint carries the forward sweep's scalar sig_fwd, lam the reverse sweep's sb.
      // When their ratio kappa is real and positive for every set (always, by the choice of
      // the reverse phase tables' scalars below), phi is used as stored and kappa goes into
      // the inner-product weights; otherwise phi is rescaled by kappa on load.
      bool kappa_real = ckpt;
      std::vector<double> kap(nsets, 1.0);
      if (ckpt)
        for (int s = 0; s < nsets; s++) {
          const cd kappa = sig_fwd[(size_t)j * nsets + s] / sb[s];
          kap[s] = kappa.real();
          if (!(kappa.real() > 0.0) || std::fabs(kappa.imag()) > 1e-12 * kappa.real()) kappa_real = false;
        }
      uint32_t f = PF_LOAD_PHI | PF_LOAD_LAM | ((ckpt && !kappa_real) ? (uint32_t)PF_LOAD_SCALE : 0u);
      const bool last = (j == 0);
      // part 1 undoes the forward pass's last rotation block
      int l1 = fp.post >= 0 ? fp.post : fp.pre;
      a.mask1 = tiles[fp.tile].rot;
      f |= PF_XT1 | PF_ROT1_BOTH;
      if (!xm) a.slot_off[SL_A] = slot_for(om.gb(l1));
      int mblock = -1;
      if (fp.ph >= 0) {
        f |= PF_GGAMMA;
        if (is_mix(fp.ph)) {
          mix_diag(a, fp.tile);
          if (ma) mblock = ma_new_block(a, fp.tile);
        } else {
          a.table = table_for(fp.tile);
          a.table_rev = xm ? a.table : table_rev_for(fp.tile);
        }
        if (mblock >= 0) {
          // the total and the per-qubit sums of layer k: consecutive outputs, one contribution each
          const int k = (fp.ph - 1) / 2;
          a.ma_total = slot_for(om.gb(k));
          a.ma_slot = slot_for(om.gbq(k, 0));
          a.ma_stride = (int64_t)maxc * nsets * (int64_t)nwg;
          for (int qq = 1; qq < n; qq++)
            if (slot_for(om.gbq(k, qq)) != a.ma_slot + qq * a.ma_stride)
              throw fail(QAOA_ERR_HIP, "internal: per-qubit slots");
        } else {
          a.slot_off[SL_B] = slot_for(diag_out(fp.ph));
        }
        if (!last) f |= PF_PHASE | PF_PHASE_BOTH;
      }
      const bool has2 = (fp.post >= 0 && fp.pre >= 0);
      if (has2) {
        a.mask2 = tiles[fp.tile].rot;
        f |= PF_XT2 | PF_ROT2_BOTH;
        if (!xm) a.slot_off[SL_C] = slot_for(om.gb(fp.pre));
      }
      if (!last) f |= (ckpt ? 0u : (uint32_t)PF_STORE_PHI) | PF_STORE_LAM;
      a.flags = f;
      for (int s = 0; s < nsets; s++) {
        SetParams<R> q;
        std::memset(&q, 0, sizeof(q));
        q.lut = -1;
        q.lam_rho = (R)1;
        if (fp.ph >= 0) q.tflip = tflip(s, fp.ph);
        double wk = 1.0;  // kappa, when it is a weight
        if (ckpt && !kappa_real) {
          // rescale the checkpoint to the reverse sweep's scalar (phi and lam share one)
          const cd kappa = sig_fwd[(size_t)j * nsets + s] / sb[s];
          q.out_re = (R)kappa.real();
          q.out_im = (R)kappa.imag();
        } else if (ckpt) {
          wk = kap[s];
        }
        q.w1 = std::norm(sb[s]) * wk;
        q.tau1 = -tau[s * L + l1];
        sb[s] *= cpow_int(fi[s * L + l1], rotbits(fp.tile));
        q.w2 = 1.0;
        if (fp.ph >= 0 && !last) {
          // the table takes sb / t and lam leaves the phase with scalar t; with checkpoints
          // t is chosen so that lam reaches the next checkpoint with its scalar, which makes
          // the next pass's kappa exactly 1
          cd t(1.0, 0.0);
          if (ckpt && has2) t = sig_fwd[(size_t)(j - 1) * nsets + s] / cpow_int(fi[s * L + fp.pre], rotbits(fp.tile));
          const cd fold = sb[s] / t;
          if (mblock >= 0) {
            ma_fill(mblock, s, (fp.ph - 1) / 2, fold, -1.0);
            q.lut = s;
          } else {
            q.lut = push_job(fp.ph, LutJob{gam(s, fp.ph), fold.real(), fold.imag(), 1.0});
          }
          sb[s] = t;
        }
        if (has2) {
          q.w2 = std::norm(sb[s]) * wk;
          q.tau2 = -tau[s * L + fp.pre];
          sb[s] *= cpow_int(fi[s * L + fp.pre], rotbits(fp.tile));
        }
        sps.push_back(q);
      }
      // with checkpoints phi is read and never stored: the kind that compiles its store out
      add_pass(a, ckpt ? 4 : 2, has2 ? 1 : (fp.ph >= 0 ? 3 : 0), fp.tile, fp.ph >= 0 && is_mix(fp.ph) ? xm->xd.mode : 0,
               mblock);
    }
  }

  // ---------------- upload parameters (one copy), LUTs on the device
  const size_t sp_bytes = sps.size() * sizeof(SetParams<R>);
  const size_t job_bytes = jobs.size() * sizeof(LutJob), jobm_bytes = jobs_m.size() * sizeof(LutJob);
  const size_t cnt_bytes = nout * sizeof(int);
  const size_t mal_bytes = ma_lut.size() * sizeof(std::complex<R>), mab_bytes = ma_bf.size() * sizeof(cd);
  const size_t off_jobs = (sp_bytes + 255) & ~size_t(255);
  const size_t off_jobm = (off_jobs + job_bytes + 255) & ~size_t(255);
  const size_t off_cnt = (off_jobm + jobm_bytes + 255) & ~size_t(255);
  const size_t off_mal = (off_cnt + cnt_bytes + 255) & ~size_t(255);
  const size_t off_mab = (off_mal + mal_bytes + 255) & ~size_t(255);
  const size_t total = off_mab + mab_bytes;
  unsigned char *h = (unsigned char *)(df ? df->hstage : &ctx->hparams)->get(total);
  // the previous call may still read the pinned staging buffer through its async copy (a
  // deferred instance owns its staging until the call's synchronisation)
  if (!df) HIPCHK(hipStreamSynchronize(st));
  std::memcpy(h, sps.data(), sp_bytes);
  if (job_bytes) std::memcpy(h + off_jobs, jobs.data(), job_bytes);
  if (jobm_bytes) std::memcpy(h + off_jobm, jobs_m.data(), jobm_bytes);
  std::memcpy(h + off_cnt, cnt.data(), cnt_bytes);
  if (mal_bytes) std::memcpy(h + off_mal, ma_lut.data(), mal_bytes);
  if (mab_bytes) std::memcpy(h + off_mab, ma_bf.data(), mab_bytes);
  unsigned char *d = (unsigned char *)ctx->params.get(total);
  uint64_t *fp = df ? df->fp : nullptr;
  fnv_v(fp, d);
  fnv_v(fp, h);
  fnv_v(fp, total);
  fnv_v(fp, jobs.size());
  fnv_v(fp, jobs_m.size());
  fnv_v(fp, lut_len);
  if (dev) HIPCHK(hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, st));
  void *dluts = nullptr;
  if (!jobs.empty()) {
    dluts = ctx->luts.get(jobs.size() * (size_t)lut_len * esz);
    if (dev)
      HIPCHK(launch_luts(prec, (const LutJob *)(d + off_jobs), (int)jobs.size(), lut_len, prob->dvals, dluts, st));
  }
  void *dluts_m = nullptr;
  if (!jobs_m.empty()) {
    dluts_m = ctx->luts2.get(jobs_m.size() * (size_t)lut_mix * esz);
    if (dev)
      HIPCHK(launch_luts(prec, (const LutJob *)(d + off_jobm), (int)jobs_m.size(), lut_mix, xm->xvals, dluts_m, st));
  }
  fnv_v(fp, dluts);
  fnv_v(fp, dluts_m);
  // ---------------- passes
  for (size_t i = 0; i < passes.size(); i++) {
    PassArgs<R> &a = passes[i];
    a.sp = (const SetParams<R> *)(d + i * nsets * sizeof(SetParams<R>));
    a.luts = mixlut[i] ? dluts_m : dluts;
    if (ma_block[i] >= 0) {
      a.luts = d + off_mal + (size_t)ma_block[i] * nsets * RNq * sizeof(std::complex<R>);
      a.vals = d + off_mab + (size_t)ma_block[i] * nsets * 33 * sizeof(cd);
    }
    fnv(fp, &a, sizeof(a));
    fnv_v(fp, nvs[i]);
    fnv_v(fp, sxs[i]);
    fnv_v(fp, shapes[i]);
    fnv_v(fp, mixlut[i]);
    if (!dev) continue;
    const uint32_t fl = a.flags;
    double by = 0;
    if (fl & (PF_LOAD_PHI | PF_LOAD_PSI0)) by += (double)N * esz;
    if (fl & PF_LOAD_LAM) by += (double)N * esz;
    if (fl & PF_STORE_PHI) by += (double)N * esz;
    if (fl & PF_STORE_LAM) by += (double)N * esz;
    if ((fl & (PF_EXPECT | PF_LAMBDA | PF_GGAMMA | PF_PHASE)) && !mixlut[i]) by += (double)N * prob->tbytes;
    by *= nsets;
    KTimer kt(ctx, st, xm ? QAOA_KC_XMIX : (nvs[i] >= 2 ? QAOA_KC_REV_PASS : QAOA_KC_FWD_PASS), by, 0.0);
    hipError_t e;
    if (xm) {
      if constexpr (sizeof(R) == 4) e = launch_hpass_f32(a, nvs[i], sxs[i], shapes[i], prob->tbytes, mixlut[i], st);
      else e = launch_hpass_f64(a, nvs[i], sxs[i], shapes[i], prob->tbytes, mixlut[i], st);
    } else {
      if constexpr (sizeof(R) == 4) e = launch_pass_f32(a, nvs[i], sxs[i], shapes[i], prob->tbytes, st);
      else e = launch_pass_f64(a, nvs[i], sxs[i], shapes[i], prob->tbytes, st);
    }
    if (e != hipSuccess) throw fail(QAOA_ERR_HIP, std::string("pass launch: ") + hipGetErrorString(e));
    kt.done();
  }
  // ---------------- reductions
  double *dres = (double *)ctx->results.get((size_t)nsets * nout * sizeof(double));
  if (dev) {
    KTimer kt(ctx, st, QAOA_KC_OTHER, (double)part_elems * 8.0, 0.0);
    HIPCHK(launch_finalize(dpart, (const int *)(d + off_cnt), maxc, nsets, nwg, nout, dres, st));
    kt.done();
  }
  double *hres = (double *)(df ? df->rstage : &ctx->hresults)->get((size_t)nsets * nout * sizeof(double));
  fnv_v(fp, dres);
  fnv_v(fp, hres);
  fnv_v(fp, dpart);
  fnv_v(fp, nout);
  fnv_v(fp, maxc);
  if (dev) HIPCHK(hipMemcpyAsync(hres, dres, (size_t)nsets * nout * sizeof(double), hipMemcpyDeviceToHost, st));
  if (d_state_out) {
    // nsets == 1 here: final state(x) = sigma_p * phi(x ^ F), F = all bits when an odd
    // number of rounds used the tau = -cot form
    int odd = 0;
    for (int k = 0; k < p; k++) odd ^= swp[k];
    const uint64_t flip = odd ? (N - 1) : 0;
    HIPCHK(launch_scale_copy(prec, fwd_out(npf - 1), d_state_out, N, sig_p[0].real(), sig_p[0].imag(),
                             flip, st));
  }
  auto read_out = [=]() {
  for (int s = 0; s < nsets; s++) {
    const double *r = hres + (size_t)s * nout;
    const double E = r[om.E()], Nr = r[om.Nr()];
    if (out_expect) out_expect[s] = E / Nr;
    if (grad && out_grad) {
      const double ntrue = std::norm(sig_p[s]) * Nr;
      for (int k = 0; k < p; k++) {
        if (ma) {  // g_q = 2 (S - 2 S_q): S over all states, S_q over those with bit q set
          for (int qq = 0; qq < n; qq++)
            out_grad[(size_t)s * SL + (size_t)k * n + qq] = 2.0 * (r[om.gb(k)] - 2.0 * r[om.gbq(k, qq)]) / ntrue;
          out_grad[(size_t)s * SL + (size_t)p * n + k] = 2.0 * r[om.gg(k)] / ntrue;
          continue;
        }
        out_grad[(size_t)s * SL + k] = 2.0 * r[om.gb(k)] / ntrue;
        out_grad[(size_t)s * SL + p + k] = 2.0 * r[om.gg(k)] / ntrue;
      }
    }
  }
  };
  if (df) {
    df->finish->push_back(read_out);
    return;
  }
  HIPCHK(hipStreamSynchronize(st));
  profile_collect(ctx);
  read_out();
}

// Whole-state path: items of n <= SMALL_MAX_N, one workgroup each.
void run_small(const std::vector<SmallItem> &items_in, int precision, const double *angles, int nsets,
               int p, int grad, double *hout, qaoa_ctx *ctx, hipStream_t st,
               std::vector<std::function<void()>> *finish = nullptr, bool launch = true, uint64_t *fp = nullptr) {
  // items whose state fits the register-resident kernel go first, grouped by (n, table width);
  // the rest run in the LDS kernel
  std::vector<SmallItem> items;
  std::vector<std::tuple<int, int, size_t, size_t>> groups;  // n, tbytes, first, count (first = LDS kernel)
  for (int n : {12, 13})
    for (int tb : {1, 2}) {
      if (!whole_supported(precision, n)) continue;
      const size_t first = items.size();
      for (auto &it : items_in)
        if (it.n == n && it.tbytes == tb) items.push_back(it);
      if (items.size() > first) groups.emplace_back(n, tb, first, items.size() - first);
    }
  const size_t nwhole = items.size();
  int max_n = 1, max_tb = 1, max_lut = 1;
  for (auto &it : items_in) {
    max_lut = std::max(max_lut, it.lut_len);
    if (whole_supported(precision, it.n)) continue;
    items.push_back(it);
    max_n = std::max(max_n, it.n);
    max_tb = std::max(max_tb, it.tbytes);
  }
  max_lut = (max_lut + 15) & ~15;
  const int rowlen = 1 + 2 * p;
  size_t ib = items.size() * sizeof(SmallItem);
  size_t ab = (size_t)nsets * 2 * p * sizeof(double);
  size_t off_a = (ib + 255) & ~size_t(255);
  size_t total = off_a + ab;
  // With p <= 1024 the angle set fits in LDS beside the state: the kernels copy it in at the
  // start, so items and angles stay in mapped host memory and no copy precedes the launch (the
  // previous call's kernels have finished: every call synchronises its stream before returning).
  const int stage = p <= 1024 ? 1 : 0;
  if (!stage && finish) throw fail(QAOA_ERR_UNSUPPORTED, "deferred whole-state launches need p <= 1024");
  unsigned char *d;
  if (stage) {
    ctx->small_params.get(total);
    unsigned char *h = (unsigned char *)ctx->small_params.h;
    std::memcpy(h, items.data(), ib);
    std::memcpy(h + off_a, angles, ab);
    d = (unsigned char *)ctx->small_params.d;
  } else {
    // the pinned staging buffer is shared with other calls' uploads: wait for them first
    HIPCHK(hipStreamSynchronize(st));
    unsigned char *h = (unsigned char *)ctx->hparams.get(total);
    std::memcpy(h, items.data(), ib);
    std::memcpy(h + off_a, angles, ab);
    d = (unsigned char *)ctx->items.get(total);
    HIPCHK(hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, st));
  }
  int nrow = 0;
  for (auto &it : items) nrow = std::max(nrow, it.out_index + 1);
  // the kernels write their result rows straight into mapped host memory
  ctx->small_out.get((size_t)nrow * rowlen * sizeof(double));
  double *dres = (double *)ctx->small_out.d;
  const SmallItem *ditems = (const SmallItem *)d;
  const double *dang = (const double *)(d + off_a);
  fnv_v(fp, d);
  fnv_v(fp, dres);
  fnv_v(fp, total);
  fnv_v(fp, max_lut);
  for (auto &g : groups) fnv_v(fp, g);
  fnv_v(fp, items.size());
  fnv_v(fp, nwhole);
  // algorithmic work per item: the table read once; FP32 flops of the method per amplitude:
  // 6 per qubit rotation and 6 per phase multiply in each layer, and with the gradient the
  // same again on the state and on the adjoint vector plus 4 per qubit and 4 per layer for
  // the derivative sums; 4 for <C> and the norm
  auto work = [&](size_t first, size_t count, double &by, double &fl) {
    by = fl = 0.0;
    for (size_t i = first; i < first + count; i++) {
      const SmallItem &it = items[i];
      const double N = (double)(1ull << it.n);
      by += (double)it.tbytes * N;
      fl += (double)p * N * (grad ? 22.0 * it.n + 22.0 : 6.0 * it.n + 6.0) + 4.0 * N;
    }
  };
  for (auto &g : groups) {
    if (!launch) break;
    double by, fl;
    work(std::get<2>(g), std::get<3>(g), by, fl);
    KTimer kt(ctx, st, QAOA_KC_SMALL, by, fl);
    HIPCHK(launch_whole(precision, std::get<0>(g), std::get<1>(g), ditems + std::get<2>(g), (int)std::get<3>(g),
                        max_lut, dang, p, grad, dres, st, stage));
    kt.done();
  }
  if (items.size() > nwhole && launch) {
    double by, fl;
    work(nwhole, items.size() - nwhole, by, fl);
    KTimer kt(ctx, st, QAOA_KC_SMALL, by, fl);
    HIPCHK(launch_small(precision, ditems + nwhole, (int)(items.size() - nwhole), max_n, max_tb, max_lut, dang, p,
                        grad, dres, st, stage));
    kt.done();
  }
  const void *src = ctx->small_out.h;
  const size_t rbytes = (size_t)nrow * rowlen * sizeof(double);
  if (finish) {
    finish->push_back([=]() { std::memcpy(hout, src, rbytes); });
    return;
  }
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(hout, src, rbytes);
  profile_collect(ctx);
}

void check_angles(int p, const double *angles, size_t count) {
  REQUIRE(p >= 1 && p <= 4096, "p must be in [1, 4096]");
  REQUIRE(angles != nullptr, "angles is NULL");
  for (size_t i = 0; i < count; i++) REQUIRE(std::isfinite(angles[i]), "angles must be finite");
}

void check_pair(const qaoa_problem *prob, const qaoa_mixer *mix, int precision) {
  REQUIRE(prob && mix, "problem or mixer is NULL");
  REQUIRE(prob->ctx == mix->ctx, "problem and mixer belong to different contexts");
  REQUIRE(precision == QAOA_FP32 || precision == QAOA_FP64, "precision must be QAOA_FP32 or QAOA_FP64");
  REQUIRE(prob->n == mix->n, "mixer and problem have different qubit counts");
  if (mix->kind == 0 || mix->kind == 3 || mix->kind == 4)
    REQUIRE(prob->k < 0, "X-type mixers need an unconstrained problem");
  else REQUIRE(prob->k == mix->k, "the mixer's Hamming weight differs from the problem's");
  if (mix->kind != 2 && !prob->table)
    throw fail(QAOA_ERR_UNSUPPORTED, "the problem holds degeneracies only: it serves the Grover mixer");
}

bool small_path(const qaoa_problem *prob, int precision) {
  return prob->n <= (precision == QAOA_FP32 ? SMALL_MAX_N_F32 : SMALL_MAX_N_F64);
}

SmallItem small_item(const qaoa_problem *prob, int set, int row) {
  SmallItem it;
  it.table = prob->table;
  it.vals = prob->dvals;
  it.sym = prob->sym ? 1 : 0;
  it.n = prob->n;
  it.tbytes = prob->tbytes;
  it.lut_len = (int)prob->max_value + 1;
  it.angle_set = set;
  it.c0 = prob->mean;
  it.out_index = row;
  return it;
}

// ---------------------------------------------------------------- Grover mixer

// Degeneracy of every table index (histogram of the stored table), on first use.
void ensure_counts(qaoa_problem *prob, hipStream_t st) {
  if (!prob->hcounts.empty()) return;
  const int nb = (int)prob->max_value + 1;
  if (nb > GROVER_MAX_CLASSES) throw fail(QAOA_ERR_UNSUPPORTED, "more than 2048 cost classes for the Grover mixer");
  DevBuf dc;
  unsigned long long *d = (unsigned long long *)dc.get((size_t)nb * sizeof(unsigned long long));
  HIPCHK(hipMemsetAsync(d, 0, (size_t)nb * sizeof(unsigned long long), st));
  HIPCHK(launch_hist_table(prob->table, prob->tbytes, prob->N, nb, d, st));
  std::vector<unsigned long long> h(nb);
  HIPCHK(hipMemcpyAsync(h.data(), d, (size_t)nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> c(nb);
  for (int i = 0; i < nb; i++) c[i] = (double)h[i];
  if (hipMalloc(&prob->dcounts, (size_t)nb * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    prob->dcounts = nullptr;
    throw fail(QAOA_ERR_OUT_OF_MEMORY, "degeneracy allocation failed");
  }
  HIPCHK(hipMemcpyAsync(prob->dcounts, c.data(), (size_t)nb * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  prob->hcounts = c;
}

GroverItem grover_item(const qaoa_problem *prob, int set, int row) {
  GroverItem it;
  it.vals = prob->dvals;
  it.counts = prob->dcounts;
  it.nclass = (int)prob->hcounts.size();
  it.angle_set = set;
  it.out_index = row;
  it.total = (double)prob->N;
  it.c0 = prob->mean;
  it.amp_out = nullptr;
  return it;
}

// Grover-mixer items (one workgroup each, FP64 on the cost classes); hout rows of 1 + 2p.
void run_grover(const std::vector<GroverItem> &items, const double *angles, int nsets, int p, int grad,
                double *hout, qaoa_ctx *ctx, hipStream_t st) {
  const int rowlen = 1 + 2 * p;
  size_t ib = items.size() * sizeof(GroverItem);
  size_t ab = (size_t)nsets * 2 * p * sizeof(double);
  size_t off_a = (ib + 255) & ~size_t(255);
  unsigned char *h = (unsigned char *)ctx->hparams.get(off_a + ab);
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(h, items.data(), ib);
  std::memcpy(h + off_a, angles, ab);
  unsigned char *d = (unsigned char *)ctx->gitems.get(off_a + ab);
  HIPCHK(hipMemcpyAsync(d, h, off_a + ab, hipMemcpyHostToDevice, st));
  int nrow = 0;
  for (auto &it : items) nrow = std::max(nrow, it.out_index + 1);
  double *dres = (double *)ctx->results.get((size_t)nrow * rowlen * sizeof(double));
  double work = 0;
  for (auto &it : items) work += (double)it.nclass;
  KTimer kt(ctx, st, QAOA_KC_GROVER, work * 8.0 * 2.0, 0.0);
  HIPCHK(launch_grover((const GroverItem *)d, (int)items.size(), (const double *)(d + off_a), p, grad, dres, st));
  kt.done();
  HIPCHK(hipMemcpyAsync(hout, dres, (size_t)nrow * rowlen * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  profile_collect(ctx);
}

void evaluate_grover(qaoa_problem *prob, int p, const double *angles, int nsets, const void *d_psi0, int precision,
                     int grad, double *out_expect, double *out_grad, void *d_state, hipStream_t st) {
  if (d_psi0) throw fail(QAOA_ERR_UNSUPPORTED, "the Grover mixer path starts from the equal superposition only");
  ensure_counts(prob, st);
  std::vector<GroverItem> items;
  for (int s = 0; s < nsets; s++) items.push_back(grover_item(prob, s, s));
  double2 *amp = nullptr;
  if (d_state) {
    REQUIRE(prob->table != nullptr, "state output needs a tabulated problem");
    amp = (double2 *)prob->ctx->gamps.get(items[0].nclass * sizeof(double2));
    items[0].amp_out = amp;
  }
  std::vector<double> hout((size_t)nsets * (1 + 2 * p));
  run_grover(items, angles, nsets, p, grad, hout.data(), prob->ctx, st);
  for (int s = 0; s < nsets; s++) {
    const double *r = hout.data() + (size_t)s * (1 + 2 * p);
    if (out_expect) out_expect[s] = r[0];
    if (grad && out_grad) std::memcpy(out_grad + (size_t)s * 2 * p, r + 1, 2 * p * sizeof(double));
  }
  if (d_state) {
    HIPCHK(launch_grover_expand(prob->table, prob->tbytes, prob->N, amp, d_state, precision, st));
    HIPCHK(hipStreamSynchronize(st));
  }
}

// The tuner. Candidate plans differ in one option at a time (coordinate descent from the fixed
// rule over the options that change this shape's plan: checkpointed or in-place reverse sweep,
// narrow-run cover, which tile takes the narrowest runs, the register-group rules, the tile
// order of the first round, the XCD-aware workgroup order). Each candidate runs the caller's
// evaluation shape on its first min(p, 4) layers (enough rounds for the round-boundary passes
// of both tile orders to appear) on the caller's stream, timed by its kernels' durations; a
// change is kept when it is at least 2 % faster (smaller differences measured on a few layers
// did not carry over to full-depth evaluations).
template <typename R>
PlanOpts plan_for(qaoa_problem *prob, int p, const double *angles, int nsets, int grad, const qaoa_mixer *xm,
                  hipStream_t st, bool may_tune) {
  qaoa_ctx *ctx = prob->ctx;
  const int prec = sizeof(R) == 4 ? QAOA_FP32 : QAOA_FP64;
  const int T = prec == QAOA_FP32 ? TILE_BITS_F32 : TILE_BITS_F64;
  const int cmin = prec == QAOA_FP32 ? MIN_CONTIG_F32 : MIN_CONTIG_F64;
  const int cnarrow = prec == QAOA_FP32 ? MIN_CONTIG_NARROW_F32 : MIN_CONTIG_NARROW_F64;
  const int n = prob->n;
  const PlanOpts def;
  const int L = xm ? 2 * p : p;
  const int K = (int)make_tiles(n, T, cmin, cnarrow, def).size();
  const size_t vbytes = (size_t)nsets * ((size_t)1 << n) * 2 * sizeof(R);
  const bool fits = grad && ctx->checkpoint_mode != 0 && ckpt_fits(ctx, (size_t)(1 + L * (K - 1)) * vbytes, vbytes);
  const int mixcode = xm ? 1 + 16 * xm->kind + xm->xd.mode : 0;
  const std::array<int, 5> key = {n, prec, grad ? 1 : 0, mixcode, fits ? 1 : 0};
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) return it->second;
  if (!ctx->autotune || !may_tune) return def;

  const bool ma = xm && xm->kind == 4;
  const int pt = std::min(p, 4);
  const int SL = ma ? p * (n + 1) : 2 * p, SLt = ma ? pt * (n + 1) : 2 * pt;
  const int nb = ma ? n : 1;  // beta angles per layer
  std::vector<double> at((size_t)nsets * SLt);
  for (int s = 0; s < nsets; s++) {
    const double *src = angles + (size_t)s * SL;
    double *dst = at.data() + (size_t)s * SLt;
    std::memcpy(dst, src, sizeof(double) * pt * nb);
    std::memcpy(dst + pt * nb, src + p * nb, sizeof(double) * pt);
  }
  std::vector<double> e(nsets), g(grad ? (size_t)nsets * SLt : 0);
  auto run = [&](const PlanOpts &o) {
    run_x_path<R>(prob, pt, at.data(), nsets, nullptr, grad, e.data(), grad ? g.data() : nullptr, nullptr, st, xm,
                  nullptr, &o);
  };
  // A trial's cost is the summed duration of its kernels (events around each launch), the
  // best of three runs after one to settle allocations: host planning, which a replayed graph
  // or a pipelined batched call hides, does not enter it. The caller's kernel totals and any
  // event pairs it has not folded yet are set aside while the trials run.
  struct ProfSave {
    qaoa_ctx *c;
    bool was;
    KTotals tot[QAOA_KC_COUNT];
    decltype(qaoa_ctx::pending) pend;
    ~ProfSave() {
      c->profiling = was;
      std::copy(tot, tot + QAOA_KC_COUNT, c->totals);
      c->pending = std::move(pend);
    }
  } prof_save{ctx, ctx->profiling, {}, std::move(ctx->pending)};
  std::copy(ctx->totals, ctx->totals + QAOA_KC_COUNT, prof_save.tot);
  ctx->pending.clear();
  ctx->profiling = false;
  auto timed = [&](const PlanOpts &o) {
    run(o);
    double best = 1e300;
    for (int r = 0; r < 3; r++) {
      for (auto &t : ctx->totals) t = KTotals{};
      ctx->profiling = true;
      run(o);  // synchronises the stream before it returns its results
      profile_collect(ctx);
      ctx->profiling = false;
      double ms = 0;
      for (const auto &t : ctx->totals) ms += t.ms;
      best = std::min(best, ms);
    }
    return best;
  };
  PlanOpts best = def;
  if (!fits) best.ckpt = 0;
  double tbest = timed(best);
  auto consider = [&](PlanOpts o) {
    const double t = timed(o);
    if (t < 0.98 * tbest) {
      best = o;
      tbest = t;
    }
  };
  if (fits) {
    PlanOpts o = best;
    o.ckpt = 0;
    consider(o);
  }
  for (int which = 0; which < 4; which++)
    if (plan_knob_applies(which, n, T, cmin, cnarrow, best)) {
      PlanOpts o = best;
      if (which == 0) o.narrow ^= 1;
      if (which == 1) o.narrow_top ^= 1;
      if (which == 2) o.lowbits ^= 1;
      if (which == 3) o.swap ^= 1;
      consider(o);
    }
  if (K >= 2) {
    PlanOpts o = best;
    o.down ^= 1;
    consider(o);
  }
  if (n - T >= 3) {
    PlanOpts o = best;
    o.xcd ^= 1;
    consider(o);
  }
  if (!xm && swz_applies(n, T, cmin, cnarrow, prec, best)) {
    PlanOpts o = best;
    o.swz ^= 1;
    consider(o);
  }
  ctx->plans[key] = best;
  return best;
}

void evaluate_x(qaoa_problem *prob, int p, const double *angles, int nsets, const void *d_psi0,
                int precision, int grad, double *out_expect, double *out_grad, void *d_state,
                hipStream_t st) {
  if (small_path(prob, precision) && !d_psi0 && !d_state) {
    if (prob->max_value + 1 > MAX_LUT) throw fail(QAOA_ERR_UNSUPPORTED, "largest cost value exceeds the LUT limit");
    std::vector<SmallItem> items;
    for (int s = 0; s < nsets; s++) items.push_back(small_item(prob, s, s));
    std::vector<double> hout((size_t)nsets * (1 + 2 * p));
    run_small(items, precision, angles, nsets, p, grad, hout.data(), prob->ctx, st);
    for (int s = 0; s < nsets; s++) {
      const double *r = hout.data() + (size_t)s * (1 + 2 * p);
      if (out_expect) out_expect[s] = r[0];
      if (grad && out_grad) std::memcpy(out_grad + (size_t)s * 2 * p, r + 1, 2 * p * sizeof(double));
    }
    return;
  }
  const int T = precision == QAOA_FP32 ? TILE_BITS_F32 : TILE_BITS_F64;
  if (prob->n <= T)
    throw fail(QAOA_ERR_UNSUPPORTED, "initial state or state output needs n > tile size (use n >= 14)");
  if (precision == QAOA_FP32)
    run_x_path<float>(prob, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
  else
    run_x_path<double>(prob, p, angles, nsets, d_psi0, grad, out_expect, out_grad, d_state, st);
}

}  // namespace

// ---------------------------------------------------------------- C ABI

// ---------------------------------------------------------------- allocation-free scratch

// Device memory of qaoa_expect_grad_pairs_noalloc: the whole-state items, the angle sets and
// the result rows of one call. A file-scope device array, so each GPU the library runs on holds
// its own copy from load to process end and no call allocates it. In host code the name is a
// host-side stand-in, never a device address: host code uses only the address that
// hipGetSymbolAddress returns for the current device (kept per device in g_scratch_dev).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static unsigned char *g_scratch_dev[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;
// Host staging of the items of one call (static, no heap): calls that overlap race on it as
// they race on the device array.
static SmallItem g_noalloc_items[NOALLOC_SCRATCH_BYTES / sizeof(SmallItem)];

// Address of this device's scratch array; `dev` must be the current device.
static unsigned char *scratch_address(int dev) {
  REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = (unsigned char *)ptr;
  }
  return g_scratch_dev[dev];
}

extern "C" {

const char *qaoa_status_string(int status) {
  switch (status) {
    case QAOA_OK: return "ok";
    case QAOA_ERR_INVALID_ARG: return "invalid argument";
    case QAOA_ERR_OUT_OF_MEMORY: return "out of memory";
    case QAOA_ERR_HIP: return "HIP runtime error";
    case QAOA_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char *qaoa_last_error(void) { return g_last_error.c_str(); }

int qaoa_ctx_create(int hip_device, qaoa_ctx **out) {
  return guarded([&] {
    REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    REQUIRE(hip_device >= 0 && hip_device < count, "no such HIP device");
    DeviceGuard g(hip_device);
    auto c = std::make_unique<qaoa_ctx>();
    c->device = hip_device;
    // QAOA_GRAD_CHECKPOINT: "0" never keep forward checkpoints, "1" always, unset: when the
    // free device memory allows
    if (const char *e = std::getenv("QAOA_GRAD_CHECKPOINT")) c->checkpoint_mode = std::atoi(e) ? 1 : 0;
    if (const char *e = std::getenv("QAOA_XPROD_TILES")) c->xprod_tiles = std::atoi(e) ? 1 : 0;
    if (const char *e = std::getenv("QAOA_BATCH_GRAPH")) c->batch_graphs = std::atoi(e) ? 1 : 0;
    if (const char *e = std::getenv("QAOA_AUTOTUNE")) c->autotune = std::atoi(e) ? 1 : 0;
    c->scratch = scratch_address(hip_device);
    *out = c.release();
  });
}

int qaoa_ctx_set_autotune(qaoa_ctx *ctx, int enable) {
  return guarded([&] {
    REQUIRE(ctx != nullptr, "ctx is NULL");
    ctx->autotune = enable != 0;
  });
}

static std::string plans_text(const qaoa_ctx *ctx) {
  std::string out = "qaoa-plans 3\n";
  char line[160];
  for (const auto &kv : ctx->plans) {
    const auto &k = kv.first;
    const PlanOpts &o = kv.second;
    std::snprintf(line, sizeof(line), "%d %d %d %d %d : %d %d %d %d %d %d %d %d\n", k[0], k[1], k[2], k[3], k[4],
                  o.narrow, o.narrow_top, o.lowbits, o.down, o.xcd, o.ckpt, o.swap, o.swz);
    out += line;
  }
  return out;
}

int qaoa_plans_text(const qaoa_ctx *ctx, char *buf, size_t len, size_t *needed) {
  return guarded([&] {
    REQUIRE(ctx != nullptr, "ctx is NULL");
    const std::string t = plans_text(ctx);
    if (needed) *needed = t.size() + 1;
    if (buf && len > 0) {
      const size_t m = std::min(len - 1, t.size());
      std::memcpy(buf, t.data(), m);
      buf[m] = 0;
    }
  });
}

int qaoa_plans_save(const qaoa_ctx *ctx, const char *path) {
  return guarded([&] {
    REQUIRE(ctx != nullptr && path != nullptr, "ctx or path is NULL");
    const std::string t = plans_text(ctx), tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    REQUIRE(f != nullptr, "cannot open the plan file for writing");
    const bool ok = std::fwrite(t.data(), 1, t.size(), f) == t.size();
    const bool closed = std::fclose(f) == 0;
    REQUIRE(ok && closed, "writing the plan file failed");
    REQUIRE(std::rename(tmp.c_str(), path) == 0, "renaming the plan file failed");
  });
}

int qaoa_plans_load(qaoa_ctx *ctx, const char *path) {
  return guarded([&] {
    REQUIRE(ctx != nullptr && path != nullptr, "ctx or path is NULL");
    FILE *f = std::fopen(path, "r");
    REQUIRE(f != nullptr, "cannot open the plan file");
    std::map<std::array<int, 5>, PlanOpts> got;
    char line[256];
    bool header = false, bad = false;
    int version = 0;
    while (std::fgets(line, sizeof(line), f)) {
      if (!header) {
        // version 1 files (written before the swap option) load with swap = 0, versions 1 and
        // 2 (before the layout option) with swz = 1
        if (std::strncmp(line, "qaoa-plans 1", 12) == 0) version = 1;
        if (std::strncmp(line, "qaoa-plans 2", 12) == 0) version = 2;
        if (std::strncmp(line, "qaoa-plans 3", 12) == 0) version = 3;
        header = version != 0;
        if (!header) bad = true;
        if (bad) break;
        continue;
      }
      std::array<int, 5> k{};
      int v[8] = {0, 0, 0, 0, 0, 0, 0, 1};
      const int want = version == 1 ? 11 : (version == 2 ? 12 : 13);
      if (std::sscanf(line, "%d %d %d %d %d : %d %d %d %d %d %d %d %d", &k[0], &k[1], &k[2], &k[3], &k[4], &v[0],
                      &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7]) != want) {
        bad = true;
        break;
      }
      bool ok = k[0] >= 1 && k[0] <= 33 && (k[1] == 0 || k[1] == 1) && (k[2] == 0 || k[2] == 1) &&
                (k[4] == 0 || k[4] == 1) && v[5] >= -1 && v[5] <= 1 && (v[6] == 0 || v[6] == 1) &&
                (v[7] == 0 || v[7] == 1);
      for (int i = 0; i < 5; i++) ok = ok && (v[i] == 0 || v[i] == 1);
      if (!ok) {
        bad = true;
        break;
      }
      PlanOpts o;
      o.narrow = (uint8_t)v[0];
      o.narrow_top = (uint8_t)v[1];
      o.lowbits = (uint8_t)v[2];
      o.down = (uint8_t)v[3];
      o.xcd = (uint8_t)v[4];
      o.ckpt = (int8_t)v[5];
      o.swap = (uint8_t)v[6];
      o.swz = (uint8_t)v[7];
      got[k] = o;
    }
    std::fclose(f);
    REQUIRE(header && !bad, "malformed plan file");
    for (const auto &kv : got) ctx->plans[kv.first] = kv.second;
  });
}

int qaoa_profile_enable(qaoa_ctx *ctx, int enable) {
  return guarded([&] {
    REQUIRE(ctx != nullptr, "ctx is NULL");
    ctx->profiling = enable != 0;
    for (auto &t : ctx->totals) t = KTotals{};
  });
}

int qaoa_profile_read(const qaoa_ctx *ctx, int kernel_class, int64_t *launches, double *ms,
                      double *bytes, double *flops) {
  return guarded([&] {
    REQUIRE(ctx != nullptr, "ctx is NULL");
    REQUIRE(kernel_class >= 0 && kernel_class < QAOA_KC_COUNT, "no such kernel class");
    const KTotals &t = ctx->totals[kernel_class];
    if (launches) *launches = t.launches;
    if (ms) *ms = t.ms;
    if (bytes) *bytes = t.bytes;
    if (flops) *flops = t.flops;
  });
}

int qaoa_stream_copy(qaoa_ctx *ctx, const void *d_src, void *d_dst, size_t bytes, void *stream) {
  return guarded([&] {
    REQUIRE(ctx != nullptr, "ctx is NULL");
    REQUIRE(d_src && d_dst, "source or destination is NULL");
    REQUIRE(bytes % 16 == 0, "bytes must be a multiple of 16");
    REQUIRE(((uintptr_t)d_src | (uintptr_t)d_dst) % 16 == 0, "buffers must be 16-byte aligned");
    DeviceGuard g(ctx->device);
    HIPCHK(launch_stream_copy(d_src, d_dst, bytes, (hipStream_t)stream));
  });
}

int qaoa_ctx_destroy(qaoa_ctx *ctx) {
  return guarded([&] {
    if (!ctx) return;
    REQUIRE(ctx->live == 0, "problems or mixers created on this context are still alive");
    DeviceGuard g(ctx->device);
    delete ctx;
  });
}

int qaoa_cost_table(qaoa_ctx *ctx, int n, int n_edges, const int32_t *u, const int32_t *v,
                    const int32_t *w, int hamming_k, qaoa_problem **out, void *stream) {
  return guarded([&] {
    REQUIRE(ctx && out, "ctx or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 32, "n must be in [1, 32]");
    REQUIRE(n_edges >= 0 && n_edges <= 512, "n_edges must be in [0, 512]");
    REQUIRE(n_edges == 0 || (u && v), "edge arrays are NULL");
    REQUIRE(hamming_k <= n, "hamming_k must be <= n");
    int64_t W = 0;
    for (int e = 0; e < n_edges; e++) {
      REQUIRE(u[e] >= 0 && u[e] < n && v[e] >= 0 && v[e] < n, "edge endpoint out of range");
      REQUIRE(u[e] != v[e], "self-loop edge");
      int64_t we = w ? w[e] : 1;
      REQUIRE(we >= 0, "negative edge weight");
      W += we;
    }
    REQUIRE(W <= 65535, "total edge weight must be <= 65535");
    uint64_t N = hamming_k < 0 ? (1ull << n) : (uint64_t)binom64(n, hamming_k);
    if (hamming_k >= 0) REQUIRE(N <= (1ull << 26), "feasible subspace larger than 2^26 states");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    auto prob = std::make_unique<qaoa_problem>();
    prob->ctx = ctx;
    prob->n = n;
    prob->k = hamming_k < 0 ? -1 : hamming_k;
    prob->N = N;
    prob->tbytes = W <= 255 ? 1 : 2;
    prob->total_weight = W;
    if (hamming_k < 0) prob->mean = 0.5 * (double)W;
    else if (n >= 2 && N > 0)
      prob->mean = (double)W * 2.0 * (double)binom64(n - 2, hamming_k - 1) / (double)N;
    // edges to the device
    DevBuf de;
    int32_t *dd = nullptr;
    if (n_edges > 0) {
      dd = (int32_t *)de.get(3 * n_edges * sizeof(int32_t));
      std::vector<int32_t> hv(3 * n_edges);
      for (int e = 0; e < n_edges; e++) {
        hv[e] = u[e];
        hv[n_edges + e] = v[e];
        hv[2 * n_edges + e] = w ? w[e] : 1;
      }
      HIPCHK(hipMemcpyAsync(dd, hv.data(), hv.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    if (hipMalloc(&prob->table, N * prob->tbytes) != hipSuccess) {
      (void)hipGetLastError();
      prob->table = nullptr;
      throw fail(QAOA_ERR_OUT_OF_MEMORY, "table allocation failed");
    }
    const int32_t *du = dd, *dv = dd ? dd + n_edges : nullptr, *dw = dd ? dd + 2 * n_edges : nullptr;
    if (hamming_k < 0) {
      HIPCHK(launch_cost_table_full(n, n_edges, du, dv, dw, prob->table, prob->tbytes, st));
    } else {
      std::vector<int64_t> hb(33 * 33);
      for (int a = 0; a <= 32; a++)
        for (int b = 0; b <= 32; b++) hb[a * 33 + b] = binom64(a, b);
      DevBuf db;
      int64_t *dbin = (int64_t *)db.get(hb.size() * sizeof(int64_t));
      HIPCHK(hipMemcpyAsync(dbin, hb.data(), hb.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
      HIPCHK(launch_cost_table_hw(n, hamming_k, n_edges, du, dv, dw, dbin, N, prob->table,
                                  prob->tbytes, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    DevBuf dm;
    unsigned *dmax = (unsigned *)dm.get(sizeof(unsigned));
    HIPCHK(hipMemsetAsync(dmax, 0, sizeof(unsigned), st));
    HIPCHK(launch_table_max(prob->table, prob->tbytes, N, dmax, st));
    unsigned hmax = 0;
    HIPCHK(hipMemcpyAsync(&hmax, dmax, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    prob->max_value = hmax;
    // a graph table stores the cost itself: index c has value c; C(~x) = C(x) always
    prob->hvals.resize((size_t)hmax + 1);
    for (unsigned c = 0; c <= hmax; c++) prob->hvals[c] = (double)c;
    upload_values(prob.get(), st);
    *out = prob.release();
    ctx->live++;
  });
}

int qaoa_problem_from_values(qaoa_ctx *ctx, int n, int hamming_k, const double *host_values, size_t len,
                             qaoa_problem **out, void *stream) {
  return guarded([&] {
    REQUIRE(ctx && out && host_values, "ctx, values or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 32, "n must be in [1, 32]");
    REQUIRE(hamming_k <= n, "hamming_k must be <= n");
    const uint64_t N = hamming_k < 0 ? (1ull << n) : (uint64_t)binom64(n, hamming_k);
    if (hamming_k >= 0) REQUIRE(N <= (1ull << 26), "feasible subspace larger than 2^26 states");
    REQUIRE(len == N, "len differs from the feasible-set size");
    for (size_t i = 0; i < len; i++) REQUIRE(std::isfinite(host_values[i]), "values must be finite");
    // distinct values in increasing order, and each state's index among them: an
    // open-addressing hash on the value's bits (-0 folded into +0), 4 slots per allowed value
    constexpr int HB = 12;
    constexpr size_t HS = size_t(1) << HB;
    static_assert(HS >= 4 * (size_t)MAX_LUT, "hash table too small");
    std::vector<uint64_t> hkey(HS);
    std::vector<int> hidx(HS, -1);
    auto bits_of = [](double v) {
      if (v == 0.0) v = 0.0;
      uint64_t b;
      std::memcpy(&b, &v, sizeof(b));
      return b;
    };
    auto slot_of = [&](uint64_t b) {
      size_t h = (size_t)((b * 0x9E3779B97F4A7C15ull) >> (64 - HB));
      while (hidx[h] >= 0 && hkey[h] != b) h = (h + 1) & (HS - 1);
      return h;
    };
    std::vector<double> distinct;
    for (size_t i = 0; i < len; i++) {
      const uint64_t b = bits_of(host_values[i]);
      const size_t h = slot_of(b);
      if (hidx[h] < 0) {
        if (distinct.size() == (size_t)MAX_LUT) throw fail(QAOA_ERR_UNSUPPORTED, "more than 1024 distinct cost values");
        hkey[h] = b;
        hidx[h] = (int)distinct.size();
        distinct.push_back(host_values[i] == 0.0 ? 0.0 : host_values[i]);
      }
    }
    std::vector<double> sorted = distinct;
    std::sort(sorted.begin(), sorted.end());
    std::vector<int> rank(distinct.size());
    for (size_t j = 0; j < distinct.size(); j++)
      rank[j] = (int)(std::lower_bound(sorted.begin(), sorted.end(), distinct[j]) - sorted.begin());
    auto prob = std::make_unique<qaoa_problem>();
    prob->ctx = ctx;
    prob->n = n;
    prob->k = hamming_k < 0 ? -1 : hamming_k;
    prob->N = N;
    prob->tbytes = sorted.size() <= 256 ? 1 : 2;
    prob->max_value = (int64_t)sorted.size() - 1;
    prob->hvals = sorted;
    std::vector<unsigned char> h1;
    std::vector<uint16_t> h2;
    if (prob->tbytes == 1) h1.resize(N);
    else h2.resize(N);
    long double sum = 0.0L;
    for (size_t i = 0; i < len; i++) {
      const int idx = rank[hidx[slot_of(bits_of(host_values[i]))]];
      if (prob->tbytes == 1) h1[i] = (unsigned char)idx;
      else h2[i] = (uint16_t)idx;
      sum += (long double)host_values[i];
    }
    prob->mean = (double)(sum / (long double)N);
    if (hamming_k < 0)
      for (size_t i = 0; i < len / 2 && prob->sym; i++)
        if (host_values[i] != host_values[N - 1 - i]) prob->sym = false;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if (hipMalloc(&prob->table, N * prob->tbytes) != hipSuccess) {
      (void)hipGetLastError();
      prob->table = nullptr;
      throw fail(QAOA_ERR_OUT_OF_MEMORY, "table allocation failed");
    }
    HIPCHK(hipMemcpyAsync(prob->table, prob->tbytes == 1 ? (const void *)h1.data() : (const void *)h2.data(),
                          N * prob->tbytes, hipMemcpyHostToDevice, st));
    upload_values(prob.get(), st);
    *out = prob.release();
    ctx->live++;
  });
}

int qaoa_problem_copy_values(const qaoa_problem *prob, double *host_dst, size_t len, void *stream) {
  return guarded([&] {
    REQUIRE(prob && host_dst, "problem or destination is NULL");
    REQUIRE(len == prob->N, "len differs from the feasible-set size");
    if (!prob->table) throw fail(QAOA_ERR_UNSUPPORTED, "the problem holds degeneracies only (no table)");
    DeviceGuard g(prob->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    DevBuf tmp;
    double *d = (double *)tmp.get(prob->N * sizeof(double));
    HIPCHK(launch_table_values(prob->table, prob->tbytes, prob->dvals, d, prob->N, st));
    HIPCHK(hipMemcpyAsync(host_dst, d, prob->N * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  });
}

int qaoa_problem_copy_table(const qaoa_problem *prob, int64_t *host_dst, size_t len, void *stream) {
  return guarded([&] {
    REQUIRE(prob && host_dst, "problem or destination is NULL");
    REQUIRE(len == prob->N, "len differs from the feasible-set size");
    if (!prob->table) throw fail(QAOA_ERR_UNSUPPORTED, "the problem holds degeneracies only (no table)");
    DeviceGuard g(prob->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    DevBuf tmp;
    int64_t *d = (int64_t *)tmp.get(prob->N * sizeof(int64_t));
    HIPCHK(launch_table_widen(prob->table, prob->tbytes, d, prob->N, st));
    HIPCHK(hipMemcpyAsync(host_dst, d, prob->N * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  });
}

int qaoa_problem_info(const qaoa_problem *prob, int *n, int *hamming_k, int64_t *size,
                      int64_t *max_value) {
  return guarded([&] {
    REQUIRE(prob != nullptr, "problem is NULL");
    if (n) *n = prob->n;
    if (hamming_k) *hamming_k = prob->k;
    if (size) *size = (int64_t)prob->N;
    if (max_value) *max_value = prob->max_value;
  });
}

int qaoa_problem_destroy(qaoa_problem *prob) {
  return guarded([&] {
    if (!prob) return;
    DeviceGuard g(prob->ctx->device);
    prob->ctx->live--;
    delete prob;
  });
}

int qaoa_mixer_x(qaoa_ctx *ctx, int n, qaoa_mixer **out) {
  return guarded([&] {
    REQUIRE(ctx && out, "ctx or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 32, "n must be in [1, 32]");
    auto m = std::make_unique<qaoa_mixer>();
    m->ctx = ctx;
    m->kind = 0;
    m->n = n;
    *out = m.release();
    ctx->live++;
  });
}

int qaoa_mixer_grover(qaoa_ctx *ctx, int n, int hamming_k, qaoa_mixer **out) {
  return guarded([&] {
    REQUIRE(ctx && out, "ctx or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 62, "n must be in [1, 62]");
    REQUIRE(hamming_k <= n, "hamming_k must be <= n");
    auto m = std::make_unique<qaoa_mixer>();
    m->ctx = ctx;
    m->kind = 2;
    m->n = n;
    m->k = hamming_k < 0 ? -1 : hamming_k;
    *out = m.release();
    ctx->live++;
  });
}

int qaoa_cost_degeneracies(qaoa_ctx *ctx, int n, int n_edges, const int32_t *u, const int32_t *v, const int32_t *w,
                           int hamming_k, qaoa_problem **out, void *stream) {
  return guarded([&] {
    REQUIRE(ctx && out, "ctx or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 40, "n must be in [1, 40]");
    REQUIRE(n_edges >= 0 && n_edges <= 512, "n_edges must be in [0, 512]");
    REQUIRE(n_edges == 0 || (u && v), "edge arrays are NULL");
    REQUIRE(hamming_k <= n, "hamming_k must be <= n");
    int64_t W = 0;
    for (int e = 0; e < n_edges; e++) {
      REQUIRE(u[e] >= 0 && u[e] < n && v[e] >= 0 && v[e] < n, "edge endpoint out of range");
      REQUIRE(u[e] != v[e], "self-loop edge");
      int64_t we = w ? w[e] : 1;
      REQUIRE(we >= 0, "negative edge weight");
      W += we;
    }
    REQUIRE(W <= 16383, "total edge weight must be <= 16383");
    if (hamming_k >= 0) REQUIRE(n <= 32, "n must be <= 32 for a Hamming-weight subspace");
    const uint64_t N = hamming_k < 0 ? (1ull << n) : (uint64_t)binom64(n, hamming_k);
    const int nbins = (int)W + 1;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    // edges and adjacency (CSR: neighbour << 16 | weight) to the device
    std::vector<int32_t> hv(3 * (size_t)n_edges), off(n + 1, 0), adj(2 * (size_t)n_edges);
    for (int e = 0; e < n_edges; e++) {
      hv[e] = u[e];
      hv[n_edges + e] = v[e];
      hv[2 * n_edges + e] = w ? w[e] : 1;
      off[u[e] + 1]++;
      off[v[e] + 1]++;
    }
    for (int i = 0; i < n; i++) off[i + 1] += off[i];
    {
      std::vector<int32_t> fill(off.begin(), off.end() - 1);
      for (int e = 0; e < n_edges; e++) {
        const int32_t we = w ? w[e] : 1;
        adj[fill[u[e]]++] = (v[e] << 16) | we;
        adj[fill[v[e]]++] = (u[e] << 16) | we;
      }
    }
    std::vector<int64_t> hb(33 * 33);
    for (int a = 0; a <= 32; a++)
      for (int b = 0; b <= 32; b++) hb[a * 33 + b] = binom64(a, b);
    const size_t bytes_e = std::max<size_t>(1, hv.size()) * 4, bytes_o = off.size() * 4,
                 bytes_a = std::max<size_t>(1, adj.size()) * 4, bytes_b = hb.size() * 8;
    DevBuf de, dof, dad, dbn, dcnt;
    int32_t *d_e = (int32_t *)de.get(bytes_e);
    int32_t *d_off = (int32_t *)dof.get(bytes_o);
    int32_t *d_adj = (int32_t *)dad.get(bytes_a);
    int64_t *d_bin = (int64_t *)dbn.get(bytes_b);
    unsigned long long *d_cnt = (unsigned long long *)dcnt.get((size_t)nbins * 8);
    if (!hv.empty()) HIPCHK(hipMemcpyAsync(d_e, hv.data(), hv.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_off, off.data(), bytes_o, hipMemcpyHostToDevice, st));
    if (!adj.empty()) HIPCHK(hipMemcpyAsync(d_adj, adj.data(), adj.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_bin, hb.data(), bytes_b, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(d_cnt, 0, (size_t)nbins * 8, st));
    const int32_t *eu = d_e, *ev = d_e + n_edges, *ew = d_e + 2 * n_edges;
    // neighbour masks per (vertex, distinct edge weight), when there are at most 8 weights
    std::vector<int32_t> wv;
    for (int e = 0; e < n_edges; e++) {
      const int32_t we = w ? w[e] : 1;
      if (std::find(wv.begin(), wv.end(), we) == wv.end()) wv.push_back(we);
    }
    const int nw0 = (int)wv.size();
    const bool use_masks = nw0 >= 1 && nw0 <= 8;
    const int nw = nw0 <= 1 ? 1 : (nw0 <= 2 ? 2 : (nw0 <= 4 ? 4 : 8));  // padded class count
    while ((int)wv.size() < nw) wv.push_back(0);
    DevBuf dmask, dmdeg, dwv;
    uint64_t *d_mask = nullptr;
    int32_t *d_mdeg = nullptr, *d_wv = nullptr;
    if (use_masks) {
      std::vector<uint64_t> hm((size_t)n * nw, 0);
      std::vector<int32_t> hd((size_t)n * nw, 0);
      for (int e = 0; e < n_edges; e++) {
        const int32_t we = w ? w[e] : 1;
        const int j = (int)(std::find(wv.begin(), wv.end(), we) - wv.begin());
        hm[(size_t)u[e] * nw + j] |= 1ull << v[e];
        hm[(size_t)v[e] * nw + j] |= 1ull << u[e];
        hd[(size_t)u[e] * nw + j]++;
        hd[(size_t)v[e] * nw + j]++;
      }
      d_mask = (uint64_t *)dmask.get(hm.size() * 8);
      d_mdeg = (int32_t *)dmdeg.get(hd.size() * 4);
      d_wv = (int32_t *)dwv.get(wv.size() * 4);
      HIPCHK(hipMemcpyAsync(d_mask, hm.data(), hm.size() * 8, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(d_mdeg, hd.data(), hd.size() * 4, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(d_wv, wv.data(), wv.size() * 4, hipMemcpyHostToDevice, st));
    }
    // the count, in launches of at most 2^18 threads
    const uint64_t LAUNCH = 1ull << 18;
    KTimer kt(ctx, st, QAOA_KC_COUNT_STATES, 0.0, (double)N);  // "flops": states counted
    if (hamming_k < 0) {
      const int lo = std::max(0, std::min(24, n - 20));
      const uint64_t T = 1ull << (n - lo);
      // a private histogram column per thread while it fits in LDS (160 bins: one workgroup
      // per CU above 80): contention-free atomics beat a shared histogram by 5-10x
      const bool priv = nbins <= 160;
      for (uint64_t b0 = 0; b0 < T; b0 += LAUNCH)
        HIPCHK(launch_enum_full(n, n_edges, eu, ev, ew, d_off, d_adj, d_mask, d_mdeg, d_wv, nw, lo, b0,
                                std::min(LAUNCH, T - b0), nbins, priv, d_cnt, st));
    } else {
      const uint64_t T = std::min<uint64_t>(N, 1ull << 20);
      const uint64_t per = (N + T - 1) / T;
      for (uint64_t t0 = 0; t0 < T; t0 += LAUNCH) {
        const uint64_t nt = std::min(LAUNCH, T - t0);
        HIPCHK(launch_enum_hw(n, hamming_k, n_edges, eu, ev, ew, d_bin, t0 * per, per, N, nt, nbins, d_cnt, st));
      }
    }
    kt.done();
    std::vector<unsigned long long> hc(nbins);
    HIPCHK(hipMemcpyAsync(hc.data(), d_cnt, (size_t)nbins * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    profile_collect(ctx);
    auto prob = std::make_unique<qaoa_problem>();
    prob->ctx = ctx;
    prob->n = n;
    prob->k = hamming_k < 0 ? -1 : hamming_k;
    prob->N = N;
    prob->total_weight = W;
    long double sum = 0.0L;
    unsigned long long seen = 0;
    for (int c = 0; c < nbins; c++)
      if (hc[c]) {
        prob->hvals.push_back((double)c);
        prob->hcounts.push_back((double)hc[c]);
        sum += (long double)c * (long double)hc[c];
        seen += hc[c];
      }
    if (seen != N) throw fail(QAOA_ERR_HIP, "internal: degeneracies do not add up to the state count");
    if (prob->hvals.size() > (size_t)GROVER_MAX_CLASSES)
      throw fail(QAOA_ERR_UNSUPPORTED, "more than 2048 distinct cost values");
    prob->mean = (double)(sum / (long double)N);
    prob->max_value = (int64_t)prob->hvals.size() - 1;
    upload_values(prob.get(), st);
    if (hipMalloc(&prob->dcounts, prob->hcounts.size() * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      prob->dcounts = nullptr;
      throw fail(QAOA_ERR_OUT_OF_MEMORY, "degeneracy allocation failed");
    }
    HIPCHK(hipMemcpyAsync(prob->dcounts, prob->hcounts.data(), prob->hcounts.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    *out = prob.release();
    ctx->live++;
  });
}

int qaoa_problem_degeneracies(const qaoa_problem *cprob, double *values, int64_t *counts, size_t cap, size_t *count,
                              void *stream) {
  return guarded([&] {
    REQUIRE(cprob != nullptr, "problem is NULL");
    qaoa_problem *prob = const_cast<qaoa_problem *>(cprob);
    DeviceGuard g(prob->ctx->device);
    ensure_counts(prob, (hipStream_t)stream);
    // classes with at least one state, in increasing value order
    size_t j = 0;
    for (size_t i = 0; i < prob->hcounts.size(); i++) {
      if (prob->hcounts[i] == 0.0) continue;
      if (j < cap) {
        if (values) values[j] = prob->hvals[i];
        if (counts) counts[j] = (int64_t)prob->hcounts[i];
      }
      j++;
    }
    if (count) *count = j;
    REQUIRE(j <= cap || (!values && !counts), "cap is smaller than the number of distinct values");
  });
}

static void eigen_mixer(qaoa_ctx *ctx, int kind, int n, int k, const double *host_matrix, qaoa_mixer **out,
                        void *stream, const double *host_eigenvalues = nullptr) {
  DeviceGuard g(ctx->device);
  auto m = std::make_unique<qaoa_mixer>();
  m->ctx = ctx;
  m->kind = 1;
  m->n = n;
  m->k = k < 0 ? -1 : k;
  m->clique = clique_create(kind, n, m->k, host_matrix, host_eigenvalues, (hipStream_t)stream);
  *out = m.release();
  ctx->live++;
}

int qaoa_mixer_clique(qaoa_ctx *ctx, int n, int k, qaoa_mixer **out, void *stream) {
  return guarded([&] {
    REQUIRE(ctx && out, "ctx or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 2 && n <= 20, "n must be in [2, 20]");
    REQUIRE(k >= 1 && k <= n - 1, "k must be in [1, n-1]");
    REQUIRE(binom64(n, k) <= 16384, "C(n,k) must be <= 16384");
    eigen_mixer(ctx, MIX_CLIQUE, n, k, nullptr, out, stream);
  });
}

int qaoa_mixer_ring(qaoa_ctx *ctx, int n, int k, qaoa_mixer **out, void *stream) {
  return guarded([&] {
    REQUIRE(ctx && out, "ctx or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 2 && n <= 20, "n must be in [2, 20]");
    REQUIRE(k >= 1 && k <= n - 1, "k must be in [1, n-1]");
    REQUIRE(binom64(n, k) <= 16384, "C(n,k) must be <= 16384");
    eigen_mixer(ctx, MIX_RING, n, k, nullptr, out, stream);
  });
}

int qaoa_mixer_matrix(qaoa_ctx *ctx, int n, int hamming_k, const double *host_matrix, qaoa_mixer **out,
                      void *stream) {
  return guarded([&] {
    REQUIRE(ctx && out && host_matrix, "ctx, matrix or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 20, "n must be in [1, 20]");
    REQUIRE(hamming_k <= n, "hamming_k must be <= n");
    const int64_t N = hamming_k < 0 ? (int64_t(1) << n) : binom64(n, hamming_k);
    REQUIRE(N >= 1 && N <= 16384, "the feasible set must have at most 16384 states");
    double mx = 0.0;
    for (int64_t i = 0; i < N * N; i++) {
      REQUIRE(std::isfinite(host_matrix[i]), "matrix entries must be finite");
      mx = std::max(mx, std::fabs(host_matrix[i]));
    }
    for (int64_t i = 0; i < N; i++)
      for (int64_t j = 0; j < i; j++)
        REQUIRE(std::fabs(host_matrix[i * N + j] - host_matrix[j * N + i]) <= 1e-12 * mx, "matrix is not symmetric");
    eigen_mixer(ctx, MIX_MATRIX, n, hamming_k, host_matrix, out, stream);
  });
}

static void xprod_mixer(qaoa_ctx *ctx, int n, int kind, const XDiag &xd, const std::vector<double> &vals,
                        qaoa_mixer **out) {
  DeviceGuard g(ctx->device);
  auto m = std::make_unique<qaoa_mixer>();
  m->ctx = ctx;
  m->kind = kind;
  m->n = n;
  m->xd = xd;
  if (!vals.empty()) {
    m->xlen = (int)vals.size();
    if (hipMalloc(&m->xvals, vals.size() * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      m->xvals = nullptr;
      throw fail(QAOA_ERR_OUT_OF_MEMORY, "mixer value allocation failed");
    }
    HIPCHK(hipMemcpy(m->xvals, vals.data(), vals.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<float> vf(vals.begin(), vals.end());
    if (hipMalloc(&m->xvals_f, vf.size() * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      m->xvals_f = nullptr;
      throw fail(QAOA_ERR_OUT_OF_MEMORY, "mixer value allocation failed");
    }
    HIPCHK(hipMemcpy(m->xvals_f, vf.data(), vf.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  ctx->live++;
  *out = m.release();
}

int qaoa_mixer_x_orders(qaoa_ctx *ctx, int n, const int *orders, int n_orders, qaoa_mixer **out) {
  return guarded([&] {
    REQUIRE(ctx && out && orders, "ctx, orders or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 32, "n must be in [1, 32]");
    REQUIRE(n_orders >= 1 && n_orders <= n, "n_orders must be in [1, n]");
    std::vector<bool> seen(n + 1, false);
    for (int i = 0; i < n_orders; i++) {
      REQUIRE(orders[i] >= 1 && orders[i] <= n, "orders must be in [1, n]");
      REQUIRE(!seen[orders[i]], "orders must be distinct");
      seen[orders[i]] = true;
    }
    // d(w) = sum over orders k of the Krawtchouk value K_k(w) = sum_j (-1)^j C(w, j) C(n - w, k - j)
    std::vector<double> vals(n + 1);
    for (int w = 0; w <= n; w++) {
      int64_t d = 0;
      for (int i = 0; i < n_orders; i++) {
        const int k = orders[i];
        for (int j = 0; j <= k && j <= w; j++) {
          if (k - j > n - w) continue;
          const int64_t t = binom64(w, j) * binom64(n - w, k - j);
          d += (j & 1) ? -t : t;
        }
      }
      vals[w] = (double)d;
    }
    XDiag xd{};
    xd.mode = XD_POPCOUNT;
    xprod_mixer(ctx, n, 3, xd, vals, out);
  });
}

int qaoa_mixer_x_terms(qaoa_ctx *ctx, int n, const uint64_t *masks, const double *coefs, int n_terms,
                       qaoa_mixer **out) {
  return guarded([&] {
    REQUIRE(ctx && out && masks && coefs, "ctx, masks, coefs or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 32, "n must be in [1, 32]");
    REQUIRE(n_terms >= 1 && n_terms <= XD_MAX_TERMS, "n_terms must be in [1, 10]");
    XDiag xd{};
    xd.mode = XD_TERMS;
    xd.nterms = n_terms;
    for (int t = 0; t < n_terms; t++) {
      REQUIRE(masks[t] != 0 && (masks[t] >> n) == 0, "term masks must be nonzero and below 2^n");
      REQUIRE(std::isfinite(coefs[t]), "coefficients must be finite");
      xd.masks[t] = masks[t];
    }
    // index bit t is the parity of y & masks[t]; value = sum_t coefs[t] (1 - 2 bit_t)
    std::vector<double> vals((size_t)1 << n_terms);
    for (size_t idx = 0; idx < vals.size(); idx++) {
      double v = 0.0;
      for (int t = 0; t < n_terms; t++) v += ((idx >> t) & 1) ? -coefs[t] : coefs[t];
      vals[idx] = v;
    }
    xprod_mixer(ctx, n, 3, xd, vals, out);
  });
}

int qaoa_mixer_x_multiangle(qaoa_ctx *ctx, int n, qaoa_mixer **out) {
  return guarded([&] {
    REQUIRE(ctx && out, "ctx or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 32, "n must be in [1, 32]");
    XDiag xd{};
    xd.mode = XD_QUBIT;
    xprod_mixer(ctx, n, 4, xd, {}, out);
  });
}

int qaoa_mixer_info(const qaoa_mixer *mix, int *n, int *hamming_k, int *angles_per_layer) {
  return guarded([&] {
    REQUIRE(mix != nullptr, "mixer is NULL");
    if (n) *n = mix->n;
    if (hamming_k) *hamming_k = mix->k;
    if (angles_per_layer) *angles_per_layer = (int)set_len(mix, 1);
  });
}

int qaoa_mixer_from_eigen(qaoa_ctx *ctx, int n, int hamming_k, const double *host_V, const double *host_D,
                          qaoa_mixer **out, void *stream) {
  return guarded([&] {
    REQUIRE(ctx && out && host_V && host_D, "ctx, V, D or out is NULL");
    *out = nullptr;
    REQUIRE(n >= 1 && n <= 20, "n must be in [1, 20]");
    REQUIRE(hamming_k <= n, "hamming_k must be <= n");
    const int64_t N = hamming_k < 0 ? (int64_t(1) << n) : binom64(n, hamming_k);
    REQUIRE(N >= 1 && N <= 16384, "the feasible set must have at most 16384 states");
    for (int64_t j = 0; j < N; j++) {
      REQUIRE(std::isfinite(host_D[j]), "eigenvalues must be finite");
      double nn = 0.0;
      for (int64_t i = 0; i < N; i++) {
        REQUIRE(std::isfinite(host_V[j * N + i]), "eigenvectors must be finite");
        nn += host_V[j * N + i] * host_V[j * N + i];
      }
      REQUIRE(std::fabs(nn - 1.0) <= 1e-9, "eigenvectors must have unit length");
    }
    eigen_mixer(ctx, MIX_EIGEN, n, hamming_k, host_V, out, stream, host_D);
  });
}

int qaoa_mixer_eigen(const qaoa_mixer *mix, double *host_V, double *host_D, size_t N, void *stream) {
  return guarded([&] {
    REQUIRE(mix && host_V && host_D, "mixer, V or D is NULL");
    if (mix->kind != 1) throw fail(QAOA_ERR_UNSUPPORTED, "the mixer is not applied through an eigendecomposition");
    REQUIRE((int64_t)N == clique_size(*mix->clique), "N differs from the mixer's state count");
    DeviceGuard g(mix->ctx->device);
    clique_export(*mix->clique, host_V, host_D, (hipStream_t)stream);
  });
}

int qaoa_mixer_destroy(qaoa_mixer *mix) {
  return guarded([&] {
    if (!mix) return;
    DeviceGuard g(mix->ctx->device);
    mix->ctx->live--;
    delete mix;
  });
}

// X-product and per-qubit multi-angle mixers: every layer is phase, W, mixer diagonal, W (W the
// Walsh-Hadamard transform, Eq. (2)); the gradient undoes the layers on the state and the
// adjoint vector, taking each angle's sum just before its diagonal is undone.
static void evaluate_xprod(qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *angles, int nsets,
                           const void *d_psi0, int precision, int grad, double *out_expect, double *out_grad,
                           void *d_state, hipStream_t st) {
  qaoa_ctx *ctx = prob->ctx;
  REQUIRE(prob->table != nullptr, "the problem has no value table");
  const int n = prob->n;
  const uint64_t N = 1ull << n;
  const size_t esz = precision == QAOA_FP32 ? 8 : 16;
  const bool qb = mix->kind == 4;
  const int m = qb ? n : 1, slen = p * (m + 1);
  const int lut_cost = (int)prob->max_value + 1;
  if (lut_cost > MAX_LUT) throw fail(QAOA_ERR_UNSUPPORTED, "largest cost value exceeds the LUT limit");
  // Tile passes (Y-rotation basis change) for states larger than one tile: the gradient reads
  // the forward checkpoints when they fit (the rule of the transverse-field path), else undoes
  // the state in place
  if (ctx->xprod_tiles && !d_state && (mix->xd.mode == XD_POPCOUNT || mix->xd.mode == XD_TERMS || qb) &&
      n > (precision == QAOA_FP32 ? TILE_BITS_F32 : TILE_BITS_F64) && lut_cost <= MAX_LUT && mix->xlen <= MAX_LUT) {
    if (precision == QAOA_FP32)
      run_x_path<float>(prob, p, angles, nsets, d_psi0, grad, out_expect, out_grad, nullptr, st, mix);
    else
      run_x_path<double>(prob, p, angles, nsets, d_psi0, grad, out_expect, out_grad, nullptr, st, mix);
    return;
  }
  const int bsums = qb ? 33 : 1;  // sums per beta layer: total and per-bit (per-qubit angles) or one
  const int nout = 2 + p * bsums + p;
  const unsigned nblk = xdiag_blocks(N);
  void *phi = ctx->phi.get((size_t)nsets * N * esz);
  void *lam = grad ? ctx->lam.get((size_t)nsets * N * esz) : nullptr;
  double *part = (double *)ctx->partials.get((size_t)(qb ? 33 : 2) * nsets * nblk * sizeof(double));
  const size_t abytes = (size_t)nsets * slen * sizeof(double), aoff = (abytes + 255) & ~size_t(255);
  unsigned char *dp = (unsigned char *)ctx->params.get(aoff + (size_t)nsets * nout * sizeof(double));
  double *dang = (double *)dp, *dres = (double *)(dp + aoff);
  const int lut_max = std::max(std::max(lut_cost, mix->xlen), 1024);
  void *luts = ctx->luts.get((size_t)nsets * lut_max * esz);
  unsigned char *h = (unsigned char *)ctx->hparams.get(abytes);
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(h, angles, abytes);
  HIPCHK(hipMemcpyAsync(dang, h, abytes, hipMemcpyHostToDevice, st));
  XDiag cost{};
  cost.mode = XD_TABLE;
  cost.tbytes = prob->tbytes;
  cost.table = prob->table;
  const double c0 = prob->mean;
  const double vb = (double)N * esz;  // one vector read or written once
  auto timed = [&](double bytes, auto &&launch) {
    KTimer kt(ctx, st, QAOA_KC_XMIX, bytes, 0.0);
    HIPCHK(launch());
    kt.done();
  };
  auto wht = [&](int nv) {
    timed(2.0 * nv * vb * nsets * xwht_passes(n, precision),
          [&] { return launch_xwht(precision, nv, phi, lam, n, nsets, st); });
  };
  auto cost_diag = [&](int k, double sign, int nv, int gs) {
    HIPCHK(launch_xlut(precision, prob->dvals, lut_cost, dang, slen, p * m + k, sign, nsets, luts, st));
    timed((2.0 * nv * vb + (double)N * prob->tbytes) * nsets, [&] {
      return launch_xdiag(precision, nv, gs, phi, lam, N, cost, luts, lut_cost, prob->dvals, c0, part, nsets, st);
    });
  };
  auto mix_diag = [&](int k, double sign, int nv, int gs) {
    if (qb) HIPCHK(launch_xlut_q(precision, n, dang, slen, k * n, sign, nsets, luts, st));
    else HIPCHK(launch_xlut(precision, mix->xvals, mix->xlen, dang, slen, k, sign, nsets, luts, st));
    timed(2.0 * nv * vb * nsets, [&] {
      return launch_xdiag(precision, nv, gs, phi, lam, N, mix->xd, luts, mix->xlen, mix->xvals, 0.0, part, nsets, st);
    });
  };
  if (d_psi0) {
    for (int s = 0; s < nsets; s++)
      HIPCHK(hipMemcpyAsync((unsigned char *)phi + (size_t)s * N * esz, d_psi0, N * esz, hipMemcpyDeviceToDevice, st));
  } else {
    HIPCHK(launch_xfill(precision, phi, (uint64_t)nsets * N, 1.0 / std::sqrt((double)N), st));
  }
  // forward: each diagonal is applied by the first pass of the transform that follows it
  for (int k = 0; k < p; k++) {
    HIPCHK(launch_xlut(precision, prob->dvals, lut_cost, dang, slen, p * m + k, 1.0, nsets, luts, st));
    timed((2.0 * vb * xwht_passes(n, precision) + (double)N * prob->tbytes) * nsets,
          [&] { return launch_xwht_pre(precision, phi, n, nsets, cost, luts, lut_cost, st); });
    if (qb) HIPCHK(launch_xlut_q(precision, n, dang, slen, k * n, 1.0, nsets, luts, st));
    else HIPCHK(launch_xlut(precision, mix->xvals, mix->xlen, dang, slen, k, 1.0, nsets, luts, st));
    timed(2.0 * vb * xwht_passes(n, precision) * nsets,
          [&] { return launch_xwht_pre(precision, phi, n, nsets, mix->xd, luts, mix->xlen, st); });
  }
  if (d_state) HIPCHK(hipMemcpyAsync(d_state, phi, N * esz, hipMemcpyDeviceToDevice, st));
  timed(vb * nsets * (grad ? 2.0 : 1.0) + (double)N * prob->tbytes * nsets, [&] {
    return launch_xend(precision, phi, lam, N, cost, prob->dvals, lut_cost, c0, part, nsets, st);
  });
  HIPCHK(launch_xfinal(part, (int)nblk, 2, nsets, dres, nout, 0, st));
  if (grad) {
    for (int k = p - 1; k >= 0; k--) {
      wht(2);
      mix_diag(k, -1.0, 2, 1);
      HIPCHK(launch_xfinal(part, (int)nblk, bsums, nsets, dres, nout, 2 + k * bsums, st));
      wht(2);
      cost_diag(k, -1.0, 2, 1);
      HIPCHK(launch_xfinal(part, (int)nblk, 1, nsets, dres, nout, 2 + p * bsums + k, st));
    }
  }
  std::vector<double> res((size_t)nsets * nout);
  HIPCHK(hipMemcpyAsync(res.data(), dres, res.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  profile_collect(ctx);
  for (int s = 0; s < nsets; s++) {
    const double *r = res.data() + (size_t)s * nout;
    const double nr = r[1];
    if (out_expect) out_expect[s] = r[0] / nr;
    if (grad && out_grad) {
      double *g = out_grad + (size_t)s * slen;
      for (int k = 0; k < p; k++) {
        const double *b = r + 2 + k * bsums;
        if (qb)
          for (int q = 0; q < n; q++) g[k * n + q] = 2.0 * (b[0] - 2.0 * b[1 + q]) / nr;
        else
          g[k] = 2.0 * b[0] / nr;
        g[p * m + k] = 2.0 * r[2 + p * bsums + k] / nr;
      }
    }
  }
}

static void evaluate(const qaoa_problem *cprob, const qaoa_mixer *mix, int p, const double *angles,
                     int nsets, const void *d_psi0, int precision, int grad, double *out_expect,
                     double *out_grad, void *d_state, hipStream_t st) {
  qaoa_problem *prob = const_cast<qaoa_problem *>(cprob);
  if (mix->kind == 0) {
    evaluate_x(prob, p, angles, nsets, d_psi0, precision, grad, out_expect, out_grad, d_state, st);
  } else if (mix->kind == 2) {
    evaluate_grover(prob, p, angles, nsets, d_psi0, precision, grad, out_expect, out_grad, d_state, st);
  } else if (mix->kind == 3 || mix->kind == 4) {
    evaluate_xprod(prob, mix, p, angles, nsets, d_psi0, precision, grad, out_expect, out_grad, d_state, st);
  } else {
    CliqueEval ev;
    ev.table = prob->table;
    ev.vals = prob->dvals;
    ev.tbytes = prob->tbytes;
    ev.N = (int64_t)prob->N;
    ev.lut_len = (int)prob->max_value + 1;
    ev.c0 = prob->mean;
    CliqueTimer tm;
    tm.ctx = prob->ctx;
    tm.begin = hook_begin;
    tm.end = hook_end;
    clique_set_timer(*mix->clique, tm);
    clique_evaluate(*mix->clique, ev, p, angles, nsets, d_psi0, precision, grad, out_expect,
                    out_grad, d_state, st);
    profile_collect(prob->ctx);
  }
}

int qaoa_expect(const qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *angles,
                const void *d_psi0, int precision, double *out_expect, void *stream) {
  return guarded([&] {
    check_pair(prob, mix, precision);
    check_angles(p, angles, set_len(mix, p));
    REQUIRE(out_expect != nullptr, "out_expect is NULL");
    DeviceGuard g(prob->ctx->device);
    evaluate(prob, mix, p, angles, 1, d_psi0, precision, 0, out_expect, nullptr, nullptr,
             (hipStream_t)stream);
  });
}

int qaoa_expect_grad(const qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *angles,
                     const void *d_psi0, int precision, double *out_expect, double *out_grad,
                     void *stream) {
  return guarded([&] {
    check_pair(prob, mix, precision);
    check_angles(p, angles, set_len(mix, p));
    REQUIRE(out_expect && out_grad, "output pointer is NULL");
    DeviceGuard g(prob->ctx->device);
    evaluate(prob, mix, p, angles, 1, d_psi0, precision, 1, out_expect, out_grad, nullptr,
             (hipStream_t)stream);
  });
}

int qaoa_state(const qaoa_problem *prob, const qaoa_mixer *mix, int p, const double *angles,
               const void *d_psi0, int precision, void *d_out, void *stream) {
  return guarded([&] {
    check_pair(prob, mix, precision);
    check_angles(p, angles, set_len(mix, p));
    REQUIRE(d_out != nullptr, "d_out is NULL");
    DeviceGuard g(prob->ctx->device);
    double e;
    evaluate(prob, mix, p, angles, 1, d_psi0, precision, 0, &e, nullptr, d_out, (hipStream_t)stream);
  });
}

static void batched(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_probs,
                    int n_sets, int p, const double *angles, int precision, int grad,
                    double *out_expect, double *out_grad, hipStream_t st) {
  REQUIRE(probs && mixers, "probs or mixers is NULL");
  REQUIRE(n_probs >= 1 && n_sets >= 1, "n_probs and n_sets must be >= 1");
  REQUIRE(out_expect != nullptr && (!grad || out_grad != nullptr), "output pointer is NULL");
  qaoa_ctx *ctx = probs[0] ? probs[0]->ctx : nullptr;
  for (int i = 0; i < n_probs; i++) {
    check_pair(probs[i], mixers[i], precision);
    REQUIRE(probs[i]->ctx == ctx, "all problems must share one context");
    REQUIRE(set_len(mixers[i], p) == set_len(mixers[0], p), "all mixers must take the same number of angles");
  }
  const int g2p = (int)set_len(mixers[0], p);
  check_angles(p, angles, (size_t)n_sets * g2p);
  DeviceGuard g(ctx->device);
  // Grover-mixer problems: every (problem, set) pair in one launch
  std::vector<GroverItem> gitems;
  std::vector<int> gprobs;
  for (int i = 0; i < n_probs; i++) {
    if (mixers[i]->kind != 2) continue;
    qaoa_problem *pr = const_cast<qaoa_problem *>(probs[i]);
    ensure_counts(pr, st);
    for (int s = 0; s < n_sets; s++) gitems.push_back(grover_item(pr, s, (int)gprobs.size() * n_sets + s));
    gprobs.push_back(i);
  }
  if (!gitems.empty()) {
    std::vector<double> hout((size_t)gprobs.size() * n_sets * (1 + g2p));
    run_grover(gitems, angles, n_sets, p, grad, hout.data(), ctx, st);
    for (size_t j = 0; j < gprobs.size(); j++)
      for (int s = 0; s < n_sets; s++) {
        const double *r = hout.data() + ((size_t)j * n_sets + s) * (1 + g2p);
        int i = gprobs[j];
        out_expect[(size_t)i * n_sets + s] = r[0];
        if (grad) std::memcpy(out_grad + ((size_t)i * n_sets + s) * g2p, r + 1, g2p * sizeof(double));
      }
  }
  // problems on other paths (eigenbasis mixers, X products): one evaluation each
  for (int i = 0; i < n_probs; i++) {
    if (mixers[i]->kind == 0 || mixers[i]->kind == 2) continue;
    evaluate(probs[i], mixers[i], p, angles, n_sets, nullptr, precision, grad,
             out_expect + (size_t)i * n_sets, grad ? out_grad + (size_t)i * n_sets * g2p : nullptr,
             nullptr, st);
  }
  // transverse-field problems: the whole-state pairs in one launch, then every larger problem's
  // tile passes, all enqueued back to back and read after one synchronisation; from the second
  // call with the same problems, mixers, p, sets and precision on, the device work is a HIP
  // graph captured once and replayed (its parameters are re-staged in the same pinned buffers)
  std::vector<SmallItem> items;
  std::vector<int> small_probs, tile_probs;
  for (int i = 0; i < n_probs; i++) {
    if (mixers[i]->kind != 0) continue;
    if (small_path(probs[i], precision)) {
      if (probs[i]->max_value + 1 > MAX_LUT) throw fail(QAOA_ERR_UNSUPPORTED, "largest cost value exceeds the LUT limit");
      for (int s = 0; s < n_sets; s++)
        items.push_back(small_item(probs[i], s, (int)small_probs.size() * n_sets + s));
      small_probs.push_back(i);
    } else {
      tile_probs.push_back(i);
    }
  }
  if (items.empty() && tile_probs.empty()) return;
  while (ctx->bstage.size() < tile_probs.size()) {
    ctx->bstage.push_back(std::make_unique<HostBuf>());
    ctx->brstage.push_back(std::make_unique<HostBuf>());
  }
  std::vector<double> hout((size_t)small_probs.size() * n_sets * (1 + g2p));
  std::vector<std::function<void()>> fin;
  // the graph entry of this call's key
  std::vector<uint64_t> key = {(uint64_t)precision, (uint64_t)grad, (uint64_t)p, (uint64_t)n_sets};
  for (int i = 0; i < n_probs; i++)
    if (mixers[i]->kind == 0) {
      key.push_back(probs[i]->id);
      key.push_back(mixers[i]->id);
    }
  qaoa_ctx::BGraph *G = nullptr;
  for (auto &g : ctx->bgraphs)
    if (g.key == key) G = &g;
  if (!G) {
    if (ctx->bgraphs.size() >= 64) {  // bounded cache: drop the oldest entry
      for (auto ex : ctx->bgraphs.front().execs)
        if (ex) (void)hipGraphExecDestroy(ex);
      ctx->bgraphs.erase(ctx->bgraphs.begin());
    }
    ctx->bgraphs.push_back(qaoa_ctx::BGraph{});
    G = &ctx->bgraphs.back();
    G->key = key;
    G->ckpt.assign(tile_probs.size(), -1);
  }
  // Each instance follows the plan its key has (chosen by a single evaluation that tuned it),
  // else the fixed rule: a batched call does not tune. Plans timed one instance at a time
  // picked options that made the whole call slower (the batched workload: 34.5 ms tuned,
  // 34.1 ms with the fixed rule), and the staging below may be captured, where nothing can
  // be timed.
  // Units of device work: the whole-state pairs (one launch), then each tile-path instance.
  // Staging a unit (its host planning and parameter upload) overlaps the device work of the
  // units before it, eagerly and as graphs alike: one graph per unit.
  const int u0 = items.empty() ? 0 : 1, nunits = u0 + (int)tile_probs.size();
  auto stage_unit = [&](int u, bool launch, hipStream_t s, uint64_t *fp) {
    if (u < u0) {
      run_small(items, precision, angles, n_sets, p, grad, hout.data(), ctx, s, &fin, launch, fp);
      return;
    }
    const int jj = u - u0, i = tile_probs[jj];
    XDefer df{ctx->bstage[jj].get(), ctx->brstage[jj].get(), launch, &G->ckpt[jj], &fin, fp};
    qaoa_problem *pr = const_cast<qaoa_problem *>(probs[i]);
    double *oe = out_expect + (size_t)i * n_sets, *og = grad ? out_grad + (size_t)i * n_sets * g2p : nullptr;
    if (precision == QAOA_FP32)
      run_x_path<float>(pr, p, angles, n_sets, nullptr, grad, oe, og, nullptr, s, nullptr, &df);
    else
      run_x_path<double>(pr, p, angles, n_sets, nullptr, grad, oe, og, nullptr, s, nullptr, &df);
  };
  auto drop_graphs = [&]() {
    for (auto ex : G->execs)
      if (ex) (void)hipGraphExecDestroy(ex);
    G->execs.clear();
    G->fps.clear();
  };
  const uint64_t fnv0 = 1469598103934665603ull;
  const bool graphs = ctx->batch_graphs && !ctx->profiling && p <= 1024;
  if (graphs && (!st && !ctx->gstream)) HIPCHK(hipStreamCreate(&ctx->gstream));
  hipStream_t gs = st ? st : ctx->gstream;
  if (graphs && (int)G->execs.size() == nunits) {
    // replay: re-stage each unit's parameters (the captured work must be what this call
    // would enqueue) and launch its graph; a unit planned differently (e.g. another reverse-
    // sweep scalar form) and the ones after it run eagerly, and the key is captured again
    int u = 0;
    for (; u < nunits; u++) {
      const size_t nfin = fin.size();
      uint64_t fp = fnv0;
      stage_unit(u, false, gs, &fp);
      if (fp != G->fps[u]) {
        fin.resize(nfin);
        break;
      }
      HIPCHK(hipGraphLaunch(G->execs[u], gs));
    }
    if (u < nunits) {
      for (; u < nunits; u++) stage_unit(u, true, gs, nullptr);
      drop_graphs();
      G->calls = 0;
    }
    HIPCHK(hipStreamSynchronize(gs));
  } else if (graphs && G->calls >= 1) {
    // capture unit by unit (every buffer was sized by the earlier call with this key); each
    // unit's graph is launched as soon as it is instantiated
    drop_graphs();
    if (!st) HIPCHK(hipDeviceSynchronize());  // the capture stream does not order with the null stream
    int u = 0;
    for (; u < nunits; u++) {
      uint64_t fp = fnv0;
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      const size_t nfin = fin.size();
      bool ok = hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        try {
          stage_unit(u, true, gs, &fp);
        } catch (...) {
          ok = false;
        }
        ok = (hipStreamEndCapture(gs, &graph) == hipSuccess) && ok && graph;
        ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
      }
      (void)hipGetLastError();
      if (!ok) {
        if (exec) (void)hipGraphExecDestroy(exec);
        fin.resize(nfin);
        break;
      }
      G->execs.push_back(exec);
      G->fps.push_back(fp);
      HIPCHK(hipGraphLaunch(exec, gs));
    }
    if (u < nunits) {
      // not capturable: the rest runs eagerly and this key stays eager
      for (; u < nunits; u++) stage_unit(u, true, gs, nullptr);
      drop_graphs();
      G->calls = -(1 << 30);
    }
    HIPCHK(hipStreamSynchronize(gs));
  } else {
    for (int u = 0; u < nunits; u++) stage_unit(u, true, st, nullptr);
    HIPCHK(hipStreamSynchronize(st));
    G->calls++;
  }
  profile_collect(ctx);
  for (auto &f : fin) f();
  for (size_t j = 0; j < small_probs.size(); j++)
    for (int s = 0; s < n_sets; s++) {
      const double *r = hout.data() + ((size_t)j * n_sets + s) * (1 + g2p);
      int i = small_probs[j];
      out_expect[(size_t)i * n_sets + s] = r[0];
      if (grad) std::memcpy(out_grad + ((size_t)i * n_sets + s) * g2p, r + 1, g2p * sizeof(double));
    }
}

// Pair i: probs[i] with mixers[i] at angle set i. Whole-state and Grover pairs of every problem
// share one launch each; the other pairs run problem by problem, all of a problem's sets at once.
static void paired(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_pairs, int p,
                   const double *angles, int precision, int grad, double *out_expect, double *out_grad,
                   hipStream_t st) {
  REQUIRE(probs && mixers, "probs or mixers is NULL");
  REQUIRE(n_pairs >= 1, "n_pairs must be >= 1");
  REQUIRE(out_expect != nullptr && (!grad || out_grad != nullptr), "output pointer is NULL");
  qaoa_ctx *ctx = probs[0] ? probs[0]->ctx : nullptr;
  for (int i = 0; i < n_pairs; i++) {
    check_pair(probs[i], mixers[i], precision);
    REQUIRE(probs[i]->ctx == ctx, "all problems must share one context");
    REQUIRE(set_len(mixers[i], p) == set_len(mixers[0], p), "all mixers must take the same number of angles");
  }
  const int g2p = (int)set_len(mixers[0], p);
  check_angles(p, angles, (size_t)n_pairs * g2p);
  DeviceGuard g(ctx->device);
  auto scatter = [&](const double *r, int i) {
    out_expect[i] = r[0];
    if (grad) std::memcpy(out_grad + (size_t)i * g2p, r + 1, g2p * sizeof(double));
  };
  std::vector<SmallItem> items;
  std::vector<GroverItem> gitems;
  std::vector<int> rows, grows;
  std::vector<std::pair<const qaoa_problem *, const qaoa_mixer *>> keys;
  std::vector<std::vector<int>> groups;
  for (int i = 0; i < n_pairs; i++) {
    if (mixers[i]->kind == 0 && small_path(probs[i], precision)) {
      if (probs[i]->max_value + 1 > MAX_LUT) throw fail(QAOA_ERR_UNSUPPORTED, "largest cost value exceeds the LUT limit");
      items.push_back(small_item(probs[i], i, (int)rows.size()));
      rows.push_back(i);
    } else if (mixers[i]->kind == 2) {
      qaoa_problem *pr = const_cast<qaoa_problem *>(probs[i]);
      ensure_counts(pr, st);
      gitems.push_back(grover_item(pr, i, (int)grows.size()));
      grows.push_back(i);
    } else {
      const auto key = std::make_pair(probs[i], mixers[i]);
      size_t j = 0;
      while (j < keys.size() && keys[j] != key) j++;
      if (j == keys.size()) {
        keys.push_back(key);
        groups.emplace_back();
      }
      groups[j].push_back(i);
    }
  }
  if (!items.empty()) {
    std::vector<double> hout(rows.size() * (1 + g2p));
    run_small(items, precision, angles, n_pairs, p, grad, hout.data(), ctx, st);
    for (size_t j = 0; j < rows.size(); j++) scatter(hout.data() + j * (1 + g2p), rows[j]);
  }
  if (!gitems.empty()) {
    std::vector<double> hout(grows.size() * (1 + g2p));
    run_grover(gitems, angles, n_pairs, p, grad, hout.data(), ctx, st);
    for (size_t j = 0; j < grows.size(); j++) scatter(hout.data() + j * (1 + g2p), grows[j]);
  }
  std::vector<double> a, e, gr;
  for (size_t j = 0; j < keys.size(); j++) {
    const int m = (int)groups[j].size();
    a.resize((size_t)m * g2p);
    e.resize(m);
    gr.resize((size_t)m * g2p);
    for (int t = 0; t < m; t++)
      std::memcpy(&a[(size_t)t * g2p], angles + (size_t)groups[j][t] * g2p, g2p * sizeof(double));
    evaluate(keys[j].first, keys[j].second, p, a.data(), m, nullptr, precision, grad, e.data(),
             grad ? gr.data() : nullptr, nullptr, st);
    for (int t = 0; t < m; t++) {
      const int i = groups[j][t];
      out_expect[i] = e[t];
      if (grad) std::memcpy(out_grad + (size_t)i * g2p, &gr[(size_t)t * g2p], g2p * sizeof(double));
    }
  }
}

int qaoa_expect_pairs(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_pairs, int p,
                      const double *angles, int precision, double *out_expect, void *stream) {
  return guarded([&] {
    paired(probs, mixers, n_pairs, p, angles, precision, 0, out_expect, nullptr, (hipStream_t)stream);
  });
}

int qaoa_expect_grad_pairs(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_pairs, int p,
                           const double *angles, int precision, double *out_expect, double *out_grad,
                           void *stream) {
  return guarded([&] {
    paired(probs, mixers, n_pairs, p, angles, precision, 1, out_expect, out_grad, (hipStream_t)stream);
  });
}

int qaoa_expect_grad_pairs_noalloc(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers, int n_pairs,
                                   int p, const double *angles, int precision, double *out_expect, double *out_grad,
                                   void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    REQUIRE(probs && mixers, "probs or mixers is NULL");
    REQUIRE(n_pairs >= 1, "n_pairs must be >= 1");
    REQUIRE(out_expect && out_grad, "output pointer is NULL");
    qaoa_ctx *ctx = probs[0] ? probs[0]->ctx : nullptr;
    for (int i = 0; i < n_pairs; i++) {
      check_pair(probs[i], mixers[i], precision);
      REQUIRE(probs[i]->ctx == ctx, "all problems must share one context");
      if (mixers[i]->kind != 0 || !small_path(probs[i], precision))
        throw fail(QAOA_ERR_UNSUPPORTED, "the allocation-free call takes transverse-field pairs whose state fits "
                                         "one workgroup (n <= 13 for QAOA_FP32, n <= 12 for QAOA_FP64)");
      if (probs[i]->max_value + 1 > MAX_LUT) throw fail(QAOA_ERR_UNSUPPORTED, "largest cost value exceeds the LUT limit");
    }
    check_angles(p, angles, (size_t)n_pairs * 2 * p);
    // layout of the scratch array: items | angle sets | result rows, each 256-byte aligned
    const int rowlen = 1 + 2 * p;
    const size_t ib = (size_t)n_pairs * sizeof(SmallItem);
    const size_t off_a = (ib + 255) & ~size_t(255);
    const size_t ab = (size_t)n_pairs * 2 * p * sizeof(double);
    const size_t off_r = (off_a + ab + 255) & ~size_t(255);
    const size_t total = off_r + (size_t)n_pairs * rowlen * sizeof(double);
    if (total > NOALLOC_SCRATCH_BYTES)
      throw fail(QAOA_ERR_INVALID_ARG, "n_pairs x p needs " + std::to_string(total) + " bytes of scratch, more than the " +
                                           std::to_string(NOALLOC_SCRATCH_BYTES) + " the allocation-free call holds");
    DeviceGuard g(ctx->device);
    unsigned char *d = ctx->scratch;
    REQUIRE(d == scratch_address(ctx->device), "scratch address differs from the context's device");
    // items grouped as the whole-state path groups them: register-resident kernel by
    // (n, table width), then the LDS kernel; row i of the results is pair i
    struct Group { int n, tb; size_t first, count; };
    Group groups[4];
    int ng = 0;
    size_t m = 0;
    for (int n : {12, 13})
      for (int tb : {1, 2}) {
        if (!whole_supported(precision, n)) continue;
        const size_t first = m;
        for (int i = 0; i < n_pairs; i++)
          if (probs[i]->n == n && probs[i]->tbytes == tb) g_noalloc_items[m++] = small_item(probs[i], i, i);
        if (m > first) groups[ng++] = Group{n, tb, first, m - first};
      }
    const size_t nwhole = m;
    int max_n = 1, max_tb = 1, max_lut = 1;
    for (int i = 0; i < n_pairs; i++) {
      max_lut = std::max(max_lut, (int)probs[i]->max_value + 1);
      if (whole_supported(precision, probs[i]->n)) continue;
      g_noalloc_items[m++] = small_item(probs[i], i, i);
      max_n = std::max(max_n, probs[i]->n);
      max_tb = std::max(max_tb, probs[i]->tbytes);
    }
    max_lut = (max_lut + 15) & ~15;
    HIPCHK(hipMemcpyAsync(d, g_noalloc_items, ib, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d + off_a, angles, ab, hipMemcpyHostToDevice, st));
    const SmallItem *ditems = (const SmallItem *)d;
    const double *dang = (const double *)(d + off_a);
    double *dres = (double *)(d + off_r);
    for (int j = 0; j < ng; j++)
      HIPCHK(launch_whole(precision, groups[j].n, groups[j].tb, ditems + groups[j].first, (int)groups[j].count,
                          max_lut, dang, p, 1, dres, st, 0));
    if ((size_t)n_pairs > nwhole)
      HIPCHK(launch_small(precision, ditems + nwhole, (int)(n_pairs - nwhole), max_n, max_tb, max_lut, dang, p, 1,
                          dres, st, 0));
    // row i = [<C>, gradient]: the first column to out_expect, the rest to out_grad
    const size_t pitch = (size_t)rowlen * sizeof(double);
    HIPCHK(hipMemcpy2DAsync(out_expect, sizeof(double), dres, pitch, sizeof(double), n_pairs,
                            hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpy2DAsync(out_grad, 2 * p * sizeof(double), dres + 1, pitch, 2 * p * sizeof(double), n_pairs,
                            hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  });
}

int qaoa_expect_batched(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers,
                        int n_probs, int n_sets, int p, const double *angles, int precision,
                        double *out_expect, void *stream) {
  return guarded([&] {
    batched(probs, mixers, n_probs, n_sets, p, angles, precision, 0, out_expect, nullptr,
            (hipStream_t)stream);
  });
}

int qaoa_expect_grad_batched(const qaoa_problem *const *probs, const qaoa_mixer *const *mixers,
                             int n_probs, int n_sets, int p, const double *angles, int precision,
                             double *out_expect, double *out_grad, void *stream) {
  return guarded([&] {
    batched(probs, mixers, n_probs, n_sets, p, angles, precision, 1, out_expect, out_grad,
            (hipStream_t)stream);
  });
}

}  // extern "C"
