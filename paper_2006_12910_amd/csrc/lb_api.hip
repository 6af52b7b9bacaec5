// lb_api.hip -- C ABI of the library (declared in include/lb.h): argument
// validation, workspace layout, per-step launch sequence, hipGraph capture of
// step chunks, batching, host<->device transfers and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "lb.h"
#include "launch.h"

using namespace lbk;

namespace {

thread_local std::string g_err;

lb_status fail(lb_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(LB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
int storage_bytes(int st) { return st == LB_F64 ? 8 : (st == LB_F32 ? 4 : 2); }

constexpr int NPARTIALS = 1024;
constexpr size_t STAGE_TARGET = size_t(16) << 20;  // bytes of the host-transfer staging band

struct Layout {
  int pitch = 0, band_rows = 0;
  size_t desc = 0, hdr = 0, f0 = 0, f1 = 0, label = 0, nodew = 0, ps0 = 0, ps1 = 0, pforce = 0,
         items = 0, near = 0, near_bytes = 0,
         partials = 0, stage = 0, prefix = 0, total = 0;
};

// header block: step counter, health word, density sum, drift control
struct Header {
  uint64_t tstep;
  uint32_t health;
  uint32_t pad;
  double mass;
  double mass_ctl[2];  // reference density sum, relative tolerance (0: off)
};

// FP64 density sum: one block per ~4 rows of 256 nodes (rows are summed
// whole), at most one per row and at most NPARTIALS blocks
int mass_blocks_of(int nx, int ny) {
  const long long nodes = (long long)nx * ny;
  return (int)std::min<long long>({(long long)NPARTIALS, (long long)ny,
                                   std::max<long long>(1, nodes / 1024)});
}

// A label plane holds obstacles, particles and walls.  Walls of a domain
// without obstacles or particles could also be index walls (mirror writes, no
// plane), but as solid label rows they let the two-step sweep run on
// channels; only domains with a pressure face keep index walls.
bool needs_labels(const lb_domain_desc *d) {
  return d->obstacles != 0 || d->max_particles > 0 ||
         ((d->bc_x == LB_WALL || d->bc_y == LB_WALL) && d->bc_x != LB_PRESSURE);
}

Layout layout_of(const lb_domain_desc *d) {
  Layout L;
  L.pitch = (d->nx + 63) / 64 * 64;
  const size_t plane = (size_t)d->ny * L.pitch;
  const size_t fbytes = 9 * plane * storage_bytes(d->storage);
  const size_t row_stage = (size_t)9 * d->nx * sizeof(double);
  L.band_rows = (int)std::max<size_t>(1, std::min<size_t>(d->ny, STAGE_TARGET / row_stage));
  size_t o = 0;
  L.desc = o; o += align256(sizeof(DevDomain));
  L.hdr = o; o += align256(sizeof(Header));
  L.f0 = o; o += align256(fbytes);
  L.f1 = o; o += align256(fbytes);
  L.label = o; if (needs_labels(d)) o += align256(plane);
  L.nodew = o; if (needs_labels(d)) o += align256(plane * sizeof(uint16_t));
  const size_t np = (size_t)std::max(d->max_particles, 0);
  L.ps0 = o; o += align256(np * sizeof(PState));
  L.ps1 = o; o += align256(np * sizeof(PState));
  L.pforce = o; o += align256(np * sizeof(PForce));
  L.items = o; o += align256(np * sizeof(PItem));
  // tile flags of the overlapped particle step: two sets, sized for the
  // smallest tiles (64 x 4 nodes)
  L.near_bytes = np ? (size_t)((d->nx + 63) / 64) * (size_t)((d->ny + 3) / 4) : 0;
  L.near = o; o += 2 * align256(L.near_bytes);
  L.partials = o; o += align256(NPARTIALS * sizeof(double));
  L.stage = o; o += align256((size_t)L.band_rows * row_stage);
  L.prefix = o; o += align256(8 * sizeof(int));
  L.total = o;
  return L;
}

lb_status validate(const lb_domain_desc *d) {
  if (!d) return fail(LB_EINVAL, "desc is null");
  if (d->abi_version != LB_ABI_VERSION) return fail(LB_EINVAL, "abi_version mismatch");
  if (d->nx < 3 || d->ny < 3 || d->nx > 65536 || d->ny > 65536)
    return fail(LB_EINVAL, "nx, ny must be in [3, 65536]");
  if (d->storage < LB_F64 || d->storage > LB_BF16_DELTA) return fail(LB_EINVAL, "bad storage");
  {
    const long long vbytes = d->storage == LB_F64 ? 8 : (d->storage == LB_F32 ? 4 : 2);
    if ((long long)((d->nx + 63) / 64 * 64) * d->ny * 9 * vbytes >= (1LL << 32))
      return fail(LB_EINVAL, "lattice too large: a population buffer must span fewer than 2^32 bytes");
  }
  if (d->bc_x < LB_PERIODIC || d->bc_x > LB_PRESSURE) return fail(LB_EINVAL, "bad bc_x");
  if (d->bc_y != LB_PERIODIC && d->bc_y != LB_WALL) return fail(LB_EINVAL, "bad bc_y");
  if (d->storage < LB_F64 || d->storage > LB_BF16_DELTA) return fail(LB_EINVAL, "bad storage");
  if (d->rounding != LB_ROUND_NEAREST && d->rounding != LB_ROUND_STOCHASTIC)
    return fail(LB_EINVAL, "bad rounding");
  if (d->rounding == LB_ROUND_STOCHASTIC && d->storage == LB_F64)
    return fail(LB_EINVAL, "stochastic rounding needs FP32 or 16-bit storage");
  if (d->rounding == LB_ROUND_STOCHASTIC && d->storage == LB_F32 && d->compute == LB_COMPUTE_F64)
    return fail(LB_EINVAL, "stochastic rounding of FP32 storage needs FP32 arithmetic");
  if (d->compute != LB_COMPUTE_NATIVE && d->compute != LB_COMPUTE_F64)
    return fail(LB_EINVAL, "bad compute");
  if (d->max_particles < 0 || d->max_particles > MAX_PARTICLES)
    return fail(LB_EINVAL, "max_particles must be in [0, 250]");
  if (!(d->rho0 > 0.0) || !std::isfinite(d->rho0)) return fail(LB_EINVAL, "rho0 must be > 0");
  if (!d->power_law && !(d->tau > 0.5)) return fail(LB_EINVAL, "tau must be > 1/2");
  if (d->power_law) {
    if (!(d->tau_min > 0.5) || !(d->tau_max >= d->tau_min) || !(d->n_index > 0.0) || !(d->K > 0.0))
      return fail(LB_EINVAL, "power law needs n > 0, K > 0, 1/2 < tau_min <= tau_max");
  }
  if (!(d->kT >= 0.0)) return fail(LB_EINVAL, "kT must be >= 0");
  if (d->collision != LB_BGK && d->collision != LB_TRT)
    return fail(LB_EINVAL, "collision must be LB_BGK or LB_TRT");
  if (d->collision == LB_TRT && !(d->magic > 0.0 && std::isfinite(d->magic)))
    return fail(LB_EINVAL, "TRT magic number must be finite and > 0");
  if (d->collision == LB_TRT && d->kT > 0.0)
    return fail(LB_EUNSUPPORTED,
                "TRT with thermal noise: the noise amplitudes follow the BGK relaxation of each mode");
  if (!std::isfinite(d->gx) || !std::isfinite(d->gy)) return fail(LB_EINVAL, "g not finite");
  if (d->bc_x == LB_PRESSURE && (!(d->rho_in > 0.0) || !(d->rho_out > 0.0)))
    return fail(LB_EINVAL, "pressure faces need rho_in, rho_out > 0");
  if (d->max_particles > 0 && (!(d->lj_rit > 0.0) || !(d->lj_floor > 0.0) || !(d->lj_psi >= 0.0)))
    return fail(LB_EINVAL, "particles need lj_rit > 0, lj_floor > 0, lj_psi >= 0");
  if (d->init_kind != LB_INIT_REST && d->init_kind != LB_INIT_FIELDS)
    return fail(LB_EINVAL, "bad init_kind");
  if (d->init_kind == LB_INIT_FIELDS && (!d->init_rho || !d->init_ux || !d->init_uy))
    return fail(LB_EINVAL, "LB_INIT_FIELDS needs init_rho, init_ux, init_uy");
  return LB_OK;
}

int plm_of(double n) {
  if (n == 0.5) return PL_HALF;
  if (n == 0.75) return PL_3Q;
  if (n == 1.5) return PL_3H;
  return PL_GENERIC;
}

int feat_of(const lb_domain_desc *d) {
  int f = 0;
  if (needs_labels(d)) f |= F_LABELS;
  if (d->kT > 0.0) f |= F_NOISE;
  if (d->power_law) f |= F_POWER;
  if (d->bc_x == LB_PRESSURE) f |= F_PRESSURE;
  if (d->rounding == LB_ROUND_STOCHASTIC) f |= F_STOCH;
  if (d->collision == LB_TRT) f |= F_TRT;
  return f;
}

bool get_kernels(int st, int feat, int plm, int wide, KernelSet *k) {
  switch (st) {
    case LB_F64: return kernels_f64(feat, plm, wide, k);
    case LB_F32: return kernels_f32(feat, plm, wide, k);
    case LB_F16_DELTA: return kernels_f16(feat, plm, wide, k);
    case LB_BF16_DELTA: return kernels_bf16(feat, plm, wide, k);
  }
  return false;
}

int default_tile_w(int nx) { return nx >= 256 ? 256 : (nx >= 128 ? 128 : 64); }

// The sweep streams its stores past the caches when the step's working set
// (both population buffers of every domain in the launch) is at least this
// large; below it the next step finds the written lines in the 256 MB
// last-level cache.
constexpr size_t STREAM_STORE_MIN_BYTES = (size_t)256 << 20;
size_t sweep_working_set(const DevDomain &h) {
  return 2 * 9 * (size_t)storage_bytes(h.storage) * (size_t)h.pitch * (size_t)h.ny;
}

// Graph cache of captured step chunks, keyed by chunk length.
struct GraphCache {
  std::map<int, hipGraphExec_t> execs;
  void clear() {
    for (auto &kv : execs) (void)hipGraphExecDestroy(kv.second);
    execs.clear();
  }
};

}  // namespace

namespace lbk {
// the error record of the D3Q19 entry points (lb3_api.hip): the same
// thread-local text lb_last_error returns
lb_status lb_fail(lb_status s, const std::string &msg) { return fail(s, msg); }
// The error record where an allocation has just failed: the message is kept
// if it can be, and nothing is thrown.
lb_status lb_fail_nothrow(lb_status s, const char *msg) noexcept {
  try {
    g_err = msg;
  } catch (...) {
  }
  return s;
}
}  // namespace lbk

struct lb_domain {
  lb_domain_desc desc{};
  Layout L;
  int device = 0;  // the device current at creation (the workspace's)
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  DevDomain hd{};
  int feat = 0, plm = 0;
  KernelSet ks{};
  int np = 0;
  int64_t t = 0;
  bool use_graph = true;
  int chunk = 256;
  bool two_step = true;  // LB_OPT_TWO_STEP
  bool overlap = false;  // LB_OPT_OVERLAP
  int64_t mass_interval = 256;  // LB_OPT_MASS_INTERVAL
  hipStream_t side = nullptr;  // particle chain of an overlapped step
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  GraphCache graphs;
  int in_batches = 0;
  std::vector<uint8_t> host_labels;  // walls + obstacles, [ny][pitch]
  // asynchronous moment output: moments computed (on stream), copied out
  // (on the caller's copy stream); a copy in flight until lb_moments_wait
  hipEvent_t rep_ready = nullptr, rep_copied = nullptr;
  bool rep_pending = false;

  DevDomain *ddesc() const { return (DevDomain *)(ws + L.desc); }
  Header *dhdr() const { return (Header *)(ws + L.hdr); }
  int *dprefix() const { return (int *)(ws + L.prefix); }
  int *dprefix2() const { return dprefix() + 2; }  // tiles of the two-step sweep
  int *dprefixm() const { return dprefix() + 4; }  // blocks of the density sum
  PItem *ditems() const { return (PItem *)(ws + L.items); }
  int ntiles() const { return hd.tiles_x * hd.tiles_y; }
  int ntiles2() const { return hd.tiles2_x * hd.tiles2_y; }
};

struct lb_batch {
  std::vector<lb_domain *> doms;
  char *ws = nullptr;
  hipStream_t stream = nullptr, cap = nullptr;
  KernelSet ks{};
  int total_tiles = 0, total_tiles2 = 0, total_mass_blocks = 0, nitems = 0;
  bool two_step = false;  // every domain takes the two-step sweep
  int rows2 = 0;          // its tile height, shared by the launch
  std::vector<DevDomain> hdescs;  // host copies of the descriptors
  std::vector<int> hprefix;       // and of the prefix tables
  size_t off_desc = 0, off_prefix = 0, off_items = 0, bytes = 0;
  bool use_graph = true;
  int chunk = 256;
  int64_t t = 0;                // steps since creation
  int64_t mass_interval = 256;  // LB_OPT_MASS_INTERVAL
  GraphCache graphs;
  DevDomain *ddesc() const { return (DevDomain *)(ws + off_desc); }
  int *dprefix() const { return (int *)(ws + off_prefix); }
  int *dprefix2() const { return dprefix() + doms.size() + 1; }
  int *dprefixm() const { return dprefix() + 2 * (doms.size() + 1); }  // density-sum blocks
  PItem *ditems() const { return (PItem *)(ws + off_items); }
};

namespace {

// Two-step sweep tiles: TS_COLS columns by `rows` rows.
void set_two_step_rows(DevDomain &hd, int rows) {
  hd.rows2 = rows;
  hd.tiles2_x = (hd.nx + TS_COLS - 1) / TS_COLS;
  hd.tiles2_y = (hd.ny + rows - 1) / rows;
}
bool valid_two_step_rows(int storage, int64_t rows) {
  for (int k = 0; k < 3; ++k)
    if (rows == two_step_rows_of(storage, k)) return true;
  return false;
}

// Tile heights the autotuner chose, per (storage, label plane, stochastic
// rounding, size class = floor(log2(sites))), for this process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_rows2_cache;
std::tuple<int, int, int, int> tune_key(int storage, int feat, long long sites) {
  int cls = 0;
  while ((1LL << (cls + 1)) <= sites) ++cls;
  return {storage, (feat & F_LABELS) ? 1 : 0, (feat & F_STOCH) ? 1 : 0, cls};
}

// A tile is tile_w threads (nodes) along x by (256 / tile_w) * rpt rows.
void set_tiles(DevDomain &hd, int tile_w, int rpt) {
  hd.tile_w = tile_w;
  hd.rows_per_thread = rpt;
  hd.tiles_x = (hd.nx + tile_w - 1) / tile_w;
  const int th = (256 / tile_w) * rpt;
  hd.tiles_y = (hd.ny + th - 1) / th;
}

lb_status push_desc(lb_domain *d) {
  HIPCHK(hipMemcpyAsync(d->ddesc(), &d->hd, sizeof(DevDomain), hipMemcpyHostToDevice, d->stream));
  int pre[6] = {0, d->ntiles(), 0, d->ntiles2(), 0, d->hd.mass_blocks};
  HIPCHK(hipMemcpyAsync(d->dprefix(), pre, sizeof(pre), hipMemcpyHostToDevice, d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  return LB_OK;
}

lb_status check_health(lb_domain *d) {
  uint32_t h = 0;
  HIPCHK(hipMemcpyAsync(&h, &d->dhdr()->health, sizeof(h), hipMemcpyDeviceToHost, d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  if (h) {
    std::string m = "device latched:";
    if (h & HEALTH_NONFINITE) m += " non-finite density;";
    if (h & HEALTH_FAST_PARTICLE) m += " particle faster than 0.5 nodes/step;";
    if (h & HEALTH_LINK_OVERFLOW) m += " particle link list overflow;";
    if (h & HEALTH_MASS_DRIFT) m += " density sum drifted beyond the set tolerance;";
    return fail(LB_EUNSTABLE, m);
  }
  return LB_OK;
}

// What one step (or step pair) of a domain or batch launches.
struct StepPlan {
  const KernelSet *ks;
  const DevDomain *doms;
  const int *prefix;   // single-step tiles per domain
  const int *prefix2;  // two-step tiles per domain
  int ndom, blocks, blocks2;
  const PItem *items;
  int nitems;
  bool two;  // two-step sweep (no particles, so no pre/post passes)
  int rows2 = 0;  // its tile height (every domain of the launch shares it)
  // no domain of the launch holds more than one particle: the post pass of a
  // step and the pre pass of the next run as one launch (k_post_pre)
  bool fuse_pp = false;
  // overlapped particle steps (one domain): the particle chain on `side`
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int ntiles = 0;
};

// Steps of one domain with particles, the particle coupling overlapping the
// bulk of the sweep (the analogue of the paper's pipelining of the particle
// interaction of one step with the streaming of the next, Sec. 7).  Step k
// forks: stream s sweeps the tiles no coupling of the step touches, while
// `side` runs k_post of step k - 1, k_pre of step k, the tile flags of step
// k + 1 (from P(T + 1), which k_pre has just computed) and then the sweep of
// the flagged tiles; the branches join before the next step.  The two
// branches touch disjoint memory: the flagged tiles cover, with the sweep's
// halo and a margin, every node whose label or link slot the coupling reads
// or writes; the flags of a step and of the next one live in the two halves
// of near_tiles.  Every node is still computed by the same kernel code from
// the same inputs, so the result is bit-identical to the serial order.  The
// last step's k_post runs after the join, so a call ends in the same state.
void record_overlapped(const StepPlan &p, int n, hipStream_t s) {
  launch_near_tiles(p.doms, p.ntiles, 0, s);
  for (int k = 0; k < n; ++k) {
    (void)hipEventRecord(p.ev_fork, s);
    (void)hipStreamWaitEvent(p.side, p.ev_fork, 0);
    if (k > 0) p.ks->post(p.doms, p.items, p.nitems, k - 1, p.side);
    p.ks->pre(p.doms, p.items, p.nitems, k, p.side);
    launch_near_tiles(p.doms, p.ntiles, k + 1, p.side);
    p.ks->sweep(p.doms, p.prefix, p.ndom, k, p.blocks, 2, p.side);
    p.ks->sweep(p.doms, p.prefix, p.ndom, k, p.blocks, 1, s);
    (void)hipEventRecord(p.ev_join, p.side);
    (void)hipStreamWaitEvent(s, p.ev_join, 0);
  }
  p.ks->post(p.doms, p.items, p.nitems, n - 1, s);
  launch_advance(p.doms, p.ndom, n, s);
}

// Enqueue `n` steps of the launch sequence on stream s (eager or under
// capture).  With the two-step sweep, each four steps are a pair of two-step
// launches (the first leaves the state in the buffer of the other parity, the
// second brings it back, so the state is where single steps expect it after
// every pair); the n mod 4 remaining steps are single steps.
void record_steps(const StepPlan &p, int n, hipStream_t s) {
  int k = 0;
  if (p.two) {
    for (; k + 4 <= n; k += 4) {
      p.ks->sweep2(p.doms, p.prefix2, p.ndom, k, 0, p.blocks2, p.rows2, s);
      p.ks->sweep2(p.doms, p.prefix2, p.ndom, k + 2, 1, p.blocks2, p.rows2, s);
    }
  }
  if (p.side != nullptr && p.nitems > 0 && n > 0) {
    record_overlapped(p, n, s);
    return;
  }
  for (; k < n; ++k) {
    // with fuse_pp, the pre pass of step k > 0 ran in the launch before
    if (p.nitems > 0 && !(p.fuse_pp && k > 0)) p.ks->pre(p.doms, p.items, p.nitems, k, s);
    p.ks->sweep(p.doms, p.prefix, p.ndom, k, p.blocks, 0, s);
    if (p.nitems > 0) {
      if (p.fuse_pp && k + 1 < n)
        p.ks->post_pre(p.doms, p.items, p.nitems, k, s);
      else
        p.ks->post(p.doms, p.items, p.nitems, k, s);  // a call ends after a post pass
    }
  }
  launch_advance(p.doms, p.ndom, n, s);
}

// Step counts of the captured graphs: the chunk length and every power of
// four below it.  A call of n steps replays them largest first, so a handle
// holds at most a handful of graphs, and all of them are captured by the
// first call: no later call captures or instantiates anything, whatever its
// step count.  Every size but 1 is a multiple of four, so the two-step sweep
// runs in launch pairs and only the n mod 4 last steps are single steps.
std::vector<int> graph_sizes(int chunk) {
  std::vector<int> v{chunk};
  int p = 1;
  while (p * 4 < chunk) p *= 4;
  for (; p >= 1; p /= 4)
    if (p < chunk) v.push_back(p);
  return v;
}

lb_status capture(GraphCache &gc, hipStream_t stream, hipStream_t cap, const StepPlan &p, int n) {
  if (gc.execs.count(n)) return LB_OK;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  record_steps(p, n, cap);
  hipError_t le = hipGetLastError();
  HIPCHK(hipStreamEndCapture(cap, &g));
  if (le != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(LB_EHIP, std::string("kernel launch during capture: ") + hipGetErrorString(le));
  }
  hipGraphExec_t ex = nullptr;
  hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return fail(LB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  gc.execs.emplace(n, ex);
  // upload now, so that the first replay carries no set-up cost
  HIPCHK(hipGraphUpload(ex, stream));
  return LB_OK;
}

// Enqueue n steps on `stream`: eager launches, or replays of the captured
// step graphs.
lb_status run_steps(GraphCache &gc, bool use_graph, int chunk, hipStream_t stream, hipStream_t cap,
                    const StepPlan &p, int64_t n) {
  if (!use_graph) {
    while (n > 0) {
      const int c = (int)std::min<int64_t>(n, chunk);
      record_steps(p, c, stream);
      HIPCHK(hipGetLastError());
      n -= c;
    }
    return LB_OK;
  }
  const std::vector<int> sizes = graph_sizes(chunk);
  for (int c : sizes) {
    lb_status s = capture(gc, stream, cap, p, c);
    if (s != LB_OK) return s;
  }
  for (int c : sizes) {
    const hipGraphExec_t ex = gc.execs.at(c);
    for (; n >= c; n -= c) HIPCHK(hipGraphLaunch(ex, stream));
  }
  return LB_OK;
}

// The two-step sweep serves periodic domains without particles whose kernel
// set has one (no noise, no power law, native arithmetic), unless switched
// off with LB_OPT_TWO_STEP.
// The two-step sweep needs periodic edges or walls held as solid label rows
// (its tiles wrap around the domain), and no particle or pressure face.
bool two_step_ok(const lb_domain *d) {
  const bool edges = (d->desc.bc_x == LB_PERIODIC && d->desc.bc_y == LB_PERIODIC) ||
                     (d->hd.label != nullptr && d->desc.bc_x != LB_PRESSURE);
  return d->two_step && d->ks.sweep2 != nullptr && d->np == 0 && d->desc.max_particles == 0 && edges;
}

// FP64 density sum of the current state; its final kernel also latches a
// non-finite state (the sweep checks the densities it pulls, so a blow-up in
// the last step of a call is caught here).
// Does a call that advances the step counter from t0 by n steps pass a
// multiple of the density-check interval?
bool check_due(int64_t t0, int64_t n, int64_t interval) {
  return n > 0 && (t0 + n) / interval != t0 / interval;
}

lb_status domain_mass_enqueue(lb_domain *d) {
  d->ks.mass_partial(d->ddesc(), d->dprefixm(), 1, d->hd.mass_blocks, nullptr, d->stream);
  launch_mass_final(d->ddesc(), 1, nullptr, nullptr, d->stream);
  HIPCHK(hipGetLastError());
  return LB_OK;
}

// Mirror slots of the index walls of a label-free domain in the current
// population buffer (label domains bounce back on the pulling node's own slot).
lb_status refresh_mirrors(lb_domain *d) {
  if (d->hd.label || (d->desc.bc_x != LB_WALL && d->desc.bc_y != LB_WALL)) return LB_OK;
  d->ks.mirror(d->ddesc(), d->desc.nx, d->desc.ny, d->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(d->stream));
  return LB_OK;
}

lb_status upload_labels(lb_domain *d) {
  HIPCHK(hipMemcpyAsync(d->ws + d->L.label, d->host_labels.data(), d->host_labels.size(),
                        hipMemcpyHostToDevice, d->stream));
  launch_masks_full(d->ddesc(), d->desc.nx, d->desc.ny, d->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(d->stream));
  return refresh_mirrors(d);
}

// ms per step of `n` steps run by step(n) on stream s, after one untimed
// call of the same length (which also captures its graphs).
template <class F> lb_status time_steps(F &&step, hipStream_t s, int n, double *ms_per_step) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  lb_status st = step(n);
  if (st == LB_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(LB_EHIP, "event");
  if (st == LB_OK) st = step(n);
  if (st == LB_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
    st = fail(LB_EHIP, "event");
  float ms = 0.f;
  if (st == LB_OK) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_per_step = ms / n;
  return st;
}
}  // namespace

// Every entry point runs its body through LB_GUARDED, so that no C++
// exception (a failed host allocation, say) crosses the C ABI.
#define LB_GUARDED(call)                                                           \
  try {                                                                            \
    return call;                                                                   \
  } catch (const std::bad_alloc &) {                                               \
    return lbk::lb_fail_nothrow(LB_ENOMEM, "host memory allocation failed");       \
  } catch (...) {                                                                  \
    return lbk::lb_fail_nothrow(LB_EHIP, "unexpected internal error");             \
  }

extern "C" {

const char *lb_status_string(lb_status s) {
  switch (s) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument";
    case LB_ENOMEM: return "workspace too small";
    case LB_EHIP: return "HIP runtime error";
    case LB_ESTATE: return "call not allowed in this state";
    case LB_EUNSTABLE: return "simulation became unstable";
    case LB_EUNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

const char *lb_last_error(void) { return g_err.c_str(); }

static lb_status lb_workspace_bytes_impl(const lb_domain_desc *desc, size_t *bytes) {
  if (!bytes) return fail(LB_EINVAL, "bytes is null");
  lb_status s = validate(desc);
  if (s != LB_OK) return s;
  *bytes = layout_of(desc).total;
  return LB_OK;
}

lb_status lb_workspace_bytes(const lb_domain_desc *desc, size_t *bytes) {
  LB_GUARDED(lb_workspace_bytes_impl(desc, bytes));
}

static lb_status lb_create_domain_impl(const lb_domain_desc *desc, void *dev_workspace, size_t bytes,
                                       void *hip_stream, lb_domain **out) {
  if (!out) return fail(LB_EINVAL, "out is null");
  *out = nullptr;
  lb_status s = validate(desc);
  if (s != LB_OK) return s;
  if (!dev_workspace || ((uintptr_t)dev_workspace & 255)) return fail(LB_EINVAL, "workspace must be non-null and 256-byte aligned");
  Layout L = layout_of(desc);
  if (bytes < L.total) return fail(LB_ENOMEM, "workspace smaller than lb_workspace_bytes");
  const int feat = feat_of(desc);
  const int plm = desc->power_law ? plm_of(desc->n_index) : PL_GENERIC;
  KernelSet ks{};
  if (!get_kernels(desc->storage, feat, plm, desc->compute == LB_COMPUTE_F64, &ks))
    return fail(LB_EUNSUPPORTED, "no kernel for this feature set");

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LB_EHIP, "hipGetDevice failed");
  lb_domain *d = new lb_domain();
  d->device = dev;
  d->desc = *desc;
  d->desc.init_rho = d->desc.init_ux = d->desc.init_uy = nullptr;
  d->L = L;
  d->ws = (char *)dev_workspace;
  d->stream = (hipStream_t)hip_stream;
  d->feat = feat;
  d->plm = plm;
  d->ks = ks;
  if (hipStreamCreateWithFlags(&d->cap, hipStreamNonBlocking) != hipSuccess) {
    delete d;
    return fail(LB_EHIP, "hipStreamCreateWithFlags failed");
  }
  DevDomain &h = d->hd;
  h.f[0] = d->ws + L.f0;
  h.f[1] = d->ws + L.f1;
  h.label = needs_labels(desc) ? (uint8_t *)(d->ws + L.label) : nullptr;
  h.nodew = needs_labels(desc) ? (uint16_t *)(d->ws + L.nodew) : nullptr;
  h.tstep = &d->dhdr()->tstep;
  h.health = &d->dhdr()->health;
  h.partials = (double *)(d->ws + L.partials);
  h.mass_out = &d->dhdr()->mass;
  h.mass_ctl = d->dhdr()->mass_ctl;
  h.mass_blocks = mass_blocks_of(desc->nx, desc->ny);
  h.pstate[0] = (PState *)(d->ws + L.ps0);
  h.pstate[1] = (PState *)(d->ws + L.ps1);
  h.pforce = (PForce *)(d->ws + L.pforce);
  h.near_tiles[0] = L.near_bytes ? (uint8_t *)(d->ws + L.near) : nullptr;
  h.near_tiles[1] = L.near_bytes ? (uint8_t *)(d->ws + L.near + align256(L.near_bytes)) : nullptr;
  h.nx = desc->nx;
  h.ny = desc->ny;
  h.pitch = L.pitch;
  h.bc_x = desc->bc_x;
  h.bc_y = desc->bc_y;
  h.np = 0;
  h.storage = desc->storage;
  h.key0 = (uint32_t)desc->seed;
  h.key1 = (uint32_t)(desc->seed >> 32) ^ desc->domain_id;
  h.feat = feat;
  set_tiles(h, default_tile_w(desc->nx), desc->storage >= LB_F16_DELTA ? 4 : 2);
  h.stream_stores = sweep_working_set(h) >= STREAM_STORE_MIN_BYTES;
  set_two_step_rows(h, two_step_rows(h.storage));
  h.rho0 = desc->rho0;
  h.tau = desc->power_law ? desc->tau_min : desc->tau;
  h.omega = 1.0 / h.tau;
  h.gx = desc->gx;
  h.gy = desc->gy;
  h.drho_in = desc->rho_in - desc->rho0;
  h.drho_out = desc->rho_out - desc->rho0;
  h.kT = desc->kT;
  h.pl_n = desc->n_index;
  h.pl_K = desc->K;
  h.tau_min = desc->tau_min;
  h.tau_max = desc->tau_max;
  h.lj_psi = desc->lj_psi;
  h.lj_rit = desc->lj_rit;
  h.lj_floor = desc->lj_floor;
  h.rho0_f = (float)h.rho0;
  h.tau_f = (float)h.tau;
  h.omega_f = (float)h.omega;
  h.gx_f = (float)h.gx;
  h.gy_f = (float)h.gy;
  h.drho_in_f = (float)h.drho_in;
  h.drho_out_f = (float)h.drho_out;
  h.kT_f = (float)h.kT;
  h.pl_n_f = (float)h.pl_n;
  h.pl_K_f = (float)h.pl_K;
  h.tau_min_f = (float)h.tau_min;
  h.tau_max_f = (float)h.tau_max;
  // TRT: tau_m from the magic number (with the power law the device forms
  // it from the local tau*); BGK: tau_m = tau
  const bool trt = desc->collision == LB_TRT;
  h.magic = trt ? desc->magic : 0.0;
  h.tau_m = trt ? 0.5 + desc->magic / (h.tau - 0.5) : h.tau;
  h.omega_m = 1.0 / h.tau_m;
  h.magic_f = (float)h.magic;
  h.tau_m_f = (float)h.tau_m;
  h.omega_m_f = (float)h.omega_m;
  set_collision_coefficients(h);

  auto bail = [&](lb_status st) {
    (void)hipStreamDestroy(d->cap);
    delete d;
    return st;
  };
  Header zero{};
  if (hipMemcpyAsync(d->dhdr(), &zero, sizeof(zero), hipMemcpyHostToDevice, d->stream) != hipSuccess)
    return bail(fail(LB_EHIP, "header upload failed"));
  if ((s = push_desc(d)) != LB_OK) return bail(s);
  if (h.label) {
    d->host_labels.assign((size_t)desc->ny * L.pitch, 0);
    for (int y = 0; y < desc->ny; ++y)
      for (int x = 0; x < desc->nx; ++x) {
        const bool wall = (desc->bc_y == LB_WALL && (y == 0 || y == desc->ny - 1)) ||
                          (desc->bc_x == LB_WALL && (x == 0 || x == desc->nx - 1));
        d->host_labels[(size_t)y * L.pitch + x] = wall ? LBL_SOLID : LBL_FLUID;
      }
    if ((s = upload_labels(d)) != LB_OK) return bail(s);
  }
  // initial populations: equilibrium of the fields, then the step-0 collision
  if (desc->init_kind == LB_INIT_FIELDS) {
    double *st = (double *)(d->ws + L.stage);
    const size_t nxs = (size_t)desc->nx;
    for (int r0 = 0; r0 < desc->ny; r0 += L.band_rows) {
      const int nr = std::min(L.band_rows, desc->ny - r0);
      const size_t cnt = (size_t)nr * nxs;
      if (hipMemcpyAsync(st, desc->init_rho + (size_t)r0 * nxs, cnt * 8, hipMemcpyHostToDevice, d->stream) != hipSuccess ||
          hipMemcpyAsync(st + cnt, desc->init_ux + (size_t)r0 * nxs, cnt * 8, hipMemcpyHostToDevice, d->stream) != hipSuccess ||
          hipMemcpyAsync(st + 2 * cnt, desc->init_uy + (size_t)r0 * nxs, cnt * 8, hipMemcpyHostToDevice, d->stream) != hipSuccess)
        return bail(fail(LB_EHIP, "initial field upload failed"));
      ks.init(d->ddesc(), st, st + cnt, st + 2 * cnt, r0, nr, L.pitch, d->stream);
      if (hipStreamSynchronize(d->stream) != hipSuccess) return bail(fail(LB_EHIP, "init kernel failed"));
    }
  } else {
    ks.init(d->ddesc(), nullptr, nullptr, nullptr, 0, desc->ny, L.pitch, d->stream);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(d->stream) != hipSuccess)
    return bail(fail(LB_EHIP, "initialisation failed"));
  if ((s = refresh_mirrors(d)) != LB_OK) return bail(s);
  *out = d;
  return LB_OK;
}

lb_status lb_create_domain(const lb_domain_desc *desc, void *dev_workspace, size_t bytes,
                           void *hip_stream, lb_domain **out) {
  LB_GUARDED(lb_create_domain_impl(desc, dev_workspace, bytes, hip_stream, out));
}

static lb_status lb_set_obstacles_impl(lb_domain *d, const uint8_t *mask, size_t n) {
  if (!d || !mask) return fail(LB_EINVAL, "null argument");
  if (!d->desc.obstacles) return fail(LB_ESTATE, "domain was created without obstacles");
  if (d->np > 0) return fail(LB_ESTATE, "obstacles must be set before particles are added");
  if (d->in_batches) return fail(LB_ESTATE, "domain is in a batch");
  if (n != (size_t)d->desc.nx * d->desc.ny) return fail(LB_EINVAL, "mask size must be nx*ny");
  const int nx = d->desc.nx, ny = d->desc.ny, pitch = d->L.pitch;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const bool wall = (d->desc.bc_y == LB_WALL && (y == 0 || y == ny - 1)) ||
                        (d->desc.bc_x == LB_WALL && (x == 0 || x == nx - 1));
      d->host_labels[(size_t)y * pitch + x] = (wall || mask[(size_t)y * nx + x]) ? LBL_SOLID : LBL_FLUID;
    }
  return upload_labels(d);
}

lb_status lb_set_obstacles(lb_domain *d, const uint8_t *mask, size_t n) {
  LB_GUARDED(lb_set_obstacles_impl(d, mask, n));
}

namespace {

double mimg(double v, double len, bool per) { return per ? v - len * std::floor(v / len + 0.5) : v; }

// Validated device state of one particle description (Sec. 3: m = rho_p pi R^2,
// I = m R^2 / 2).
lb_status particle_state_of(const lb_domain *d, const lb_particle &q, PState *out) {
  const int nx = d->desc.nx, ny = d->desc.ny;
  const bool perx = d->desc.bc_x == LB_PERIODIC, pery = d->desc.bc_y == LB_PERIODIC;
  if (!(q.radius > 0.0) || !(q.density_ratio > 0.0) || !std::isfinite(q.x) || !std::isfinite(q.y) ||
      q.x < 0.0 || q.y < 0.0 || q.x >= nx || q.y >= ny)
    return fail(LB_EINVAL, "particle outside the domain or bad radius/density");
  if (!std::isfinite(q.ux) || !std::isfinite(q.uy) || !std::isfinite(q.omega))
    return fail(LB_EINVAL, "particle velocity not finite");
  // widest per-particle box of the kernels: link/repulsion scan, relabelling
  const int reach = std::max((int)std::ceil(q.radius + d->desc.lj_rit) + 1, (int)std::ceil(q.radius) + 3);
  const int W = 2 * reach + 2;
  if ((perx && W > nx) || (pery && W > ny)) return fail(LB_EINVAL, "particle box wider than a periodic axis");
  if (d->desc.bc_x == LB_PRESSURE && (q.x - reach < 1.0 || q.x + reach > nx - 2.0))
    return fail(LB_EINVAL, "particle box touches a pressure face");
  if ((2 * reach + 2) * (2 * reach + 2) * 8 > 6144 * 8) return fail(LB_EINVAL, "particle radius too large");
  PState s{};
  s.x = q.x; s.y = q.y; s.ux = q.ux; s.uy = q.uy; s.omega = q.omega;
  s.radius = q.radius;
  s.rho_ratio = q.density_ratio;
  const double rhop = q.density_ratio * d->desc.rho0;
  s.mass = rhop * M_PI * q.radius * q.radius;
  s.inertia = 0.5 * s.mass * q.radius * q.radius;
  s.flags = q.flags & LB_PARTICLE_FIXED;
  *out = s;
  return LB_OK;
}

// No node of particle k of `all` may be solid; with check_others, none may lie
// inside another particle of `all` either.
lb_status check_cover(const lb_domain *d, const std::vector<PState> &all, int k, bool check_others) {
  const int nx = d->desc.nx, ny = d->desc.ny, pitch = d->L.pitch;
  const bool perx = d->desc.bc_x == LB_PERIODIC, pery = d->desc.bc_y == LB_PERIODIC;
  const PState &s = all[k];
  const int r = (int)std::ceil(s.radius) + 1;
  for (int yy = (int)std::floor(s.y) - r; yy <= (int)std::floor(s.y) + r + 1; ++yy)
    for (int xx = (int)std::floor(s.x) - r; xx <= (int)std::floor(s.x) + r + 1; ++xx) {
      int x = xx, y = yy;
      if (x < 0 || x >= nx) { if (!perx) continue; x = (x + nx) % nx; }
      if (y < 0 || y >= ny) { if (!pery) continue; y = (y + ny) % ny; }
      const double dx = mimg(x - s.x, nx, perx), dy = mimg(y - s.y, ny, pery);
      if (!(dx * dx + dy * dy < s.radius * s.radius)) continue;
      if (d->host_labels[(size_t)y * pitch + x] == LBL_SOLID)
        return fail(LB_EINVAL, "particle covers a solid node");
      if (!check_others) continue;
      for (int q = 0; q < (int)all.size(); ++q) {
        if (q == k) continue;
        const double ex = mimg(x - all[q].x, nx, perx), ey = mimg(y - all[q].y, ny, pery);
        if (ex * ex + ey * ey < all[q].radius * all[q].radius)
          return fail(LB_EINVAL, "particle overlaps another particle");
      }
    }
  return LB_OK;
}

// Work items (one per particle), descriptor upload, labels of the current
// particle state; drops the step graphs (the launch sequence changes).
lb_status particles_changed(lb_domain *d) {
  d->hd.np = d->np;
  if (d->np > 0) {
    std::vector<PItem> items(d->np);
    for (int q = 0; q < d->np; ++q) items[q] = PItem{0, q};
    HIPCHK(hipMemcpyAsync(d->ditems(), items.data(), d->np * sizeof(PItem), hipMemcpyHostToDevice,
                          d->stream));
  }
  lb_status s = push_desc(d);
  if (s != LB_OK) return s;
  if (d->np > 0) {
    launch_relabel(d->ddesc(), d->ditems(), d->np, d->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(d->stream));
  }
  d->graphs.clear();
  return LB_OK;
}

}  // namespace

static lb_status lb_add_particles_impl(lb_domain *d, const lb_particle *p, int32_t n, int32_t *first_id) {
  if (!d || (!p && n > 0)) return fail(LB_EINVAL, "null argument");
  if (d->in_batches) return fail(LB_ESTATE, "domain is in a batch");
  if (n < 0 || d->np + n > d->desc.max_particles) return fail(LB_EINVAL, "exceeds max_particles");
  if (n == 0) {
    if (first_id) *first_id = d->np;
    return LB_OK;
  }
  // current particle states (they move on the device)
  std::vector<PState> cur(d->np + n);
  if (d->np > 0) {
    HIPCHK(hipMemcpyAsync(cur.data(), d->hd.pstate[d->t & 1], d->np * sizeof(PState),
                          hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
  }
  lb_status st;
  for (int k = 0; k < n; ++k)
    if ((st = particle_state_of(d, p[k], &cur[d->np + k])) != LB_OK) return st;
  // overlap: no node of a new disc may be solid or inside another particle
  for (int k = 0; k < n; ++k)
    if ((st = check_cover(d, cur, d->np + k, true)) != LB_OK) return st;
  const int first = d->np;
  HIPCHK(hipMemcpyAsync(d->hd.pstate[d->t & 1] + first, cur.data() + first, n * sizeof(PState),
                        hipMemcpyHostToDevice, d->stream));
  std::vector<PForce> zf(n);
  std::memset(zf.data(), 0, n * sizeof(PForce));
  HIPCHK(hipMemcpyAsync(d->hd.pforce + first, zf.data(), n * sizeof(PForce), hipMemcpyHostToDevice, d->stream));
  d->np += n;
  if ((st = particles_changed(d)) != LB_OK) return st;
  if (first_id) *first_id = first;
  return LB_OK;
}

lb_status lb_add_particles(lb_domain *d, const lb_particle *p, int32_t n, int32_t *first_id) {
  LB_GUARDED(lb_add_particles_impl(d, p, n, first_id));
}

static lb_status lb_get_particle_state_impl(lb_domain *d, lb_particle_state *out, int32_t n) {
  if (!d || (!out && n > 0)) return fail(LB_EINVAL, "null argument");
  if (n != d->np) return fail(LB_EINVAL, "n must equal the particle count");
  std::vector<PState> cur(std::max(n, 1));
  std::vector<PForce> frc(std::max(n, 1));
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(cur.data(), d->hd.pstate[d->t & 1], n * sizeof(PState),
                          hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipMemcpyAsync(frc.data(), d->hd.pforce, n * sizeof(PForce), hipMemcpyDeviceToHost,
                          d->stream));
  }
  HIPCHK(hipStreamSynchronize(d->stream));
  for (int k = 0; k < n; ++k) {
    const PState &s = cur[k];
    lb_particle_state &o = out[k];
    o.p.x = s.x; o.p.y = s.y; o.p.radius = s.radius; o.p.density_ratio = s.rho_ratio;
    o.p.ux = s.ux; o.p.uy = s.uy; o.p.omega = s.omega;
    o.p.fx = s.fx; o.p.fy = s.fy; o.p.torque = s.torque;
    o.p.flags = s.flags; o.p.reserved = 0;
    o.cover_fx = frc[k].cx_; o.cover_fy = frc[k].cy_; o.cover_torque = frc[k].ctorque;
  }
  return check_health(d);
}

lb_status lb_get_particle_state(lb_domain *d, lb_particle_state *out, int32_t n) {
  LB_GUARDED(lb_get_particle_state_impl(d, out, n));
}

static lb_status lb_set_particle_state_impl(lb_domain *d, const lb_particle_state *in, int32_t n) {
  if (!d || (!in && n > 0)) return fail(LB_EINVAL, "null argument");
  if (d->in_batches) return fail(LB_ESTATE, "domain is in a batch");
  if (n < 0 || n > d->desc.max_particles) return fail(LB_EINVAL, "exceeds max_particles");
  std::vector<PState> cur(n);
  std::vector<PForce> frc(n);
  lb_status st;
  for (int k = 0; k < n; ++k) {
    if ((st = particle_state_of(d, in[k].p, &cur[k])) != LB_OK) return st;
    if (!std::isfinite(in[k].p.fx) || !std::isfinite(in[k].p.fy) || !std::isfinite(in[k].p.torque) ||
        !std::isfinite(in[k].cover_fx) || !std::isfinite(in[k].cover_fy) ||
        !std::isfinite(in[k].cover_torque))
      return fail(LB_EINVAL, "particle force not finite");
    cur[k].fx = in[k].p.fx;
    cur[k].fy = in[k].p.fy;
    cur[k].torque = in[k].p.torque;
    std::memset(&frc[k], 0, sizeof(PForce));
    frc[k].cx_ = in[k].cover_fx;
    frc[k].cy_ = in[k].cover_fy;
    frc[k].ctorque = in[k].cover_torque;
  }
  for (int k = 0; k < n; ++k)
    if ((st = check_cover(d, cur, k, false)) != LB_OK) return st;
  if (d->hd.label) {
    // labels of walls and obstacles only; the new particles relabel below
    if ((st = upload_labels(d)) != LB_OK) return st;
  }
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(d->hd.pstate[d->t & 1], cur.data(), n * sizeof(PState),
                          hipMemcpyHostToDevice, d->stream));
    HIPCHK(hipMemcpyAsync(d->hd.pforce, frc.data(), n * sizeof(PForce), hipMemcpyHostToDevice,
                          d->stream));
  }
  d->np = n;
  return particles_changed(d);
}

lb_status lb_set_particle_state(lb_domain *d, const lb_particle_state *in, int32_t n) {
  LB_GUARDED(lb_set_particle_state_impl(d, in, n));
}

static lb_status lb_set_time_impl(lb_domain *d, int64_t t) {
  if (!d) return fail(LB_EINVAL, "null domain");
  if (t < 0) return fail(LB_EINVAL, "t < 0");
  if (d->in_batches) return fail(LB_ESTATE, "domain is in a batch");
  if ((t & 1) != (d->t & 1)) {
    // the state moves to the buffer of the new parity (populations, and the
    // particle state, double-buffered the same way)
    const size_t fbytes = (size_t)9 * d->desc.ny * d->L.pitch * storage_bytes(d->desc.storage);
    HIPCHK(hipMemcpyAsync(d->hd.f[t & 1], d->hd.f[d->t & 1], fbytes, hipMemcpyDeviceToDevice, d->stream));
    if (d->np > 0)
      HIPCHK(hipMemcpyAsync(d->hd.pstate[t & 1], d->hd.pstate[d->t & 1], d->np * sizeof(PState),
                            hipMemcpyDeviceToDevice, d->stream));
  }
  const uint64_t tt = (uint64_t)t;
  HIPCHK(hipMemcpyAsync(&d->dhdr()->tstep, &tt, sizeof(tt), hipMemcpyHostToDevice, d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  d->t = t;
  return refresh_mirrors(d);
}

lb_status lb_set_time(lb_domain *d, int64_t t) {
  LB_GUARDED(lb_set_time_impl(d, t));
}

static lb_status lb_step_impl(lb_domain *d, int64_t nsteps) {
  if (!d) return fail(LB_EINVAL, "null domain");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps < 0");
  if (nsteps > 0) {
    StepPlan p{&d->ks, d->ddesc(), d->dprefix(), d->dprefix2(), 1, d->ntiles(),
               d->ntiles2(), d->ditems(), d->np, two_step_ok(d)};
    p.rows2 = d->hd.rows2;
    p.fuse_pp = d->np == 1;
    if (d->overlap && d->np > 0 && !p.two) {
      if (!d->side) {
        HIPCHK(hipStreamCreateWithFlags(&d->side, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&d->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&d->ev_join, hipEventDisableTiming));
      }
      p.side = d->side;
      p.ev_fork = d->ev_fork;
      p.ev_join = d->ev_join;
      p.ntiles = d->ntiles();
    }
    lb_status s = run_steps(d->graphs, d->use_graph, d->chunk, d->stream, d->cap, p, nsteps);
    if (s != LB_OK) return s;
  }
  d->t += nsteps;
  if (check_due(d->t - nsteps, nsteps, d->mass_interval)) return domain_mass_enqueue(d);
  return LB_OK;
}

lb_status lb_step(lb_domain *d, int64_t nsteps) {
  LB_GUARDED(lb_step_impl(d, nsteps));
}

static lb_status lb_moments_device_impl(lb_domain *d, double *rho, double *ux, double *uy) {
  if (!d || !rho || !ux || !uy) return fail(LB_EINVAL, "null argument");
  d->ks.moments(d->ddesc(), rho, ux, uy, 0, d->desc.ny, d->desc.nx, d->stream);
  HIPCHK(hipGetLastError());
  return LB_OK;
}

lb_status lb_moments_device(lb_domain *d, double *rho, double *ux, double *uy) {
  LB_GUARDED(lb_moments_device_impl(d, rho, ux, uy));
}

static lb_status lb_moments_async_impl(lb_domain *d, double *dev_stage, double *rho, double *ux, double *uy,
                                       void *copy_stream) {
  if (!d || !dev_stage || !rho || !ux || !uy) return fail(LB_EINVAL, "null argument");
  hipStream_t cs = (hipStream_t)copy_stream;
  if (cs == d->stream) return fail(LB_EINVAL, "the copy stream must differ from the domain's stream");
  if (!d->rep_ready) {
    HIPCHK(hipEventCreateWithFlags(&d->rep_ready, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&d->rep_copied, hipEventDisableTiming));
  }
  const int nx = d->desc.nx, ny = d->desc.ny;
  const size_t cnt = (size_t)nx * ny;
  // the staging memory of an earlier call may still be being copied out
  if (d->rep_pending) HIPCHK(hipStreamWaitEvent(d->stream, d->rep_copied, 0));
  d->ks.moments(d->ddesc(), dev_stage, dev_stage + cnt, dev_stage + 2 * cnt, 0, ny, nx, d->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(d->rep_ready, d->stream));
  HIPCHK(hipStreamWaitEvent(cs, d->rep_ready, 0));
  HIPCHK(hipMemcpyAsync(rho, dev_stage, cnt * 8, hipMemcpyDeviceToHost, cs));
  HIPCHK(hipMemcpyAsync(ux, dev_stage + cnt, cnt * 8, hipMemcpyDeviceToHost, cs));
  HIPCHK(hipMemcpyAsync(uy, dev_stage + 2 * cnt, cnt * 8, hipMemcpyDeviceToHost, cs));
  HIPCHK(hipEventRecord(d->rep_copied, cs));
  d->rep_pending = true;
  return LB_OK;
}

lb_status lb_moments_async(lb_domain *d, double *dev_stage, double *rho, double *ux, double *uy,
                           void *copy_stream) {
  LB_GUARDED(lb_moments_async_impl(d, dev_stage, rho, ux, uy, copy_stream));
}

static lb_status lb_moments_wait_impl(lb_domain *d) {
  if (!d) return fail(LB_EINVAL, "null domain");
  if (d->rep_pending) {
    HIPCHK(hipEventSynchronize(d->rep_copied));
    d->rep_pending = false;
  }
  return LB_OK;
}

lb_status lb_moments_wait(lb_domain *d) {
  LB_GUARDED(lb_moments_wait_impl(d));
}

static lb_status lb_moments_impl(lb_domain *d, double *rho, double *ux, double *uy) {
  if (!d || !rho || !ux || !uy) return fail(LB_EINVAL, "null argument");
  const int nx = d->desc.nx;
  double *st = (double *)(d->ws + d->L.stage);
  for (int r0 = 0; r0 < d->desc.ny; r0 += d->L.band_rows) {
    const int nr = std::min(d->L.band_rows, d->desc.ny - r0);
    const size_t cnt = (size_t)nr * nx;
    d->ks.moments(d->ddesc(), st, st + cnt, st + 2 * cnt, r0, nr, nx, d->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(rho + (size_t)r0 * nx, st, cnt * 8, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipMemcpyAsync(ux + (size_t)r0 * nx, st + cnt, cnt * 8, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipMemcpyAsync(uy + (size_t)r0 * nx, st + 2 * cnt, cnt * 8, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
  }
  return check_health(d);
}

lb_status lb_moments(lb_domain *d, double *rho, double *ux, double *uy) {
  LB_GUARDED(lb_moments_impl(d, rho, ux, uy));
}

static lb_status lb_get_particles_impl(lb_domain *d, lb_particle *out, int32_t n) {
  if (!d || (!out && n > 0)) return fail(LB_EINVAL, "null argument");
  if (n < 0 || n > d->np) return fail(LB_EINVAL, "n exceeds the particle count");
  std::vector<PState> cur(std::max(n, 1));
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(cur.data(), d->hd.pstate[d->t & 1], n * sizeof(PState),
                          hipMemcpyDeviceToHost, d->stream));
  }
  HIPCHK(hipStreamSynchronize(d->stream));
  for (int k = 0; k < n; ++k) {
    const PState &s = cur[k];
    lb_particle &q = out[k];
    q.x = s.x; q.y = s.y; q.radius = s.radius; q.density_ratio = s.rho_ratio;
    q.ux = s.ux; q.uy = s.uy; q.omega = s.omega;
    q.fx = s.fx; q.fy = s.fy; q.torque = s.torque;
    q.flags = s.flags; q.reserved = 0;
  }
  return check_health(d);
}

lb_status lb_get_particles(lb_domain *d, lb_particle *out, int32_t n) {
  LB_GUARDED(lb_get_particles_impl(d, out, n));
}

static lb_status lb_mass_impl(lb_domain *d, double *total) {
  if (!d || !total) return fail(LB_EINVAL, "null argument");
  lb_status s = domain_mass_enqueue(d);
  if (s != LB_OK) return s;
  HIPCHK(hipMemcpyAsync(total, &d->dhdr()->mass, sizeof(double), hipMemcpyDeviceToHost, d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  return check_health(d);
}

lb_status lb_mass(lb_domain *d, double *total) {
  LB_GUARDED(lb_mass_impl(d, total));
}

// Partial sums of lb_mass_static: one fixed array per GPU, for callers that
// cannot allocate.  Its host-side name is not a device address: kernels get
// the address hipGetSymbolAddress returns for each device (kept per device).
constexpr int STATIC_MASS_PARTIALS = NPARTIALS;
static __device__ __align__(256) double scratch[STATIC_MASS_PARTIALS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

// scratch's address on device dev (resolved once per device, dev current)
lb_status scratch_on(int dev, double **out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LB_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev) HIPCHK(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) HIPCHK(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      return fail(LB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = (double *)p;
  }
  *out = g_scratch[dev];
  return LB_OK;
}
}  // namespace

static lb_status lb_mass_static_impl(lb_domain *d, double *dev_total) {
  if (!d || !dev_total) return fail(LB_EINVAL, "null argument");
  if (d->hd.mass_blocks > STATIC_MASS_PARTIALS)
    return fail(LB_EINVAL, "density sum needs more partial sums than the static array holds (" +
                               std::to_string(STATIC_MASS_PARTIALS) + ")");
  double *part = nullptr;
  lb_status s = scratch_on(d->device, &part);
  if (s != LB_OK) return s;
  d->ks.mass_partial(d->ddesc(), d->dprefixm(), 1, d->hd.mass_blocks, part, d->stream);
  launch_mass_final(d->ddesc(), 1, part, dev_total, d->stream);
  HIPCHK(hipGetLastError());
  return LB_OK;
}

lb_status lb_mass_static(lb_domain *d, double *dev_total) {
  LB_GUARDED(lb_mass_static_impl(d, dev_total));
}

static lb_status lb_set_mass_check_impl(lb_domain *d, double rel_tol) {
  if (!d) return fail(LB_EINVAL, "null domain");
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return fail(LB_EINVAL, "rel_tol must be finite and >= 0");
  double ref = 0.0;
  lb_status s = lb_mass(d, &ref);
  if (s != LB_OK) return s;
  const double ctl[2] = {ref, rel_tol};
  HIPCHK(hipMemcpyAsync(d->dhdr()->mass_ctl, ctl, sizeof(ctl), hipMemcpyHostToDevice, d->stream));
  HIPCHK(hipStreamSynchronize(d->stream));
  return LB_OK;
}

lb_status lb_set_mass_check(lb_domain *d, double rel_tol) {
  LB_GUARDED(lb_set_mass_check_impl(d, rel_tol));
}

static lb_status lb_time_impl(lb_domain *d, int64_t *t) {
  if (!d || !t) return fail(LB_EINVAL, "null argument");
  *t = d->t;
  return LB_OK;
}

lb_status lb_time(lb_domain *d, int64_t *t) {
  LB_GUARDED(lb_time_impl(d, t));
}

static lb_status lb_get_populations_impl(lb_domain *d, double *hf) {
  if (!d || !hf) return fail(LB_EINVAL, "null argument");
  const int nx = d->desc.nx, ny = d->desc.ny;
  double *st = (double *)(d->ws + d->L.stage);
  for (int r0 = 0; r0 < ny; r0 += d->L.band_rows) {
    const int nr = std::min(d->L.band_rows, ny - r0);
    const size_t cnt = (size_t)nr * nx;
    d->ks.export_f(d->ddesc(), st, r0, nr, nx, d->stream);
    HIPCHK(hipGetLastError());
    for (int i = 0; i < 9; ++i)
      HIPCHK(hipMemcpyAsync(hf + ((size_t)i * ny + r0) * nx, st + i * cnt, cnt * 8,
                            hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
  }
  return check_health(d);
}

lb_status lb_get_populations(lb_domain *d, double *hf) {
  LB_GUARDED(lb_get_populations_impl(d, hf));
}

static lb_status lb_set_populations_impl(lb_domain *d, const double *hf) {
  if (!d || !hf) return fail(LB_EINVAL, "null argument");
  const int nx = d->desc.nx, ny = d->desc.ny;
  double *st = (double *)(d->ws + d->L.stage);
  for (int r0 = 0; r0 < ny; r0 += d->L.band_rows) {
    const int nr = std::min(d->L.band_rows, ny - r0);
    const size_t cnt = (size_t)nr * nx;
    for (int i = 0; i < 9; ++i)
      HIPCHK(hipMemcpyAsync(st + i * cnt, hf + ((size_t)i * ny + r0) * nx, cnt * 8,
                            hipMemcpyHostToDevice, d->stream));
    d->ks.import_f(d->ddesc(), st, r0, nr, nx, d->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(d->stream));
  }
  return refresh_mirrors(d);
}

lb_status lb_set_populations(lb_domain *d, const double *hf) {
  LB_GUARDED(lb_set_populations_impl(d, hf));
}

static lb_status lb_set_option_impl(lb_domain *d, int32_t key, int64_t value) {
  if (!d) return fail(LB_EINVAL, "null domain");
  if (d->in_batches && (key == LB_OPT_TILE_WIDTH || key == LB_OPT_ROWS_PER_THREAD ||
                        key == LB_OPT_FORCE_AVERAGE || key == LB_OPT_TWO_STEP ||
                        key == LB_OPT_TWO_STEP_ROWS))
    return fail(LB_ESTATE, "tile, force and two-step options are fixed while the domain is in a batch");
  switch (key) {
    case LB_OPT_USE_GRAPH: d->use_graph = value != 0; break;
    case LB_OPT_TILE_WIDTH:
      if (value != 64 && value != 128 && value != 256) return fail(LB_EINVAL, "tile width must be 64, 128 or 256");
      set_tiles(d->hd, (int)value, d->hd.rows_per_thread);
      break;
    case LB_OPT_ROWS_PER_THREAD:
      if (value < 1 || value > 16) return fail(LB_EINVAL, "rows per thread must be in [1, 16]");
      set_tiles(d->hd, d->hd.tile_w, (int)value);
      break;
    case LB_OPT_GRAPH_CHUNK:
      if (value < 1 || value > 4096) return fail(LB_EINVAL, "graph chunk must be in [1, 4096]");
      d->chunk = (int)value;
      break;
    case LB_OPT_FORCE_AVERAGE:
      if (value != 0 && value != 1) return fail(LB_EINVAL, "force averaging is 0 or 1");
      d->hd.feat = value ? (d->hd.feat | F_FAVG) : (d->hd.feat & ~F_FAVG);
      break;
    case LB_OPT_TWO_STEP:
      if (value != 0 && value != 1) return fail(LB_EINVAL, "two-step sweep is 0 or 1");
      d->two_step = value != 0;
      break;
    case LB_OPT_OVERLAP:
      if (value != 0 && value != 1) return fail(LB_EINVAL, "overlap is 0 or 1");
      d->overlap = value != 0;
      break;
    case LB_OPT_TWO_STEP_ROWS:
      if (!valid_two_step_rows(d->desc.storage, value))
        return fail(LB_EINVAL, "two-step tile rows: not an instantiated height for this storage");
      set_two_step_rows(d->hd, (int)value);
      break;
    case LB_OPT_MASS_INTERVAL:
      if (value < 1) return fail(LB_EINVAL, "mass check interval must be >= 1");
      d->mass_interval = value;
      return LB_OK;  // no effect on the captured graphs
    default: return fail(LB_EINVAL, "unknown option");
  }
  d->graphs.clear();
  if (key == LB_OPT_TILE_WIDTH || key == LB_OPT_ROWS_PER_THREAD || key == LB_OPT_FORCE_AVERAGE ||
      key == LB_OPT_TWO_STEP_ROWS)
    return push_desc(d);
  return LB_OK;
}

lb_status lb_set_option(lb_domain *d, int32_t key, int64_t value) {
  LB_GUARDED(lb_set_option_impl(d, key, value));
}

static lb_status lb_get_option_impl(lb_domain *d, int32_t key, int64_t *value) {
  if (!d || !value) return fail(LB_EINVAL, "null argument");
  switch (key) {
    case LB_OPT_USE_GRAPH: *value = d->use_graph; return LB_OK;
    case LB_OPT_TILE_WIDTH: *value = d->hd.tile_w; return LB_OK;
    case LB_OPT_ROWS_PER_THREAD: *value = d->hd.rows_per_thread; return LB_OK;
    case LB_OPT_GRAPH_CHUNK: *value = d->chunk; return LB_OK;
    case LB_OPT_FORCE_AVERAGE: *value = (d->hd.feat & F_FAVG) ? 1 : 0; return LB_OK;
    case LB_OPT_TWO_STEP: *value = d->two_step ? 1 : 0; return LB_OK;
    case LB_OPT_OVERLAP: *value = d->overlap ? 1 : 0; return LB_OK;
    case LB_OPT_TWO_STEP_ROWS: *value = d->hd.rows2; return LB_OK;
    case LB_OPT_MASS_INTERVAL: *value = d->mass_interval; return LB_OK;
  }
  return fail(LB_EINVAL, "unknown option");
}

lb_status lb_get_option(lb_domain *d, int32_t key, int64_t *value) {
  LB_GUARDED(lb_get_option_impl(d, key, value));
}

static lb_status lb_autotune_impl(lb_domain *d, int32_t steps, double *best_ms) {
  if (!d || steps < 1) return fail(LB_EINVAL, "bad argument");
  if (d->in_batches) return fail(LB_ESTATE, "domain is in a batch");
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int widths[3] = {64, 128, 256};
  const int rows[3] = {2, 4, 8};  // multiples of the rows every thread loads at once
  double best = 1e300;
  int bw = d->hd.tile_w, br = d->hd.rows_per_thread;
  const int saved_chunk = d->chunk;
  const bool saved_two = d->two_step;
  d->chunk = std::max(1, std::min(steps, 4096));
  d->two_step = false;  // the shapes tuned are the single-step sweep's
  d->graphs.clear();
  lb_status s = LB_OK;
  for (int w : widths) {
    if (w > 64 && w / 2 >= d->desc.nx) continue;
    for (int r : rows) {
      if ((s = lb_set_option(d, LB_OPT_TILE_WIDTH, w)) != LB_OK) break;
      if ((s = lb_set_option(d, LB_OPT_ROWS_PER_THREAD, r)) != LB_OK) break;
      if ((s = lb_step(d, steps)) != LB_OK) break;  // warm-up (and graph capture)
      if (hipEventRecord(e0, d->stream) != hipSuccess) { s = fail(LB_EHIP, "event"); break; }
      if ((s = lb_step(d, steps)) != LB_OK) break;
      if (hipEventRecord(e1, d->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        s = fail(LB_EHIP, "event");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms / steps < best) { best = ms / steps; bw = w; br = r; }
    }
    if (s != LB_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  d->chunk = saved_chunk;
  d->two_step = saved_two;
  d->graphs.clear();
  if (s != LB_OK) return s;
  if ((s = lb_set_option(d, LB_OPT_TILE_WIDTH, bw)) != LB_OK) return s;
  if ((s = lb_set_option(d, LB_OPT_ROWS_PER_THREAD, br)) != LB_OK) return s;
  if (two_step_ok(d)) {
    // the two-step sweep's tile height: cached for the class, else timed
    const auto key = tune_key(d->desc.storage, d->feat, (long long)d->desc.nx * d->desc.ny);
    int rows = 0;
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      auto it = g_rows2_cache.find(key);
      if (it != g_rows2_cache.end()) rows = it->second;
    }
    if (rows == 0) {
      double best2 = 1e300;
      const int n4 = std::max(4, (steps + 3) / 4 * 4);
      for (int k = 0; k < 3 && s == LB_OK; ++k) {
        const int h = two_step_rows_of(d->desc.storage, k);
        double ms = 0.0;
        if ((s = lb_set_option(d, LB_OPT_TWO_STEP_ROWS, h)) != LB_OK) break;
        if ((s = time_steps([&](int64_t n) { return lb_step(d, n); }, d->stream, n4, &ms)) != LB_OK)
          break;
        if (ms < best2) { best2 = ms; rows = h; }
      }
      if (s != LB_OK) return s;
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_rows2_cache[key] = rows;
      best = std::min(best, best2);
    }
    if ((s = lb_set_option(d, LB_OPT_TWO_STEP_ROWS, rows)) != LB_OK) return s;
  }
  if (best_ms) *best_ms = best;
  return check_health(d);
}

lb_status lb_autotune(lb_domain *d, int32_t steps, double *best_ms) {
  LB_GUARDED(lb_autotune_impl(d, steps, best_ms));
}

static lb_status lb_batch_autotune_impl(lb_batch *b, int32_t steps, double *best_ms) {
  if (!b || steps < 1) return fail(LB_EINVAL, "bad argument");
  if (best_ms) *best_ms = 0.0;
  if (!b->two_step) return LB_OK;  // single steps: the members' own tiles
  long long sites = 0;
  int feat = 0;
  for (auto *d : b->doms) {
    sites += (long long)d->desc.nx * d->desc.ny;
    feat |= d->feat;
  }
  const auto key = tune_key(b->doms[0]->desc.storage, feat, sites);
  int rows = 0;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_rows2_cache.find(key);
    if (it != g_rows2_cache.end()) rows = it->second;
  }
  lb_status s = LB_OK;
  if (rows == 0) {
    double best = 1e300;
    const int n4 = std::max(4, (steps + 3) / 4 * 4);
    for (int k = 0; k < 3; ++k) {
      const int h = two_step_rows_of(b->doms[0]->desc.storage, k);
      double ms = 0.0;
      if ((s = lb_batch_set_option(b, LB_OPT_TWO_STEP_ROWS, h)) != LB_OK) return s;
      if ((s = time_steps([&](int64_t n) { return lb_batch_step(b, n); }, b->stream, n4, &ms)) != LB_OK)
        return s;
      if (ms < best) { best = ms; rows = h; }
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_rows2_cache[key] = rows;
    if (best_ms) *best_ms = best;
  }
  return lb_batch_set_option(b, LB_OPT_TWO_STEP_ROWS, rows);
}

lb_status lb_batch_autotune(lb_batch *b, int32_t steps, double *best_ms) {
  LB_GUARDED(lb_batch_autotune_impl(b, steps, best_ms));
}

static lb_status lb_destroy_domain_impl(lb_domain *d) {
  if (!d) return fail(LB_EINVAL, "null domain");
  if (d->in_batches) return fail(LB_ESTATE, "destroy the batches that hold this domain first");
  (void)hipStreamSynchronize(d->stream);
  if (d->rep_ready) {
    (void)hipEventSynchronize(d->rep_copied);
    (void)hipEventDestroy(d->rep_ready);
    (void)hipEventDestroy(d->rep_copied);
  }
  if (d->side) {
    (void)hipStreamSynchronize(d->side);
    (void)hipEventDestroy(d->ev_fork);
    (void)hipEventDestroy(d->ev_join);
    (void)hipStreamDestroy(d->side);
  }
  d->graphs.clear();
  (void)hipStreamDestroy(d->cap);
  delete d;
  return LB_OK;
}

lb_status lb_destroy_domain(lb_domain *d) {
  LB_GUARDED(lb_destroy_domain_impl(d));
}

static lb_status lb_batch_workspace_bytes_impl(lb_domain *const *domains, int32_t n, size_t *bytes) {
  if (!domains || n < 1 || !bytes) return fail(LB_EINVAL, "bad argument");
  size_t items = 0;
  for (int i = 0; i < n; ++i) {
    if (!domains[i]) return fail(LB_EINVAL, "null domain");
    items += domains[i]->np;
  }
  *bytes = align256((size_t)n * sizeof(DevDomain)) + align256((size_t)3 * (n + 1) * sizeof(int)) +
           align256(std::max<size_t>(items, 1) * sizeof(PItem));
  return LB_OK;
}

lb_status lb_batch_workspace_bytes(lb_domain *const *domains, int32_t n, size_t *bytes) {
  LB_GUARDED(lb_batch_workspace_bytes_impl(domains, n, bytes));
}

static lb_status lb_batch_create_impl(lb_domain *const *domains, int32_t n, void *dev_workspace, size_t bytes,
                                      void *hip_stream, lb_batch **out) {
  if (!out) return fail(LB_EINVAL, "out is null");
  *out = nullptr;
  size_t need = 0;
  lb_status s = lb_batch_workspace_bytes(domains, n, &need);
  if (s != LB_OK) return s;
  if (!dev_workspace || ((uintptr_t)dev_workspace & 255)) return fail(LB_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < need) return fail(LB_ENOMEM, "batch workspace too small");
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < i; ++j)
      if (domains[i] == domains[j]) return fail(LB_EINVAL, "a domain appears twice");
    if (domains[i]->desc.storage != domains[0]->desc.storage ||
        domains[i]->desc.compute != domains[0]->desc.compute ||
        (domains[i]->feat & (F_NOISE | F_POWER)) != (domains[0]->feat & (F_NOISE | F_POWER)) ||
        domains[i]->plm != domains[0]->plm)
      return fail(LB_EUNSUPPORTED, "batched domains must share storage, arithmetic, noise and power law");
  }
  // label-plane and label-free domains share one launch: take the kernel set
  // with label support if any domain has a plane (it reads no labels for the
  // others)
  int lab_dom = -1;
  for (int i = 0; i < n; ++i)
    if (domains[i]->feat & F_LABELS) lab_dom = i;
  lb_batch *b = new lb_batch();
  b->doms.assign(domains, domains + n);
  b->ws = (char *)dev_workspace;
  b->stream = (hipStream_t)hip_stream;
  b->ks = domains[lab_dom >= 0 ? lab_dom : 0]->ks;
  b->off_desc = 0;
  b->off_prefix = align256((size_t)n * sizeof(DevDomain));
  b->off_items = b->off_prefix + align256((size_t)3 * (n + 1) * sizeof(int));
  b->bytes = need;
  std::vector<DevDomain> descs(n);
  // single-step tile prefix [0, n], the two-step one [n + 1, 2n + 1], the
  // density-sum blocks [2n + 2, 3n + 2]
  std::vector<int> prefix(3 * (n + 1), 0);
  std::vector<PItem> items;
  bool two = b->ks.sweep2 != nullptr;
  for (int i = 0; i < n; ++i) {
    descs[i] = domains[i]->hd;
    prefix[i + 1] = prefix[i] + domains[i]->ntiles();
    prefix[n + 2 + i] = prefix[n + 1 + i] + domains[i]->ntiles2();
    prefix[2 * n + 3 + i] = prefix[2 * n + 2 + i] + domains[i]->hd.mass_blocks;
    for (int q = 0; q < domains[i]->np; ++q) items.push_back(PItem{i, q});
    two = two && two_step_ok(domains[i]);
  }
  // one tile height per launch: the members' own if they agree, else the
  // storage format's default (the batch's descriptor copies carry it)
  int rows2 = domains[0]->hd.rows2;
  for (int i = 1; i < n; ++i)
    if (domains[i]->hd.rows2 != rows2) rows2 = two_step_rows(domains[0]->desc.storage);
  for (int i = 0; i < n; ++i) set_two_step_rows(descs[i], rows2);
  for (int i = 0; i < n; ++i)
    prefix[n + 2 + i] = prefix[n + 1 + i] + descs[i].tiles2_x * descs[i].tiles2_y;
  b->rows2 = rows2;
  b->two_step = two;
  b->total_tiles2 = prefix[2 * n + 1];
  b->total_mass_blocks = prefix[3 * n + 2];
  size_t working_set = 0;
  for (int i = 0; i < n; ++i) working_set += sweep_working_set(descs[i]);
  for (int i = 0; i < n; ++i) descs[i].stream_stores = working_set >= STREAM_STORE_MIN_BYTES;
  b->total_tiles = prefix[n];
  b->nitems = (int)items.size();
  b->hdescs = descs;
  b->hprefix = prefix;
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(LB_EHIP, "hipStreamCreateWithFlags failed");
  }
  bool ok = hipMemcpyAsync(b->ddesc(), descs.data(), n * sizeof(DevDomain), hipMemcpyHostToDevice, b->stream) == hipSuccess &&
            hipMemcpyAsync(b->dprefix(), prefix.data(), prefix.size() * sizeof(int), hipMemcpyHostToDevice, b->stream) == hipSuccess &&
            (items.empty() || hipMemcpyAsync(b->ditems(), items.data(), items.size() * sizeof(PItem), hipMemcpyHostToDevice, b->stream) == hipSuccess) &&
            hipStreamSynchronize(b->stream) == hipSuccess;
  if (!ok) {
    (void)hipStreamDestroy(b->cap);
    delete b;
    return fail(LB_EHIP, "batch upload failed");
  }
  for (auto *d : b->doms) {
    (void)hipStreamSynchronize(d->stream);
    d->in_batches += 1;
  }
  *out = b;
  return LB_OK;
}

lb_status lb_batch_create(lb_domain *const *domains, int32_t n, void *dev_workspace, size_t bytes,
                          void *hip_stream, lb_batch **out) {
  LB_GUARDED(lb_batch_create_impl(domains, n, dev_workspace, bytes, hip_stream, out));
}

static lb_status lb_batch_step_impl(lb_batch *b, int64_t nsteps) {
  if (!b) return fail(LB_EINVAL, "null batch");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps < 0");
  if (nsteps > 0) {
    StepPlan p{&b->ks, b->ddesc(), b->dprefix(), b->dprefix2(), (int)b->doms.size(),
               b->total_tiles, b->total_tiles2, b->ditems(), b->nitems, b->two_step};
    p.rows2 = b->rows2;
    p.fuse_pp = true;
    for (auto *m : b->doms) p.fuse_pp = p.fuse_pp && m->np <= 1;
    lb_status s = run_steps(b->graphs, b->use_graph, b->chunk, b->stream, b->cap, p, nsteps);
    if (s != LB_OK) return s;
  }
  for (auto *d : b->doms) d->t += nsteps;
  b->t += nsteps;
  if (check_due(b->t - nsteps, nsteps, b->mass_interval)) {
    // the FP64 density sums of every domain: two launches for the batch
    b->ks.mass_partial(b->ddesc(), b->dprefixm(), (int)b->doms.size(), b->total_mass_blocks,
                       nullptr, b->stream);
    launch_mass_final(b->ddesc(), (int)b->doms.size(), nullptr, nullptr, b->stream);
    HIPCHK(hipGetLastError());
  }
  return LB_OK;
}

lb_status lb_batch_step(lb_batch *b, int64_t nsteps) {
  LB_GUARDED(lb_batch_step_impl(b, nsteps));
}

static lb_status lb_batch_set_option_impl(lb_batch *b, int32_t key, int64_t value) {
  if (!b) return fail(LB_EINVAL, "null batch");
  switch (key) {
    case LB_OPT_USE_GRAPH: b->use_graph = value != 0; break;
    case LB_OPT_GRAPH_CHUNK:
      if (value < 1 || value > 4096) return fail(LB_EINVAL, "graph chunk must be in [1, 4096]");
      b->chunk = (int)value;
      break;
    case LB_OPT_MASS_INTERVAL:
      if (value < 1) return fail(LB_EINVAL, "mass check interval must be >= 1");
      b->mass_interval = value;
      return LB_OK;
    case LB_OPT_TWO_STEP_ROWS: {
      if (!valid_two_step_rows(b->doms[0]->desc.storage, value))
        return fail(LB_EINVAL, "two-step tile rows: not an instantiated height for this storage");
      const int n = (int)b->doms.size();
      b->rows2 = (int)value;
      for (int i = 0; i < n; ++i) {
        set_two_step_rows(b->hdescs[i], b->rows2);
        b->hprefix[n + 2 + i] = b->hprefix[n + 1 + i] + b->hdescs[i].tiles2_x * b->hdescs[i].tiles2_y;
      }
      b->total_tiles2 = b->hprefix[2 * n + 1];
      HIPCHK(hipMemcpyAsync(b->ddesc(), b->hdescs.data(), n * sizeof(DevDomain),
                            hipMemcpyHostToDevice, b->stream));
      HIPCHK(hipMemcpyAsync(b->dprefix(), b->hprefix.data(), b->hprefix.size() * sizeof(int),
                            hipMemcpyHostToDevice, b->stream));
      HIPCHK(hipStreamSynchronize(b->stream));
      break;
    }
    default: return fail(LB_EINVAL, "option not available on a batch");
  }
  b->graphs.clear();
  return LB_OK;
}

lb_status lb_batch_set_option(lb_batch *b, int32_t key, int64_t value) {
  LB_GUARDED(lb_batch_set_option_impl(b, key, value));
}

static lb_status lb_batch_get_option_impl(lb_batch *b, int32_t key, int64_t *value) {
  if (!b || !value) return fail(LB_EINVAL, "null argument");
  switch (key) {
    case LB_OPT_USE_GRAPH: *value = b->use_graph ? 1 : 0; return LB_OK;
    case LB_OPT_GRAPH_CHUNK: *value = b->chunk; return LB_OK;
    case LB_OPT_MASS_INTERVAL: *value = b->mass_interval; return LB_OK;
    case LB_OPT_TWO_STEP_ROWS: *value = b->rows2; return LB_OK;
  }
  return fail(LB_EINVAL, "option not available on a batch");
}

lb_status lb_batch_get_option(lb_batch *b, int32_t key, int64_t *value) {
  LB_GUARDED(lb_batch_get_option_impl(b, key, value));
}

static lb_status lb_batch_destroy_impl(lb_batch *b) {
  if (!b) return fail(LB_EINVAL, "null batch");
  (void)hipStreamSynchronize(b->stream);
  b->graphs.clear();
  (void)hipStreamDestroy(b->cap);
  for (auto *d : b->doms) d->in_batches -= 1;
  delete b;
  return LB_OK;
}

lb_status lb_batch_destroy(lb_batch *b) {
  LB_GUARDED(lb_batch_destroy_impl(b));
}

static lb_status lb_noise_normals_impl(uint64_t seed, uint32_t domain_id, uint32_t step, uint32_t node0,
                                       uint32_t count, int32_t fp32_arithmetic, float *dev_out,
                                       void *hip_stream) {
  if (!dev_out && count > 0) return fail(LB_EINVAL, "null output");
  if (fp32_arithmetic != 0 && fp32_arithmetic != 1) return fail(LB_EINVAL, "fp32_arithmetic must be 0 or 1");
  if (count > (1u << 28)) return fail(LB_EINVAL, "count above 2^28");
  if (count == 0) return LB_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  launch_normals((uint32_t)seed, (uint32_t)(seed >> 32) ^ domain_id, step, node0, count,
                 fp32_arithmetic == 1, dev_out, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return LB_OK;
}

lb_status lb_noise_normals(uint64_t seed, uint32_t domain_id, uint32_t step, uint32_t node0,
                           uint32_t count, int32_t fp32_arithmetic, float *dev_out,
                           void *hip_stream) {
  LB_GUARDED(lb_noise_normals_impl(seed, domain_id, step, node0, count, fp32_arithmetic, dev_out, hip_stream));
}

}  // extern "C"
