// C ABI of libhwcount.so (declared in include/hwcount.h).
//
// A context owns a HIP stream, a cache of built fields, a cache of device
// plans (one per (q, g, sweep mode): the LDS image of all level tables plus
// the x lists), scratch buffers and captured HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>
#include <unordered_map>
#include <cmath>

#include "../../include/hwcount.h"
#include "field.h"
#include "plan.h"

namespace hwc {
hipError_t launch_count(const PlanDesc& P, const PlanDesc* dP, int coeff_bytes, const void* codes, const uint32_t* perm,
                        const uint64_t* tiles, const uint32_t* ntiles, uint32_t* queue, uint32_t lo, uint32_t hi,
                        int32_t* outN, uint32_t* outLv, uint32_t plog, uint32_t* acc, uint32_t* done, uint32_t grid,
                        uint32_t block, uint32_t wpe, hipStream_t s);
hipError_t occupancy_count(uint32_t g, int coeff_bytes, uint32_t block, uint32_t lds_bytes, uint32_t wpe,
                           int* blocks_per_cu);
hipError_t prepare_kernels();
hipError_t prepare_vcount();
hipError_t occupancy_vcount(uint32_t g, uint32_t block, uint32_t lds_bytes, int* blocks_per_cu);
hipError_t launch_vcount(const VPlanDesc& V, const VPlanDesc* dV, int coeff_bytes, const void* codes, uint64_t n,
                         uint32_t lvl_lo, uint32_t lvl_hi, uint32_t tw, bool acc, int32_t* outN, uint32_t* outLv,
                         uint32_t* err, uint32_t grid, uint32_t block, hipStream_t s);
hipError_t launch_assemble(const PlanDesc& P, int coeff_bytes, const void* codes, uint64_t n, const uint32_t* lv,
                           int32_t* outN, hipStream_t s);
hipError_t launch_fill(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t launch_shift(int coeff_bytes, uint32_t g, const void* in, uint64_t n, uint32_t q, const uint32_t* step,
                        void* out, uint16_t* pid, uint32_t* counts, uint32_t* err, hipStream_t s);
hipError_t launch_bucket(int coeff_bytes, const void* codes, uint64_t n, uint32_t q, uint32_t g, uint16_t* pid,
                         uint32_t* counts, uint32_t* err, uint32_t* bucket_start, uint32_t* tile_start,
                         uint32_t* cursor, uint32_t* ntiles, uint32_t* queue, uint64_t* tiles, uint32_t* perm,
                         uint64_t max_tiles, bool classified, hipStream_t s);
hipError_t launch_batch(const JobDesc* jobs, uint32_t njobs, uint32_t gmax, uint32_t lds_bytes, uint32_t grid,
                        uint32_t block, hipStream_t s);
hipError_t occupancy_batch(uint32_t gmax, uint32_t block, uint32_t lds_bytes, int* blocks_per_cu);
uint64_t hist_scratch_bytes(uint64_t n);
hipError_t hist_run(const int32_t* N, const uint32_t* lam, uint64_t n, uint32_t g, uint32_t q, void* scratch,
                    int32_t* out_keys, uint64_t* out_counts, uint64_t cap, uint64_t* out_len, uint32_t* err,
                    hipStream_t s);
hipError_t launch_lambda(const PlanDesc& P, const PlanDesc* dP, int coeff_bytes, const void* codes, uint64_t n,
                         const uint32_t* lv, uint32_t* lam, uint32_t sqf, hipStream_t s);
hipError_t launch_gen_reps(int coeff_bytes, uint32_t q, uint32_t ncoef, uint32_t d, uint32_t i, int32_t j,
                           const uint32_t* cj, uint32_t ncj, uint64_t start, uint64_t count, void* out,
                           hipStream_t s);
hipError_t launch_single(const uint32_t* zech, const uint32_t* xs, uint64_t nx, const SingleDesc& f,
                         unsigned long long* out, hipStream_t s);
hipError_t launch_dev_table_fill(uint32_t* tab, uint32_t entries, hipStream_t s);
hipError_t launch_dev_gather(const uint32_t* tab, uint32_t entries, uint32_t chains, uint32_t steps, uint32_t grid,
                             uint32_t* sink, hipStream_t s);
hipError_t launch_valu_issue(uint32_t iters, uint32_t grid, uint32_t* sink, hipStream_t s);
hipError_t launch_lds_gather(uint32_t entries, uint32_t chains, uint32_t steps, uint32_t grid, uint32_t* sink,
                             hipStream_t s);
}  // namespace hwc

// Device memory of the allocation-free entry point (hwc_count_curves_dev_noalloc):
// one array per GPU, allocated when the code object is loaded and held until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns for the current device, kept per device below.
constexpr uint64_t kStaticScratchBytes = HWC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// With `device` current: looks up (once per device) the device address of
// that GPU's copy of `scratch`.
hipError_t setup_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace

namespace {

constexpr uint32_t kLdsLimit = hwc::kLdsImageLimit;
constexpr size_t kMaxGraphs = 8;

struct FieldEntry {
  hwc::Field F;
};

// internal flag: the factorization kernel also marks rows that are not
// square-free (code 0), used by the map of eq. (1.2)
constexpr uint32_t kFlagSqf = 1u << 30;

// Launch and layout choices for one plan (defaults or an autotuned override).
struct Tuning {
  bool split = true;            // split evaluation over mu_m cosets on form A levels
  uint32_t split_min_m = 64;    // ... of at least this many nonzero elements
  bool shift = true;            // count rows with zero coefficients as dense translates f(x + t)
  bool mfma = false;            // prime q <= 31: count by int8 matrix products where the image fits LDS (opt-in)
  uint32_t block = 0;           // threads per workgroup, 0: automatic
  uint32_t wg_per_cu = 0;       // cap on workgroups per CU, 0: occupancy limit
  uint32_t wpe = 0;             // minimum waves per SIMD of the kernel build, 0: none
  uint32_t device_tables = 0;   // bit j-1: level j's table in device memory
};

struct DevPlan {
  uint32_t q = 0, g = 0, orbit = 0;
  std::vector<std::shared_ptr<FieldEntry>> fields;
  std::vector<uint32_t> image;  // dwords
  hwc::PlanDesc desc{};
  void* d_image = nullptr;
  hwc::PlanDesc* d_desc = nullptr;   // device copy of desc (multi-plan launches)
  std::vector<uint32_t*> d_reps;
  std::vector<uint32_t*> d_gtab;     // form D tables
  std::vector<uint32_t*> d_tup, d_sgl;  // split-evaluation tuple representatives and singles
  uint32_t* d_shift = nullptr;       // q^3-byte step table of the dense translates, or nullptr
  // matrix-core path: used for counting when vpath is set.  One pass holds
  // every level; otherwise the lower levels come first and the top level's
  // points are split over the following passes, which add their counts.
  struct VPass {
    hwc::VPlanDesc desc{};
    hwc::VPlanDesc* d_desc = nullptr;
    void* d_image = nullptr;
    uint32_t lo = 0, hi = 0, tw = 4;
    uint32_t grid = 0, block = 256;
  };
  bool vpath = false;
  std::vector<VPass> vpasses;
  uint64_t dev_bytes = 0;
  uint64_t last_use = 0;
  uint32_t block = 256, grid = 0, wpe = 1;
  double tile_cost = 0;
  uint32_t pins = 0;                 // > 0 while a batch being assembled uses the plan
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Device tables of one field for the single-curve kernel.
struct SingleTabs {
  uint32_t* d_zech = nullptr;   // Zech table, one period (M entries)
  uint32_t* d_reps = nullptr;   // primitive Frobenius orbit representatives
  uint64_t nreps = 0;
  uint64_t last_use = 0;
};

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* jobs = nullptr;   // job descriptors owned by a multi-plan graph
  int set = 0;            // scratch set whose buffers the graph uses
  std::vector<const DevPlan*> plans;   // plans whose tables it reads
};

struct JobSlot {          // job descriptors of a direct multi-plan launch
  void* p = nullptr;      // device copy
  void* h = nullptr;      // pinned host staging, copied asynchronously
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};

constexpr uint32_t kSmallStride = 4 * 2048 + 16;   // per-job bucketing words (u32)
// Tile parts: a request whose top level sweeps at least this many points by
// orbits has each tile's top-level sweep cut into 2^kPartLog parts, so that
// the last tiles of a launch do not hold a few waves long after the rest of
// the GPU has run dry (one 2^20-curve request at q = 293, g = 2: 80 -> 72 ms)
// and a job of few tiles spreads over the waves in flight
constexpr uint32_t kPartMinPoints = 8192;
constexpr uint32_t kPartLog = 3;
constexpr int kJobSlots = 4;

// Scratch of the work enqueued on one stream.  Calls on different streams
// use different sets, so their kernels can overlap on the device; calls that
// share a set are ordered by its event (a stream waits for the set's previous
// work when that work went to another stream), so every set's work forms one
// chain and its event, once complete, means all of it is.
struct ScratchSet {
  Buf pid, small, tiles, perm, lv, hist, tcodes, acc;                // one request
  Buf bpid, bperm, btiles, bsmall, btcodes, bacc;   // multi-plan launches
  JobSlot slots[kJobSlots];
  int next_slot = 0;
  hipStream_t last = nullptr;
  hipEvent_t ev = nullptr;
  bool ev_valid = false;
};
constexpr int kSets = 4;           // sets for streams

}  // namespace

struct hwc_field {
  std::shared_ptr<FieldEntry> e;
};

struct hwc_ctx {
  int device = -1;
  uint64_t budget = 0;
  hipStream_t stream = nullptr;     // context stream (also used for capture)
  std::mutex mu;
  std::string err;
  std::map<std::tuple<uint32_t, uint32_t, uint32_t>, std::shared_ptr<FieldEntry>> fields;
  std::map<std::tuple<uint32_t, uint32_t, uint32_t>, std::unique_ptr<DevPlan>> plans;
  uint64_t table_bytes = 0, hits = 0, misses = 0, tick = 0, evictions = 0;
  int cus = 0;
  // scratch of the synchronous host-buffer, map, single-curve and diagnostic calls
  Buf N, codes, hout;
  Buf mcodes, mN, mlam, mhk, mhc, mcj;   // map of eq. (1.2): one chunk of representatives
  std::map<std::tuple<uint32_t, uint32_t, uint32_t>, SingleTabs> single;   // one-curve tables
  uint32_t* d_err = nullptr;
  std::list<GraphEntry> graphs;
  // scratch of the asynchronous calls, one set per stream (round robin past kSets)
  ScratchSet sets[kSets];
  std::vector<std::pair<hipStream_t, int>> set_of;
  int next_set = 0;
  // device memory released while work may still read it: freed once every
  // set's work is complete (hipFree would otherwise wait for the whole device)
  std::vector<void*> grave;
  uint64_t grave_bytes = 0;
  // profiling: events around the phases of each direct (non-graph) call
  bool profile = false;
  Tuning defaults;
  std::map<std::tuple<uint32_t, uint32_t, uint32_t>, Tuning> tuned;   // per (q, g, orbit)
  std::vector<std::array<hipEvent_t, 4>> prof;
  std::vector<hipEvent_t> event_pool;
  // completion of the last allocation-free call (its work reads plan tables
  // that a release must not free while it runs)
  hipEvent_t static_ev = nullptr;
  bool static_ev_valid = false;
};

namespace {

int fail(hwc_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPX(ctx, expr)                                                                                   \
  do {                                                                                                    \
    hipError_t _e = (expr);                                                                               \
    if (_e != hipSuccess) return fail((ctx), HWC_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
  } while (0)

// Device memory that queued work may still read is not freed at once: it is
// kept until every set's work is complete (reap), so releasing it never
// waits for the device in the middle of a stream.
void defer_free(hwc_ctx* c, void* p, uint64_t bytes) {
  if (!p) return;
  c->grave.push_back(p);
  c->grave_bytes += bytes;
}

// Frees the deferred memory once no set has work in flight (wait: wait for
// that work first).  Returns false when something was still running.
bool reap(hwc_ctx* c, bool wait) {
  if (c->grave.empty()) return true;
  for (auto& st : c->sets) {
    if (!st.ev_valid) continue;
    if (wait) {
      if (hipEventSynchronize(st.ev) != hipSuccess) return false;
    } else if (hipEventQuery(st.ev) != hipSuccess) {
      return false;
    }
  }
  if (c->static_ev_valid) {
    if (wait) {
      if (hipEventSynchronize(c->static_ev) != hipSuccess) return false;
    } else if (hipEventQuery(c->static_ev) != hipSuccess) {
      return false;
    }
  }
  for (void* p : c->grave) (void)hipFree(p);
  c->grave.clear();
  c->grave_bytes = 0;
  return true;
}

void wait_set(hwc_ctx* c, int set) {
  ScratchSet& st = c->sets[set];
  if (st.ev_valid) (void)hipEventSynchronize(st.ev);
}

void destroy_graph(hwc_ctx* c, GraphEntry& g) {
  wait_set(c, g.set);   // a replay may still run
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  defer_free(c, g.jobs, 0);
  g.exec = nullptr;
  g.graph = nullptr;
  g.jobs = nullptr;
}

// drop the graphs that use scratch set `set` (-1: every graph)
void drop_graphs(hwc_ctx* c, int set = -1) {
  for (auto it = c->graphs.begin(); it != c->graphs.end();) {
    if (set < 0 || it->set == set) {
      destroy_graph(c, *it);
      it = c->graphs.erase(it);
    } else {
      ++it;
    }
  }
}

// drop the graphs that read the tables of plan P
void drop_graphs_of_plan(hwc_ctx* c, const DevPlan* P) {
  for (auto it = c->graphs.begin(); it != c->graphs.end();) {
    if (std::find(it->plans.begin(), it->plans.end(), P) != it->plans.end()) {
      destroy_graph(c, *it);
      it = c->graphs.erase(it);
    } else {
      ++it;
    }
  }
}

// The scratch set of stream s: its own while there are free sets, then
// shared round robin.
int set_for(hwc_ctx* c, hipStream_t s) {
  for (const auto& kv : c->set_of)
    if (kv.first == s) return kv.second;
  const int k = c->next_set % kSets;
  c->next_set++;
  c->set_of.emplace_back(s, k);
  return k;
}

// order this call's work on s after the previous work of its set
int order_begin(hwc_ctx* c, int set, hipStream_t s) {
  ScratchSet& st = c->sets[set];
  if (st.ev_valid && st.last != s) HIPX(c, hipStreamWaitEvent(s, st.ev, 0));
  return HWC_OK;
}
int order_end(hwc_ctx* c, int set, hipStream_t s) {
  ScratchSet& st = c->sets[set];
  HIPX(c, hipEventRecord(st.ev, s));
  st.last = s;
  st.ev_valid = true;
  return HWC_OK;
}

// grow a scratch buffer of set `set` (never shrinks)
int ensure(hwc_ctx* c, int set, Buf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return HWC_OK;
  if (b.p) {
    drop_graphs(c, set);   // captured graphs may hold the old pointer
    defer_free(c, b.p, b.bytes);
  }
  b.p = nullptr;
  b.bytes = 0;
  size_t want = std::max<size_t>(bytes, 256);
  want = (want + 4095) & ~size_t(4095);
  HIPX(c, hipMalloc(&b.p, want));
  b.bytes = want;
  return HWC_OK;
}

// buffers of the synchronous calls (their work is complete when they return)
int ensure_sync(hwc_ctx* c, Buf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return HWC_OK;
  if (b.p) HIPX(c, hipFree(b.p));
  b.p = nullptr;
  b.bytes = 0;
  size_t want = std::max<size_t>(bytes, 256);
  want = (want + 4095) & ~size_t(4095);
  HIPX(c, hipMalloc(&b.p, want));
  b.bytes = want;
  return HWC_OK;
}

std::shared_ptr<FieldEntry> get_field(hwc_ctx* c, uint32_t p, uint32_t e, uint32_t k, int* rc) {
  auto key = std::make_tuple(p, e, k);
  auto it = c->fields.find(key);
  if (it != c->fields.end()) return it->second;
  auto fe = std::make_shared<FieldEntry>();
  std::string msg = hwc::build_field(p, e, k, &fe->F);
  if (!msg.empty()) {
    *rc = fail(c, msg == "field too large" ? HWC_ERR_FIELD_TOO_LARGE : HWC_ERR_NOT_ODD_PRIME_POWER, msg);
    return nullptr;
  }
  c->fields[key] = fe;
  return fe;
}

// Releases the plan's device memory (deferred: queued work may still read it).
void free_plan(hwc_ctx* c, DevPlan* P) {
  drop_graphs_of_plan(c, P);
  defer_free(c, P->d_image, 0);
  defer_free(c, P->d_desc, 0);
  for (auto* r : P->d_reps) defer_free(c, r, 0);
  for (auto* t : P->d_gtab) defer_free(c, t, 0);
  for (auto* t : P->d_tup) defer_free(c, t, 0);
  for (auto* t : P->d_sgl) defer_free(c, t, 0);
  defer_free(c, P->d_shift, 0);
  for (auto& v : P->vpasses) {
    defer_free(c, v.d_image, 0);
    defer_free(c, v.d_desc, 0);
  }
  c->grave_bytes += P->dev_bytes;
  P->d_shift = nullptr;
  P->vpasses.clear();
  P->vpath = false;
  P->d_tup.clear();
  P->d_sgl.clear();
  P->d_image = nullptr;
  P->d_desc = nullptr;
  P->d_reps.clear();
  P->d_gtab.clear();
}

uint32_t align16(uint32_t v) { return (v + 15u) & ~15u; }

// Bytes of LDS a level table takes in a given form (D lives in device memory).
uint32_t lds_table_bytes(uint32_t form, uint64_t M) {
  if (form == hwc::kFormA) return align16((uint32_t)(10 * M));
  if (form == hwc::kFormC) return align16((uint32_t)(4 * M));
  if (form == hwc::kFormE) return align16((uint32_t)(2 * M));
  if (form == hwc::kFormF) {
    const uint64_t h1 = M / 2 + 1;   // entries of the half table
    return align16((uint32_t)(2 * h1)) + align16((uint32_t)(4 * ((h1 + 31) / 32)));
  }
  if (form == hwc::kFormG) return align16((uint32_t)(4 * (M / 2 + 1)));
  return 0;
}

// Split factor of a level: m = 4 when 4 | q-1, else 3 when 3 | q-1 (form A
// levels only), else 2; 0 when the level is not split.
uint32_t split_factor(uint32_t q, uint32_t form, uint32_t M, const Tuning& T) {
  if (!T.split || M < T.split_min_m) return 0;
  if ((q - 1) % 4 == 0) return 4;
  if (form == hwc::kFormA && (q - 1) % 3 == 0) return 3;
  return 2;                                      // forms C/D: mu_4 or mu_2
}

// Forms of the levels: A where 6M fits u16, C where M fits 15 bits, E where
// M fits 16 bits, G (u32 half table) or else F (17-bit half table) where it
// fits 17 bits, else D; one level at most in an element form (C, E, F or G:
// its table starts the image), the others above it in D; a G level that
// leaves the image too large first moves the levels below it to device
// memory, smallest first (a level of F_{q^i} below F_{q^j} holds about
// q^(i-j) of the points), and becomes F only if that is not enough; then move
// the largest LDS levels to D until the image fits.
std::vector<uint32_t> choose_forms(uint32_t q, uint32_t g, uint32_t device_mask) {
  std::vector<uint32_t> form(g);
  std::vector<uint64_t> M(g);
  uint64_t Qj = 1;
  bool element = false;
  for (uint32_t j = 0; j < g; ++j) {
    Qj *= q;
    M[j] = Qj - 1;
    form[j] = M[j] <= hwc::kFormAMaxM   ? hwc::kFormA
              : M[j] <= hwc::kFormCMaxM ? hwc::kFormC
              : M[j] <= hwc::kFormEMaxM ? hwc::kFormE
              : M[j] <= hwc::kFormFMaxM ? hwc::kFormG
                                        : hwc::kFormD;
    if (form[j] == hwc::kFormC || form[j] == hwc::kFormE || form[j] == hwc::kFormG) {
      if (element) form[j] = hwc::kFormD;
      element = true;
    }
  }
  auto total = [&]() {
    uint64_t t = 0;
    for (uint32_t j = 0; j < g; ++j) t += lds_table_bytes(form[j], M[j]) + align16(4 * q);
    return t;
  };
  for (uint32_t j = 0; j < g; ++j)
    if ((device_mask >> j) & 1u) form[j] = hwc::kFormD;
  for (uint32_t j = 0; j < g; ++j) {
    if (form[j] != hwc::kFormG || total() <= kLdsLimit) continue;
    const std::vector<uint32_t> keep = form;
    for (uint32_t i = 0; i < j && total() > kLdsLimit; ++i) form[i] = hwc::kFormD;
    if (total() > kLdsLimit) {
      form = keep;
      form[j] = hwc::kFormF;
    }
  }
  for (int j = (int)g - 1; j >= 0 && total() > kLdsLimit; --j) form[j] = hwc::kFormD;
  return form;
}

// floor(v / div) = (v * m) >> s for every v <= vmax, with v, m 24-bit operands
// and the product below 2^31 (so that a signed or unsigned shift agree):
// m = ceil(2^s / div) and vmax (m div - 2^s) < 2^s.
bool div_magic(uint64_t vmax, uint32_t div, uint32_t* m, uint32_t* s) {
  if (vmax >= (1u << 24)) return false;
  for (int sh = 31; sh >= 1; --sh) {
    const uint64_t mm = ((1ull << sh) + div - 1) / div;
    if (mm >= (1u << 24) || vmax * mm >= (1ull << 31)) continue;
    if (vmax * (mm * div - (1ull << sh)) >= (1ull << sh)) continue;
    *m = (uint32_t)mm;
    *s = (uint32_t)sh;
    return true;
  }
  return false;
}

// Appends the points pts[i0, i1) of level j (j + 1 coordinates) to an image
// of the matrix-core path: their coordinate blocks and the character table
// with tw-byte entries (plan.h, VPlanDesc) -- the table after the blocks, or
// first when the image is empty (offset 0: nothing to fold into the product,
// which keeps large blocks of a split level reachable).  False when the image
// would pass `limit` or the quotient constants do not exist.
bool append_vlevel(std::vector<uint8_t>& img, const hwc::Field& F, uint32_t j, const std::vector<uint32_t>& xs,
                   size_t i0, size_t i1, uint32_t p, uint32_t NC, uint32_t tw, bool bal, uint32_t sb, uint64_t limit,
                   hwc::VLevel* out) {
  const uint32_t KC = j + 1, M = (uint32_t)F.M;
  hwc::VLevel L{};
  L.pts = (uint32_t)(i1 - i0);
  L.nblk = (L.pts + 31) / 32;
  L.pad = L.nblk * 32 - L.pts;
  uint64_t Q = 1;
  for (uint32_t d = 0; d < KC; ++d) Q *= p;
  const bool table_first = img.empty();
  const uint64_t unit = (uint64_t)tw * hwc::kVSlotUnit;
  uint64_t to, vo;
  if (table_first) {
    to = 0;
    vo = (tw * Q + 15) / 16 * 16;
  } else {
    while (img.size() % 16) img.push_back(0);
    vo = img.size();
    // the table's offset: after the blocks, a multiple of tw * 127
    to = (vo + (uint64_t)L.nblk * KC * 512 + unit - 1) / unit * unit;
  }
  const uint64_t vend = vo + (uint64_t)L.nblk * KC * 512;
  const uint64_t cap = (uint64_t)(16 - NC) * 127;   // what the spare slots can add, in units of 127
  // balanced form: coordinate 0 offset by 127 tw p, the others by 127 sb p^2
  const uint64_t h = (p - 1) / 2, off0 = bal ? 127ull * tw * p : 0, offd = 127ull * sb * p * p;
  if (std::max(vend, to + tw * Q) > limit || (off0 + to) / hwc::kVSlotUnit > cap) return false;
  L.vo = (uint32_t)vo;
  L.to = (uint32_t)to;
  if (bal) {
    const uint64_t span0 = (uint64_t)tw * NC * h * h, spand = (uint64_t)sb * p * NC * h * h;
    if (tw % sb || off0 < span0 || offd < spand || sb * p * p > cap || sb * p * p < 256) return false;
    if (!div_magic(off0 + span0, tw * p, &L.m0, &L.s0)) return false;
    if (off0 + span0 + L.to >= (1u << 24) || offd + spand >= (1u << 24)) return false;
    const uint64_t div = (uint64_t)sb * p * p, m = ((1ull << 32) + div - 1) / div;
    if (m >= (1u << 24) || (offd + spand) * (m * div - (1ull << 32)) >= (1ull << 32)) return false;
    L.m1 = (uint32_t)m;
    L.s1 = 32;
  } else {
    const uint64_t vmax1 = (uint64_t)NC * (p - 1) * (p - 1);
    if (!div_magic(tw * vmax1, tw * p, &L.m0, &L.s0) || !div_magic(vmax1, p, &L.m1, &L.s1)) return false;
    if (tw * vmax1 + L.to >= (1u << 24)) return false;   // coordinate 0 with the offset stays a 24-bit operand
  }
  L.nbm0 = (uint32_t)(0u - (uint32_t)((uint64_t)L.to * L.m0));
  if (img.size() < vend) img.resize(vend, 0);
  // spare slots: coordinate 0 rows sum to (off0 + to) / 127, the others
  // (balanced form) to sb p^2; the curve side holds 127 there
  for (uint32_t pi = 0; pi < L.nblk * 32; ++pi) {
    for (uint32_t d = 0; d < (bal ? KC : 1u); ++d) {
      uint32_t rest = (uint32_t)(d == 0 ? (off0 + L.to) / hwc::kVSlotUnit : offd / hwc::kVSlotUnit);
      for (uint32_t k = NC; k < 16; ++k) {
        const uint32_t a = rest < 127 ? rest : 127;
        img[L.vo + ((size_t)((pi / 32) * KC + d) * 32 + pi % 32) * 16 + k] = (uint8_t)a;
        rest -= a;
      }
    }
  }
  for (uint32_t pi = 0; pi < L.pts; ++pi) {
    const uint32_t bb = pi / 32, row = pi % 32;
    for (uint32_t i = 0; i < NC; ++i) {
      uint32_t el = F.exp[(uint64_t)i * xs[i0 + pi] % M];   // x^i, packed coordinates
      for (uint32_t d = 0; d < KC; ++d, el /= p) {
        const uint32_t digit = el % p;
        int32_t a;
        if (bal) {
          const int32_t db = 2 * digit > p ? (int32_t)digit - (int32_t)p : (int32_t)digit;
          a = d == 0 ? (int32_t)(tw / sb) * db : (int32_t)p * db;
        } else {
          a = (int32_t)(d == 0 ? tw * digit : digit);
        }
        img[L.vo + ((size_t)(bb * KC + d) * 32 + row) * 16 + i] = (uint8_t)(int8_t)a;
      }
    }
  }
  if (img.size() < L.to + tw * Q) img.resize(L.to + tw * Q, 0);
  for (uint64_t el = 0; el < Q; ++el) {
    const uint32_t v = el == 0 ? hwc::kVZero : (F.log[el] & 1u);
    for (uint32_t b = 0; b < tw; ++b) img[L.to + el * tw + b] = (uint8_t)(v >> (8 * b));
  }
  while (img.size() % 16) img.push_back(0);
  *out = L;
  return true;
}

// The passes of the matrix-core path for prime q <= 31 (plan.h, VPlanDesc).
// Leaves vpath unset when q is not such a prime or the levels do not fit.
int build_vplan(hwc_ctx* c, DevPlan* P, uint32_t p, uint32_t e, uint32_t g, uint32_t orbit, uint32_t block_opt,
                bool* ok) {
  *ok = false;
  if (e != 1 || p > hwc::kVMaxP) return HWC_OK;
  const uint32_t NC = 2 * g + 3;
  std::vector<std::vector<uint32_t>> xs(g);
  for (uint32_t j = 0; j < g; ++j) {
    const hwc::Field& F = P->fields[j]->F;
    if (orbit) xs[j] = F.prim_reps;
    else for (uint32_t L = 0; L < (uint32_t)F.M; ++L) xs[j].push_back(L);
  }
  struct Built { std::vector<uint8_t> img; hwc::VPlanDesc d{}; uint32_t lo, hi, tw; };
  std::vector<Built> passes;
  // the balanced form where its constants exist (p = 11, 13; plan.h)
  const uint32_t sb = p == 13 ? 2u : 4u;
  auto use_bal = [&](uint32_t tw) { return (p == 13 || p == 11) && tw % sb == 0; };
  auto start_pass = [&](uint32_t lo, uint32_t hi, uint32_t tw) {
    Built b;
    b.d.p = p; b.d.g = g; b.d.ncoef = NC; b.d.orbit = orbit;
    b.d.bal = use_bal(tw) ? 1u : 0u;
    b.d.sb = sb;
    b.lo = lo; b.hi = hi; b.tw = tw;
    return b;
  };
  const uint64_t limit = hwc::kLdsImageLimit;
  {   // every level in one image
    Built b = start_pass(0, g - 1, 4);
    bool fits = true;
    for (uint32_t j = 0; j < g && fits; ++j)
      fits = append_vlevel(b.img, P->fields[j]->F, j, xs[j], 0, xs[j].size(), p, NC, 4, b.d.bal, sb, limit,
                           &b.d.lv[j]);
    if (fits) passes.push_back(std::move(b));
  }
  if (passes.empty()) {
    // the lower levels in one image, the top level's points over several
    const uint32_t top = g - 1;
    if (g > 1) {
      Built b = start_pass(0, top - 1, 4);
      for (uint32_t j = 0; j < top; ++j)
        if (!append_vlevel(b.img, P->fields[j]->F, j, xs[j], 0, xs[j].size(), p, NC, 4, b.d.bal, sb, limit,
                           &b.d.lv[j]))
          return HWC_OK;
      passes.push_back(std::move(b));
    }
    uint64_t Q = 1;
    for (uint32_t d = 0; d <= top; ++d) Q *= p;
    const uint32_t tw = 4 * Q <= 48 * 1024 ? 4 : 2;
    if (tw == 2 && 2 * (p - 1) > 127) return HWC_OK;
    const uint64_t blk_bytes = (uint64_t)(top + 1) * 512, room = limit - 1024 - tw * Q;
    if (tw * Q + 1024 >= limit || room < blk_bytes) return HWC_OK;
    const size_t per = (size_t)(room / blk_bytes) * 32;
    for (size_t i0 = 0; i0 < xs[top].size(); i0 += per) {
      Built b = start_pass(top, top, tw);
      const size_t i1 = std::min(xs[top].size(), i0 + per);
      if (!append_vlevel(b.img, P->fields[top]->F, top, xs[top], i0, i1, p, NC, tw, b.d.bal, sb, limit,
                         &b.d.lv[top]))
        return HWC_OK;
      passes.push_back(std::move(b));
    }
  }
  for (auto& b : passes) {
    DevPlan::VPass v;
    v.lo = b.lo; v.hi = b.hi; v.tw = b.tw;
    v.desc = b.d;
    v.desc.image_bytes = (uint32_t)b.img.size();
    HIPX(c, hipMalloc(&v.d_image, b.img.size()));
    HIPX(c, hipMemcpy(v.d_image, b.img.data(), b.img.size(), hipMemcpyHostToDevice));
    v.desc.image = static_cast<const uint32_t*>(v.d_image);
    HIPX(c, hipMalloc(&v.d_desc, sizeof(hwc::VPlanDesc)));
    HIPX(c, hipMemcpy(v.d_desc, &v.desc, sizeof(v.desc), hipMemcpyHostToDevice));
    P->dev_bytes += b.img.size() + sizeof(v.desc);
    c->table_bytes += b.img.size() + sizeof(v.desc);
    // the block size that keeps the most waves per CU resident (LDS holds one
    // image per workgroup), unless a block size is set
    int best_waves = 0;
    for (uint32_t blk : {256u, 512u, 1024u}) {
      if (block_opt && blk != block_opt) continue;
      int bpc = 0;
      HIPX(c, hwc::occupancy_vcount(g, blk, v.desc.image_bytes, &bpc));
      if (bpc * (int)blk > best_waves * 64) {
        best_waves = bpc * (int)blk / 64;
        v.block = blk;
        v.grid = (uint32_t)(c->cus * bpc);
      }
    }
    P->vpasses.push_back(v);
    if (best_waves < 1) return HWC_OK;
  }
  *ok = true;
  return HWC_OK;
}

// Build (or fetch) the device plan for (q, g, orbit).
int get_plan(hwc_ctx* c, uint32_t q, uint32_t g, uint32_t orbit, DevPlan** out) {
  auto key = std::make_tuple(q, g, orbit);
  auto it = c->plans.find(key);
  if (it != c->plans.end()) {
    c->hits++;
    it->second->last_use = ++c->tick;
    *out = it->second.get();
    return HWC_OK;
  }
  c->misses++;
  uint32_t p, e;
  if (!hwc::factor_odd_prime_power(q, &p, &e)) return fail(c, HWC_ERR_NOT_ODD_PRIME_POWER, "q is not an odd prime power");
  if (g < 1 || g > (uint32_t)hwc::kMaxG) return fail(c, HWC_ERR_BAD_G, "g must be in 1..4");
  double Qg = 1;
  for (uint32_t j = 0; j < g; ++j) Qg *= q;
  if (Qg > 16777216.0 || q > 32768) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "F_{q^g} larger than 2^24 elements");
  Tuning T = c->defaults;
  {
    auto tt = c->tuned.find(key);
    if (tt != c->tuned.end()) T = tt->second;
  }
  const std::vector<uint32_t> form = choose_forms(q, g, T.device_tables);
  if (8 * q > kLdsLimit) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "q too large");
  auto P = std::make_unique<DevPlan>();
  P->q = q; P->g = g; P->orbit = orbit;
  int rc = HWC_OK;
  for (uint32_t j = 1; j <= g; ++j) {
    auto fe = get_field(c, p, e, j, &rc);
    if (!fe) return rc;
    P->fields.push_back(fe);
  }
  // LDS image: level tables (forms A and C), then embedding tables
  std::vector<uint16_t> img;
  auto put = [&](const std::vector<uint16_t>& v) {
    uint32_t off = (uint32_t)img.size() * 2;
    img.insert(img.end(), v.begin(), v.end());
    while ((img.size() * 2) % 16) img.push_back(0);
    return off;
  };
  hwc::PlanDesc& D = P->desc;
  D.q = q; D.p = p; D.g = g; D.ncoef = 2 * g + 3; D.orbit = orbit;
  std::vector<std::vector<uint32_t>> gtabs(g);
  // forms C and D hold 2 Z (byte units) with the marker 2M over two periods,
  // form E one period of Z with the marker M; the (single) form C or E table
  // goes first, at byte offset 0 of the image
  for (uint32_t j = 0; j < g; ++j) {
    if (form[j] != hwc::kFormC && form[j] != hwc::kFormE && form[j] != hwc::kFormF && form[j] != hwc::kFormG)
      continue;
    const hwc::Field& F = P->fields[j]->F;
    const uint32_t M = (uint32_t)F.M;
    if (!img.empty()) return fail(c, HWC_ERR_DEVICE, "two LDS levels in element form");
    std::vector<uint16_t> tab;
    if (form[j] == hwc::kFormC) {
      tab.resize(2 * (size_t)M);
      for (uint32_t i = 0; i < 2 * M; ++i) {
        const uint32_t z = F.zech[i % M];
        tab[i] = (uint16_t)(z == M ? 2 * M : 2 * z);
      }
    } else if (form[j] == hwc::kFormE) {
      tab.resize(M);
      for (uint32_t i = 0; i < M; ++i) tab[i] = (uint16_t)F.zech[i];   // Z(i) < M, or the marker M
    } else if (form[j] == hwc::kFormF) {
      // low halves of Z(0..M/2) (17-bit values, the marker M at M/2), padded
      // to 16 bytes, then the 17th bits as u32 words (little-endian halves)
      const uint32_t h1 = M / 2 + 1;
      tab.assign(((size_t)h1 + 7) / 8 * 8, 0);
      std::vector<uint32_t> bits(((size_t)h1 + 31) / 32, 0);
      for (uint32_t i = 0; i < h1; ++i) {
        const uint32_t z = F.zech[i];
        tab[i] = (uint16_t)(z & 0xFFFFu);
        bits[i >> 5] |= ((z >> 16) & 1u) << (i & 31);
      }
      for (uint32_t w : bits) {
        tab.push_back((uint16_t)(w & 0xFFFFu));
        tab.push_back((uint16_t)(w >> 16));
      }
    } else {
      // u32 halves of 2 Z(0..M/2) (byte units; little-endian pairs of u16),
      // the marker 2 M2 = 4M at M/2, so that folding it by M2 gives M2
      const uint32_t h1 = M / 2 + 1;
      tab.assign(2 * (size_t)h1, 0);
      for (uint32_t i = 0; i < h1; ++i) {
        const uint32_t z = F.zech[i];
        const uint32_t v = z == M ? 4 * M : 2 * z;
        tab[2 * (size_t)i] = (uint16_t)(v & 0xFFFFu);
        tab[2 * (size_t)i + 1] = (uint16_t)(v >> 16);
      }
    }
    D.lv[j].tab_off = put(tab);
  }
  for (uint32_t j = 0; j < g; ++j) {
    const hwc::Field& F = P->fields[j]->F;
    const uint32_t M = (uint32_t)F.M;
    hwc::LevelDesc& L = D.lv[j];
    L.M = M;
    L.form = form[j];
    if (form[j] == hwc::kFormA) {
      std::vector<uint16_t> tab(5 * (size_t)M, 0);
      for (uint32_t i = 0; i < 3 * M; ++i) {
        const uint32_t z = F.zech[i % M];
        tab[i] = (uint16_t)(z == M ? 6 * M : 2 * z);
      }
      L.tab_off = put(tab);
    } else if (form[j] == hwc::kFormD) {
      L.tab_off = 0;
      gtabs[j].resize(2 * (size_t)M);
      for (uint32_t i = 0; i < 2 * M; ++i) {
        const uint32_t z = F.zech[i % M];
        gtabs[j][i] = z == M ? 2 * M : 2 * z;
      }
    }
    if (orbit) {
      L.nx = (uint32_t)F.prim_reps.size();
      L.weight = j + 1;
    } else {
      L.nx = M;
      L.weight = 1;
    }
  }
  for (uint32_t j = 0; j < g; ++j) {
    // u32 entries: logs reach M - 1, beyond u16 for the largest fields
    const hwc::Field& F = P->fields[j]->F;
    std::vector<uint16_t> emb(2 * F.q);
    for (uint64_t i = 0; i < F.q; ++i) {
      emb[2 * i] = (uint16_t)(F.emb[i] & 0xFFFFu);
      emb[2 * i + 1] = (uint16_t)(F.emb[i] >> 16);
    }
    D.lv[j].emb_off = put(emb);
  }
  D.image_bytes = (uint32_t)img.size() * 2;
  if (D.image_bytes > kLdsLimit) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "LDS image too large");
  P->image.assign(img.size() / 2, 0);
  std::memcpy(P->image.data(), img.data(), img.size() * 2);
  // device memory for the plan, admitted against the budget
  uint64_t bytes = D.image_bytes + sizeof(hwc::PlanDesc);
  for (uint32_t j = 0; j < g; ++j) {
    if (orbit) bytes += P->fields[j]->F.prim_reps.size() * 4;
    bytes += gtabs[j].size() * 4;
  }
  if (c->budget && bytes > c->budget)
    return fail(c, HWC_ERR_OOM_BUDGET, "tables exceed the context's HBM budget");
  HIPX(c, hipMalloc(&P->d_image, D.image_bytes));
  HIPX(c, hipMemcpy(P->d_image, P->image.data(), D.image_bytes, hipMemcpyHostToDevice));
  D.image = static_cast<const uint32_t*>(P->d_image);
  P->d_reps.assign(g, nullptr);
  P->d_gtab.assign(g, nullptr);
  for (uint32_t j = 0; j < g; ++j) {
    D.lv[j].xs = nullptr;
    D.lv[j].gtab = nullptr;
    if (orbit) {
      const auto& reps = P->fields[j]->F.prim_reps;
      HIPX(c, hipMalloc(&P->d_reps[j], std::max<size_t>(reps.size(), 1) * 4));
      if (!reps.empty()) HIPX(c, hipMemcpy(P->d_reps[j], reps.data(), reps.size() * 4, hipMemcpyHostToDevice));
      D.lv[j].xs = P->d_reps[j];
    }
    if (!gtabs[j].empty()) {
      HIPX(c, hipMalloc(&P->d_gtab[j], gtabs[j].size() * 4));
      HIPX(c, hipMemcpy(P->d_gtab[j], gtabs[j].data(), gtabs[j].size() * 4, hipMemcpyHostToDevice));
      D.lv[j].gtab = P->d_gtab[j];
    }
  }
  // split evaluation over mu_m cosets
  P->d_tup.assign(g, nullptr);
  P->d_sgl.assign(g, nullptr);
  for (uint32_t j = 0; j < g; ++j) {
    hwc::LevelDesc& L = D.lv[j];
    L.msplit = 0; L.nt = 0; L.ns = 0; L.xs_t = nullptr; L.xs_s = nullptr;
    const uint32_t m = split_factor(q, L.form, L.M, T);
    if (!m) continue;
    L.msplit = m;
    if (!orbit) {
      L.nt = L.M / m;
      continue;
    }
    std::vector<uint32_t> tup, sgl;
    hwc::split_orbits(P->fields[j]->F, m, &tup, &sgl);
    L.nt = (uint32_t)tup.size();
    L.ns = (uint32_t)sgl.size();
    HIPX(c, hipMalloc(&P->d_tup[j], std::max<size_t>(tup.size(), 1) * 4));
    HIPX(c, hipMalloc(&P->d_sgl[j], std::max<size_t>(sgl.size(), 1) * 4));
    if (!tup.empty()) HIPX(c, hipMemcpy(P->d_tup[j], tup.data(), tup.size() * 4, hipMemcpyHostToDevice));
    if (!sgl.empty()) HIPX(c, hipMemcpy(P->d_sgl[j], sgl.data(), sgl.size() * 4, hipMemcpyHostToDevice));
    L.xs_t = P->d_tup[j];
    L.xs_s = P->d_sgl[j];
    P->dev_bytes += (tup.size() + sgl.size()) * 4;
    c->table_bytes += (tup.size() + sgl.size()) * 4;
  }
  // dense translates: step[t][a][b] = a + t b over F_q (codes), q^3 bytes
  if (T.shift && q <= hwc::kShiftMaxQ) {
    const hwc::Field& F1 = P->fields[0]->F;   // F_q itself: emb = log of a code
    std::vector<uint32_t> expq(q - 1);
    for (uint32_t cc = 1; cc < q; ++cc) expq[F1.emb[cc]] = cc;
    auto add = [&](uint32_t a, uint32_t b) {   // digit-wise in base p
      uint32_t r = 0, pw = 1;
      for (uint32_t i = 0; i < e; ++i, pw *= p) r += ((a / pw % p + b / pw % p) % p) * pw;
      return r;
    };
    auto mul = [&](uint32_t a, uint32_t b) -> uint32_t {
      if (a == 0 || b == 0) return 0;
      return expq[(F1.emb[a] + F1.emb[b]) % (q - 1)];
    };
    const uint32_t nc = 2 * g + 3, tw = hwc::shift_tmat_words(nc), rw = hwc::shift_tmat_row_words(nc);
    const size_t toff = (size_t)hwc::shift_tmat_offset_words(q) * 4;
    std::vector<uint8_t> st(toff + (size_t)(hwc::kShiftTries + 1) * tw * 4, 0);
    for (uint32_t t = 0; t < q; ++t)
      for (uint32_t b = 0; b < q; ++b) {
        const uint32_t tb = mul(t, b);
        for (uint32_t a = 0; a < q; ++a) st[((size_t)t * q + a) * q + b] = (uint8_t)add(a, tb);
      }
    if (e == 1) {   // prime q: the translate as a matrix, binom(j, i) t^(j-i) mod q
      std::vector<uint32_t> binom((size_t)nc * nc, 0);
      for (uint32_t j = 0; j < nc; ++j)
        for (uint32_t i = 0; i <= j; ++i)
          binom[j * nc + i] = (i == 0 || i == j) ? 1u : (binom[(j - 1) * nc + i - 1] + binom[(j - 1) * nc + i]) % q;
      for (uint32_t t = 0; t <= hwc::kShiftTries && t < q; ++t)
        for (uint32_t i = 0; i + 1 < nc; ++i) {
          uint32_t tp = 1;   // t^(j-i)
          for (uint32_t j = i; j < nc; ++j, tp = tp * t % q)
            st[toff + ((size_t)t * tw + i * rw + j / 4) * 4 + j % 4] = (uint8_t)(binom[j * nc + i] * tp % q);
        }
    }
    HIPX(c, hipMalloc(&P->d_shift, st.size()));
    HIPX(c, hipMemcpy(P->d_shift, st.data(), st.size(), hipMemcpyHostToDevice));
    P->dev_bytes += st.size();
    c->table_bytes += st.size();
  }
  HIPX(c, hipMalloc(&P->d_desc, sizeof(hwc::PlanDesc)));
  HIPX(c, hipMemcpy(P->d_desc, &D, sizeof(hwc::PlanDesc), hipMemcpyHostToDevice));
  P->dev_bytes += bytes;
  c->table_bytes += bytes;
  // launch shape: the block size that keeps the most waves resident per CU
  // (the image limits the workgroups per CU through LDS, the kernel's
  // registers limit the waves), the smaller block on a tie
  int bpc = 0;
  P->wpe = T.wpe ? T.wpe : 1;
  if (T.block) {
    P->block = T.block;
  } else {
    int best = -1;
    for (uint32_t b : {256u, 512u, 1024u}) {
      int n = 0;
      HIPX(c, hwc::occupancy_count(g, 1, b, D.image_bytes, P->wpe, &n));
      const int waves = n * (int)(b / hwc::kWave);
      if (waves > best) {
        best = waves;
        P->block = b;
      }
    }
  }
  HIPX(c, hwc::occupancy_count(g, 1, P->block, D.image_bytes, P->wpe, &bpc));
  if (bpc < 1) bpc = 1;
  if (T.wg_per_cu && (int)T.wg_per_cu < bpc) bpc = (int)T.wg_per_cu;
  P->grid = (uint32_t)(c->cus * bpc);
  if (T.mfma) {
    bool ok = false;
    int rv = build_vplan(c, P.get(), p, e, g, orbit, T.block, &ok);
    if (rv) return rv;
    P->vpath = ok;
  }
  if (c->budget) {
    // admission by the HBM budget: least recently used plans make room; their
    // memory counts against the budget until it is actually freed (once the
    // work reading it is done)
    (void)reap(c, false);
    while (c->table_bytes + c->grave_bytes > c->budget) {
      auto victim = c->plans.end();
      for (auto i2 = c->plans.begin(); i2 != c->plans.end(); ++i2)
        if (i2->second->pins == 0 && (victim == c->plans.end() || i2->second->last_use < victim->second->last_use))
          victim = i2;
      if (victim == c->plans.end()) break;
      c->table_bytes -= victim->second->dev_bytes;
      free_plan(c, victim->second.get());
      c->plans.erase(victim);
      c->evictions++;
      (void)reap(c, false);
    }
    if (c->table_bytes + c->grave_bytes > c->budget && c->grave_bytes) (void)reap(c, true);
    if (c->table_bytes + c->grave_bytes > c->budget) {
      c->table_bytes -= P->dev_bytes;
      free_plan(c, P.get());
      (void)reap(c, false);
      return fail(c, HWC_ERR_OOM_BUDGET, "tables exceed the context's HBM budget");
    }
  }
  // relative cost of one tile, for ordering mixed batches (longest first)
  P->tile_cost = 0;
  for (uint32_t j = 0; j < g; ++j)
    P->tile_cost += (double)D.lv[j].nx * (2 * g + 2) *
                    (form[j] == hwc::kFormA   ? 1.0
                     : form[j] == hwc::kFormC ? 1.5
                     : form[j] == hwc::kFormE ? 2.0
                     : form[j] == hwc::kFormF ? 3.0
                     : form[j] == hwc::kFormG ? 2.5
                                              : 6.0);
  P->last_use = ++c->tick;
  *out = P.get();
  c->plans[key] = std::move(P);
  return HWC_OK;
}

struct Scratch {
  uint16_t* pid;
  uint32_t *counts, *bucket_start, *tile_start, *cursor, *ntiles, *queue;
  uint64_t* tiles;
  uint32_t* perm;
  uint32_t* lv;
  void* hist;
  void* tcodes;   // dense translates of the rows (plans with a step table)
  uint32_t* acc;  // tile parts: [n][g] summed level counts, then [max_tiles] finished parts
  uint64_t max_tiles;
};

// Byte sizes of the scratch parts of one request of n rows (plain: per-level
// results, also needed for the factorization partition and the passes of the
// matrix-product path; tcodes: dense translates of the rows).
struct ScratchSizes {
  uint64_t pid, small, tiles, perm, lv, hist, tcodes, acc;
  uint64_t max_tiles;
};
ScratchSizes scratch_sizes(uint64_t n, uint32_t g, int cb, bool plain, bool hist, bool tcodes, bool parts = false) {
  const uint32_t npat = hwc::pattern_count(g);
  ScratchSizes z{};
  z.max_tiles = n / hwc::kWave + npat + 1;
  z.pid = std::max<uint64_t>(n, 1) * 2;
  z.small = (uint64_t)(4 * npat + 16) * 4;
  z.tiles = z.max_tiles * 8;
  z.perm = std::max<uint64_t>(n, 1) * 4;
  z.lv = plain ? std::max<uint64_t>(n, 1) * g * 4 : 0;
  z.hist = hist ? hwc::hist_scratch_bytes(n) : 0;
  z.tcodes = tcodes ? std::max<uint64_t>(n, 1) * (2 * g + 3) * (uint64_t)cb : 0;
  z.acc = parts ? (n * g + z.max_tiles) * 4 : 0;
  return z;
}

// Points the parts of S at base + offsets (256-byte aligned); returns the bytes used.
uint64_t carve_scratch(const ScratchSizes& z, uint32_t g, uint8_t* base, Scratch* s) {
  const uint32_t npat = hwc::pattern_count(g);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) -> void* {
    void* p = base ? static_cast<void*>(base + off) : nullptr;
    off += (bytes + 255) / 256 * 256;
    return bytes ? p : nullptr;
  };
  s->max_tiles = z.max_tiles;
  s->pid = static_cast<uint16_t*>(take(z.pid));
  uint32_t* sm = static_cast<uint32_t*>(take(z.small));
  s->counts = sm;
  s->bucket_start = sm ? sm + npat : nullptr;
  s->tile_start = sm ? sm + 2 * npat : nullptr;
  s->cursor = sm ? sm + 3 * npat : nullptr;
  s->ntiles = sm ? sm + 4 * npat : nullptr;
  s->queue = sm ? sm + 4 * npat + 4 : nullptr;
  s->tiles = static_cast<uint64_t*>(take(z.tiles));
  s->perm = static_cast<uint32_t*>(take(z.perm));
  s->lv = static_cast<uint32_t*>(take(z.lv));
  s->hist = take(z.hist);
  s->tcodes = take(z.tcodes);
  s->acc = static_cast<uint32_t*>(take(z.acc));
  return off;
}

int get_scratch(hwc_ctx* c, int set, uint64_t n, uint32_t g, int cb, bool plain, bool hist, bool tcodes,
                bool parts, Scratch* s) {
  const ScratchSizes z = scratch_sizes(n, g, cb, plain, hist, tcodes, parts);
  ScratchSet& st = c->sets[set];
  int rc;
  if ((rc = ensure(c, set, st.pid, z.pid))) return rc;
  if ((rc = ensure(c, set, st.small, z.small))) return rc;
  if ((rc = ensure(c, set, st.tiles, z.tiles))) return rc;
  if ((rc = ensure(c, set, st.perm, z.perm))) return rc;
  if (plain && (rc = ensure(c, set, st.lv, z.lv))) return rc;
  if (hist && (rc = ensure(c, set, st.hist, z.hist))) return rc;
  if (tcodes && (rc = ensure(c, set, st.tcodes, z.tcodes))) return rc;
  if (parts && (rc = ensure(c, set, st.acc, z.acc))) return rc;
  const uint32_t npat = hwc::pattern_count(g);
  s->max_tiles = z.max_tiles;
  s->pid = static_cast<uint16_t*>(st.pid.p);
  uint32_t* sm = static_cast<uint32_t*>(st.small.p);
  s->counts = sm;
  s->bucket_start = sm + npat;
  s->tile_start = sm + 2 * npat;
  s->cursor = sm + 3 * npat;
  s->ntiles = sm + 4 * npat;
  s->queue = sm + 4 * npat + 4;
  s->tiles = static_cast<uint64_t*>(st.tiles.p);
  s->perm = static_cast<uint32_t*>(st.perm.p);
  s->lv = plain ? static_cast<uint32_t*>(st.lv.p) : nullptr;
  s->hist = hist ? st.hist.p : nullptr;
  s->tcodes = tcodes ? st.tcodes.p : nullptr;
  s->acc = parts ? static_cast<uint32_t*>(st.acc.p) : nullptr;
  return HWC_OK;
}

// Workgroups of a persistent launch over about `tiles` tiles: at most the
// resident grid, and no more than the tiles need, so that a small request's
// tiles land one workgroup per CU (the dispatcher spreads workgroups over
// the CUs) instead of on whichever waves win the queue first, which can put
// several of them on one CU while others idle.
uint32_t persistent_grid(uint32_t resident, uint32_t block, uint64_t tiles) {
  const uint64_t per = std::max<uint32_t>(block / hwc::kWave, 1);
  const uint64_t need = (tiles + per - 1) / per;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(resident, need));
}

// log2 of the parts each tile's top-level sweep is cut into (kPartMinPoints):
// orbit sweeps of the Zech path only (the point lists are explicit), not the
// plain form (one launch per level, whole tiles)
uint32_t part_log(const DevPlan* P, uint32_t flags) {
  if (P->vpath || !P->orbit || (flags & HWC_PLAIN)) return 0;
  const hwc::LevelDesc& top = P->desc.lv[P->g - 1];
  return top.xs && top.nx >= kPartMinPoints ? kPartLog : 0;
}

// Enqueue the whole count of one request on stream s.
int take_event(hwc_ctx* c, hipEvent_t* ev) {
  if (!c->event_pool.empty()) {
    *ev = c->event_pool.back();
    c->event_pool.pop_back();
    return HWC_OK;
  }
  HIPX(c, hipEventCreate(ev));
  return HWC_OK;
}

int enqueue(hwc_ctx* c, DevPlan* P, const Scratch& S, const void* codes, int cb, uint64_t n, int32_t* N,
            uint32_t* lam, int32_t* hk, uint64_t* hc, uint64_t hcap, uint64_t* hlen, uint32_t flags, hipStream_t s,
            bool record = false) {
  const uint32_t g = P->g;
  std::array<hipEvent_t, 4> ev{};
  if (record) {
    for (auto& e : ev) {
      int rc = take_event(c, &e);
      if (rc) return rc;
    }
    HIPX(c, hipEventRecord(ev[0], s));
  }
  if (P->vpath) {
    // matrix-core path: rows in input order, no bucketing
    if (record) HIPX(c, hipEventRecord(ev[1], s));
    if (n > 0) {
      const auto& V = P->vpasses;
      if (V.size() == 1 && !(flags & HWC_PLAIN)) {
        HIPX(c, hwc::launch_vcount(V[0].desc, V[0].d_desc, cb, codes, n, 0, g - 1, 4, false, N, lam ? S.lv : nullptr,
                                   c->d_err, V[0].grid, V[0].block, s));
      } else {
        // one launch per level (plain form) or per pass, counts added up per curve
        HIPX(c, hwc::launch_fill(S.lv, 0, n * g, s));
        for (const auto& v : V)
          for (uint32_t j = v.lo; j <= v.hi; ++j) {
            if (!(flags & HWC_PLAIN) && j != v.lo) break;
            const uint32_t hi = (flags & HWC_PLAIN) ? j : v.hi;
            HIPX(c, hwc::launch_vcount(v.desc, v.d_desc, cb, codes, n, j, hi, v.tw, true, nullptr, S.lv, c->d_err,
                                       v.grid, v.block, s));
          }
        HIPX(c, hwc::launch_assemble(P->desc, cb, codes, n, S.lv, N, s));
      }
      if (lam)
        HIPX(c, hwc::launch_lambda(P->desc, P->d_desc, cb, codes, n, S.lv, lam, (flags & kFlagSqf) ? 1u : 0u, s));
    }
    if (record) HIPX(c, hipEventRecord(ev[2], s));
    if (hk) HIPX(c, hwc::hist_run(N, lam, n, g, P->q, S.hist, hk, hc, hcap, hlen, c->d_err, s));
    if (record) {
      HIPX(c, hipEventRecord(ev[3], s));
      c->prof.push_back(ev);
    }
    return HWC_OK;
  }
  const bool shifted = P->d_shift && n > 0;
  if (shifted) {   // translate and classify in one pass
    HIPX(c, hwc::launch_fill(S.counts, 0, hwc::pattern_count(g), s));
    HIPX(c, hwc::launch_shift(cb, g, codes, n, P->q, P->d_shift, S.tcodes, S.pid, S.counts, c->d_err, s));
    codes = S.tcodes;
  }
  HIPX(c, hwc::launch_bucket(cb, codes, n, P->q, g, S.pid, S.counts, c->d_err, S.bucket_start, S.tile_start,
                             S.cursor, S.ntiles, S.queue, S.tiles, S.perm, S.max_tiles, shifted, s));
  if (record) HIPX(c, hipEventRecord(ev[1], s));
  if (n > 0) {
    if (flags & HWC_PLAIN) {
      for (uint32_t j = 0; j < g; ++j)
        HIPX(c, hwc::launch_count(P->desc, P->d_desc, cb, codes, S.perm, S.tiles, S.ntiles, nullptr, j, j, nullptr, S.lv,
                                  0, nullptr, nullptr, P->grid, P->block, P->wpe, s));
      HIPX(c, hwc::launch_assemble(P->desc, cb, codes, n, S.lv, N, s));
    } else {
      // a tile per bucket's ragged end besides the full ones (translated rows
      // fall in a few buckets; more tiles are still all counted)
      const uint32_t grid = persistent_grid(P->grid, P->block, (n + hwc::kWave - 1) / hwc::kWave + 4);
      const uint32_t plog = S.acc ? part_log(P, flags) : 0u;
      if (plog) HIPX(c, hwc::launch_fill(S.acc, 0, n * g + S.max_tiles, s));
      HIPX(c, hwc::launch_count(P->desc, P->d_desc, cb, codes, S.perm, S.tiles, S.ntiles, S.queue, 0, g - 1, N,
                                lam ? S.lv : nullptr, plog, plog ? S.acc : nullptr, plog ? S.acc + n * g : nullptr,
                                grid, P->block, P->wpe, s));
    }
    if (lam) HIPX(c, hwc::launch_lambda(P->desc, P->d_desc, cb, codes, n, S.lv, lam, (flags & kFlagSqf) ? 1u : 0u, s));
  }
  if (record) HIPX(c, hipEventRecord(ev[2], s));
  if (hk) HIPX(c, hwc::hist_run(N, lam, n, g, P->q, S.hist, hk, hc, hcap, hlen, c->d_err, s));
  if (record) {
    HIPX(c, hipEventRecord(ev[3], s));
    c->prof.push_back(ev);
  }
  return HWC_OK;
}

int check_args(hwc_ctx* c, uint32_t q, uint32_t g, uint32_t flags) {
  if (!c) return HWC_ERR_ARG;
  if (c->device < 0) return fail(c, HWC_ERR_NO_DEVICE, "host-only context cannot count");
  if (flags & ~(HWC_FULL_SWEEP | HWC_PLAIN | HWC_VALIDATE | HWC_NO_GRAPH)) return fail(c, HWC_ERR_ARG, "unknown flag");
  uint32_t p, e;
  if (!hwc::factor_odd_prime_power(q, &p, &e)) return fail(c, HWC_ERR_NOT_ODD_PRIME_POWER, "q is not an odd prime power");
  if (g < 1 || g > (uint32_t)hwc::kMaxG) return fail(c, HWC_ERR_BAD_G, "g must be in 1..4");
  return HWC_OK;
}

// Argument checks and the plan of one device-pointer request.
int prepare_dev(hwc_ctx* c, uint32_t q, uint32_t g, const void* codes, int cb, uint64_t n, int32_t* N, int32_t* hk,
                uint64_t* hc, uint64_t* hlen, uint32_t flags, uint32_t* lam, bool build, DevPlan** out) {
  int rc = check_args(c, q, g, flags & ~kFlagSqf);
  if (rc) return rc;
  if (cb != 1 && cb != 2) return fail(c, HWC_ERR_ARG, "coeff_bytes must be 1 or 2");
  if (cb == 1 && q > 127) return fail(c, HWC_ERR_ARG, "int8 codes need q <= 127");
  if (n > 0 && (!codes || !N)) return fail(c, HWC_ERR_ARG, "null device pointer");
  if (hk && (!hc || !hlen)) return fail(c, HWC_ERR_ARG, "histogram needs counts and length pointers");
  if (n >= (1ull << 31)) return fail(c, HWC_ERR_ARG, "n too large");
  HIPX(c, hipSetDevice(c->device));
  DevPlan* P = nullptr;
  const auto key = std::make_tuple(q, g, (flags & HWC_FULL_SWEEP) ? 0u : 1u);
  if (build) {
    if ((rc = get_plan(c, q, g, std::get<2>(key), &P))) return rc;
  } else {
    auto it = c->plans.find(key);
    if (it == c->plans.end())
      return fail(c, HWC_ERR_ARG, "the plan of (q, g) is not resident: build it first (hwc_plan_info or a count)");
    P = it->second.get();
    P->last_use = ++c->tick;
  }
  if (lam && P->desc.lv[0].form != hwc::kFormA)
    return fail(c, HWC_ERR_FIELD_TOO_LARGE, "the factorization partition needs q <= 10923");
  if (hk) {   // the histogram key (mixed radix 2q^k+3, plus the partition's rank) must fit 63 bits
    double bits = lam ? std::log2((double)hwc::lam_code_list(g, nullptr)) : 0.0, qk = 1;
    for (uint32_t k = 0; k < g; ++k) {
      qk *= q;
      bits += std::log2(2 * qk + 3);
    }
    if (bits > 63.0) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "histogram key wider than 63 bits for this (q, g)");
  }
  *out = P;
  return HWC_OK;
}

bool needs_lv(const DevPlan* P, uint32_t flags, const uint32_t* lam) {
  return (flags & HWC_PLAIN) != 0 || lam != nullptr || (P->vpath && P->vpasses.size() > 1);
}
bool needs_tcodes(const DevPlan* P) { return P->d_shift != nullptr && !P->vpath; }

int run_dev(hwc_ctx* c, uint32_t q, uint32_t g, const void* codes, int cb, uint64_t n, int32_t* N, int32_t* hk,
            uint64_t* hc, uint64_t hcap, uint64_t* hlen, uint32_t flags, hipStream_t s, uint32_t* lam = nullptr) {
  DevPlan* P = nullptr;
  int rc = prepare_dev(c, q, g, codes, cb, n, N, hk, hc, hlen, flags, lam, true, &P);
  if (rc) return rc;
  const int set = set_for(c, s);
  (void)reap(c, false);
  Scratch S;
  if ((rc = get_scratch(c, set, n, g, cb, needs_lv(P, flags, lam), hk != nullptr, needs_tcodes(P),
                        part_log(P, flags) > 0, &S)))
    return rc;
  const bool use_graph = !(flags & (HWC_PLAIN | HWC_NO_GRAPH)) && n > 0 && !c->profile;
  if ((rc = order_begin(c, set, s))) return rc;
  if (!use_graph) {
    rc = enqueue(c, P, S, codes, cb, n, N, lam, hk, hc, hcap, hlen, flags, s, c->profile);
    if (rc) return rc;
    return order_end(c, set, s);
  }
  std::vector<uint64_t> key = {1, (uint64_t)(uintptr_t)P, n, (uint64_t)cb, (uint64_t)(uintptr_t)codes,
                               (uint64_t)(uintptr_t)N, (uint64_t)(uintptr_t)hk, (uint64_t)(uintptr_t)hc, hcap,
                               (uint64_t)(uintptr_t)hlen, flags, (uint64_t)(uintptr_t)lam, (uint64_t)set};
  for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it) {
    if (it->key == key) {
      c->graphs.splice(c->graphs.begin(), c->graphs, it);
      HIPX(c, hipGraphLaunch(c->graphs.front().exec, s));
      return order_end(c, set, s);
    }
  }
  // capture on the context stream, replay on s
  if (s != c->stream) HIPX(c, hipStreamSynchronize(c->stream));
  GraphEntry ge;
  ge.key = key;
  ge.set = set;
  ge.plans = {P};
  HIPX(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  rc = enqueue(c, P, S, codes, cb, n, N, lam, hk, hc, hcap, hlen, flags, c->stream);
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(c->stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ee != hipSuccess) return fail(c, HWC_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(ee));
  ge.graph = graph;
  HIPX(c, hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0));
  c->graphs.push_front(ge);
  while (c->graphs.size() > kMaxGraphs) {
    destroy_graph(c, c->graphs.back());
    c->graphs.pop_back();
  }
  HIPX(c, hipGraphLaunch(c->graphs.front().exec, s));
  return order_end(c, set, s);
}

// The allocation-free form of run_dev: the plan must already be resident
// (building it allocates), every scratch part is carved out of this GPU's
// static array, kernels are launched directly (instantiating a graph
// allocates) and nothing is allocated or freed.  Overlapping calls on one GPU
// share the array and race; the caller orders them.
int run_dev_noalloc(hwc_ctx* c, uint32_t q, uint32_t g, const void* codes, int cb, uint64_t n, int32_t* N,
                    int32_t* hk, uint64_t* hc, uint64_t hcap, uint64_t* hlen, uint32_t flags, hipStream_t s) {
  DevPlan* P = nullptr;
  int rc = prepare_dev(c, q, g, codes, cb, n, N, hk, hc, hlen, flags, nullptr, false, &P);
  if (rc) return rc;
  void* base = static_scratch(c->device);
  if (!base) return fail(c, HWC_ERR_DEVICE, "the static scratch of this device was not set up");
  const ScratchSizes z = scratch_sizes(n, g, cb, needs_lv(P, flags, nullptr), hk != nullptr, needs_tcodes(P));
  Scratch S;
  const uint64_t need = carve_scratch(z, g, nullptr, &S);
  if (need > kStaticScratchBytes)
    return fail(c, HWC_ERR_ARG, "request needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                    std::to_string(kStaticScratchBytes));
  carve_scratch(z, g, static_cast<uint8_t*>(base), &S);
  if ((rc = enqueue(c, P, S, codes, cb, n, N, nullptr, hk, hc, hcap, hlen, flags, s, false))) return rc;
  HIPX(c, hipEventRecord(c->static_ev, s));
  c->static_ev_valid = true;
  return HWC_OK;
}

// ---- several requests in one persistent launch ----

// One persistent launch of a batch: sorted jobs [begin, end) and its shape.
struct BatchSeg {
  size_t begin = 0, end = 0;
  uint32_t lds = 0, block = 256, grid = 0, gmax = 1;
};

struct BatchPlan {
  std::vector<size_t> order;        // Zech-path jobs, most expensive tiles first
  std::vector<size_t> vjobs;        // matrix-product jobs (input order), launched after the batch kernel
  std::vector<DevPlan*> plans;      // per job (input order)
  std::vector<uint64_t> off, toff;  // row and tile offsets (sorted order)
  std::vector<uint64_t> max_tiles;
  std::vector<uint64_t> tco;        // byte offset of the job's dense translates, or kNoShift
  std::vector<BatchSeg> segs;       // launches over `order`
  std::vector<uint32_t> plog;       // tile parts (log2) per sorted job
  std::vector<uint64_t> aoff;       // word offset of the job's part counts in bacc
  uint64_t ntot = 0, tiles_tot = 0, nhist = 0, tbytes = 0, nlv = 0, acc_words = 0;
};


constexpr uint64_t kNoShift = ~0ull;

// Rows the batch kernel reads for sorted job r: the dense translates when its
// plan has a step table, else the caller's rows.
const void* batch_rows(const ScratchSet& st, const hwc_job& J, const BatchPlan& B, size_t r) {
  return B.tco[r] == kNoShift ? J.d_coeffs : static_cast<const void*>(static_cast<char*>(st.btcodes.p) + B.tco[r]);
}

// Every job of a batch on stream s: the Zech-path jobs in one persistent
// multi-plan launch (after their bucketing), their histograms, then each
// matrix-product job as its own launches (ordered on the same stream; in a
// captured graph they are nodes of the same graph).
int enqueue_batch(hwc_ctx* c, const hwc_job* jobs, const BatchPlan& B, const hwc::JobDesc* d_jobs, int set,
                  uint32_t flags, hipStream_t s) {
  const ScratchSet& st = c->sets[set];
  const size_t nz = B.order.size();
  if (nz) {
    uint16_t* pid = static_cast<uint16_t*>(st.bpid.p);
    uint32_t* perm = static_cast<uint32_t*>(st.bperm.p);
    uint64_t* tiles = static_cast<uint64_t*>(st.btiles.p);
    uint32_t* small = static_cast<uint32_t*>(st.bsmall.p);
    for (size_t r = 0; r < nz; ++r) {
      const hwc_job& J = jobs[B.order[r]];
      const DevPlan* P = B.plans[B.order[r]];
      uint32_t* sm = small + r * kSmallStride;
      const void* rows = batch_rows(st, J, B, r);
      const bool shifted = rows != J.d_coeffs;
      if (shifted) {   // translate and classify in one pass
        HIPX(c, hwc::launch_fill(sm, 0, hwc::pattern_count(J.g), s));
        HIPX(c, hwc::launch_shift(J.coeff_bytes, J.g, J.d_coeffs, J.n, P->q, P->d_shift, const_cast<void*>(rows),
                                  pid + B.off[r], sm, c->d_err, s));
      }
      HIPX(c, hwc::launch_bucket(J.coeff_bytes, rows, J.n, P->q, P->g, pid + B.off[r], sm, c->d_err, sm + 2048,
                                 sm + 4096, sm + 6144, sm + 8192, sm + 8196, tiles + B.toff[r], perm + B.off[r],
                                 B.max_tiles[r], shifted, s));
    }
    // the part counts and finished-part counters start at zero (a fill
    // kernel, which graph capture records as an ordinary kernel node)
    if (B.acc_words) HIPX(c, hwc::launch_fill(static_cast<uint32_t*>(st.bacc.p), 0, B.acc_words, s));
    for (const BatchSeg& G : B.segs)
      HIPX(c, hwc::launch_batch(d_jobs + G.begin, (uint32_t)(G.end - G.begin), G.gmax, G.lds, G.grid, G.block, s));
    for (size_t r = 0; r < nz; ++r) {
      const hwc_job& J = jobs[B.order[r]];
      if (!J.d_hist_keys) continue;
      HIPX(c, hwc::hist_run(J.d_out_N, nullptr, J.n, J.g, J.q, st.hist.p, J.d_hist_keys, J.d_hist_counts,
                            J.hist_capacity, J.d_hist_len, c->d_err, s));
    }
  }
  for (size_t i : B.vjobs) {
    const hwc_job& J = jobs[i];
    Scratch S{};
    S.lv = static_cast<uint32_t*>(st.lv.p);
    S.hist = st.hist.p;
    int rc = enqueue(c, B.plans[i], S, J.d_coeffs, J.coeff_bytes, J.n, J.d_out_N, nullptr, J.d_hist_keys,
                     J.d_hist_counts, J.hist_capacity, J.d_hist_len, flags, s);
    if (rc) return rc;
  }
  return HWC_OK;
}

int run_batch(hwc_ctx* c, const hwc_job* jobs, size_t njobs, uint32_t flags, hipStream_t s) {
  if (njobs == 0) return HWC_OK;
  if (njobs > 65535) return fail(c, HWC_ERR_ARG, "at most 65535 jobs per batch");
  if (flags & HWC_PLAIN) {   // the plain form is one launch per level of each job
    for (size_t i = 0; i < njobs; ++i) {
      const hwc_job& J = jobs[i];
      int rc = run_dev(c, J.q, J.g, J.d_coeffs, J.coeff_bytes, J.n, J.d_out_N, J.d_hist_keys, J.d_hist_counts,
                       J.hist_capacity, J.d_hist_len, flags, s);
      if (rc) return rc;
    }
    return HWC_OK;
  }
  int rc;
  for (size_t i = 0; i < njobs; ++i) {
    const hwc_job& J = jobs[i];
    if ((rc = check_args(c, J.q, J.g, flags))) return rc;
    if (J.coeff_bytes != 1 && J.coeff_bytes != 2) return fail(c, HWC_ERR_ARG, "coeff_bytes must be 1 or 2");
    if (J.coeff_bytes == 1 && J.q > 127) return fail(c, HWC_ERR_ARG, "int8 codes need q <= 127");
    if (J.n > 0 && (!J.d_coeffs || !J.d_out_N)) return fail(c, HWC_ERR_ARG, "null device pointer");
    if (J.d_hist_keys && (!J.d_hist_counts || !J.d_hist_len)) return fail(c, HWC_ERR_ARG, "histogram pointers");
    if (J.n >= (1ull << 31)) return fail(c, HWC_ERR_ARG, "n too large");
  }
  HIPX(c, hipSetDevice(c->device));
  BatchPlan B;
  B.plans.assign(njobs, nullptr);
  const uint32_t orbit = (flags & HWC_FULL_SWEEP) ? 0u : 1u;
  for (size_t i = 0; i < njobs; ++i) {
    rc = get_plan(c, jobs[i].q, jobs[i].g, orbit, &B.plans[i]);
    if (rc) {
      for (size_t k = 0; k < i; ++k) B.plans[k]->pins--;
      return rc;
    }
    B.plans[i]->pins++;
  }
  struct Unpin {
    BatchPlan& b;
    ~Unpin() { for (auto* p : b.plans) if (p) p->pins--; }
  } unpin{B};
  const int set = set_for(c, s);
  (void)reap(c, false);
  ScratchSet& st = c->sets[set];
  for (size_t i = 0; i < njobs; ++i) {
    if (B.plans[i]->vpath) {
      B.vjobs.push_back(i);
      const hwc_job& J = jobs[i];
      if (B.plans[i]->vpasses.size() > 1) B.nlv = std::max<uint64_t>(B.nlv, J.n * J.g);
      if (J.d_hist_keys) B.nhist = std::max<uint64_t>(B.nhist, J.n);
    } else {
      B.order.push_back(i);
    }
  }
  std::stable_sort(B.order.begin(), B.order.end(),
                   [&](size_t a, size_t b) { return B.plans[a]->tile_cost > B.plans[b]->tile_cost; });
  const size_t nz = B.order.size();
  // one launch over every job: the workgroup holds the largest image, the
  // kernel the largest genus, and the block size is the one that keeps the
  // most waves busy -- resident, and no more than there are tiles -- the
  // smaller on a tie, so that a small batch spreads over every CU instead of
  // filling a few with large workgroups.  (One launch per LDS size
  // class, so that small plans keep more workgroups per CU, measured slower
  // on the 71 fields below 300: each launch costs at least one tile's
  // latency, and the classes' tiles no longer share the CUs.)
  if (nz) {
    BatchSeg G;
    G.begin = 0;
    G.end = nz;
    for (size_t r = 0; r < nz; ++r) {
      const DevPlan* P = B.plans[B.order[r]];
      G.lds = std::max(G.lds, P->desc.image_bytes);
      G.gmax = std::max(G.gmax, P->g);
    }
    uint64_t tiles = 0;
    for (size_t k = G.begin; k < G.end; ++k) tiles += (jobs[B.order[k]].n + hwc::kWave - 1) / hwc::kWave + 4;
    int64_t best = -1;
    int bpc_best = 1;
    for (uint32_t b : {256u, 512u, 1024u}) {
      int n = 0;
      HIPX(c, hwc::occupancy_batch(G.gmax, b, G.lds, &n));
      const int64_t busy = std::min<int64_t>((int64_t)tiles, (int64_t)n * (b / hwc::kWave) * c->cus);
      if (busy > best) {
        best = busy;
        G.block = b;
        bpc_best = std::max(n, 1);
      }
    }
    G.grid = persistent_grid((uint32_t)(c->cus * bpc_best), G.block, tiles);
    B.segs.push_back(G);
  }
  for (size_t r = 0; r < nz; ++r) {
    const hwc_job& J = jobs[B.order[r]];
    const uint64_t mt = J.n / hwc::kWave + hwc::pattern_count(J.g) + 1;
    B.off.push_back(B.ntot);
    B.toff.push_back(B.tiles_tot);
    B.max_tiles.push_back(mt);
    B.ntot += J.n;
    B.tiles_tot += mt;
    const uint32_t pl = part_log(B.plans[B.order[r]], flags);
    B.plog.push_back(pl);
    B.aoff.push_back(B.acc_words);
    if (pl) B.acc_words += J.n * J.g + mt;
    if (B.plans[B.order[r]]->d_shift && J.n > 0) {
      B.tco.push_back(B.tbytes);
      B.tbytes += (J.n * (2 * J.g + 3) * J.coeff_bytes + 255) / 256 * 256;
    } else {
      B.tco.push_back(kNoShift);
    }
    if (J.d_hist_keys) B.nhist = std::max<uint64_t>(B.nhist, J.n);
  }
  if (nz) {
    if ((rc = ensure(c, set, st.bpid, std::max<uint64_t>(B.ntot, 1) * 2))) return rc;
    if ((rc = ensure(c, set, st.bperm, std::max<uint64_t>(B.ntot, 1) * 4))) return rc;
    if ((rc = ensure(c, set, st.btiles, B.tiles_tot * 8))) return rc;
    if ((rc = ensure(c, set, st.bsmall, nz * kSmallStride * 4))) return rc;
    if (B.tbytes && (rc = ensure(c, set, st.btcodes, B.tbytes))) return rc;
  }
  if (B.nhist && (rc = ensure(c, set, st.hist, hwc::hist_scratch_bytes(B.nhist)))) return rc;
  if (B.nlv && (rc = ensure(c, set, st.lv, B.nlv * 4))) return rc;
  if (B.acc_words && (rc = ensure(c, set, st.bacc, B.acc_words * 4))) return rc;
  std::vector<hwc::JobDesc> hj(std::max<size_t>(nz, 1));
  for (size_t r = 0; r < nz; ++r) {
    const hwc_job& J = jobs[B.order[r]];
    hj[r].plan = B.plans[B.order[r]]->d_desc;
    hj[r].codes = batch_rows(st, J, B, r);
    hj[r].perm = static_cast<uint32_t*>(st.bperm.p) + B.off[r];
    hj[r].tiles = static_cast<uint64_t*>(st.btiles.p) + B.toff[r];
    // the bucketing of sorted job r writes its tile count and clears its queue
    // in its words of the small scratch (launch_bucket in enqueue_batch)
    hj[r].ntiles = static_cast<uint32_t*>(st.bsmall.p) + r * kSmallStride + 8192;
    hj[r].queue = static_cast<uint32_t*>(st.bsmall.p) + r * kSmallStride + 8196;
    hj[r].outN = J.d_out_N;
    hj[r].cb = (uint32_t)J.coeff_bytes;
    hj[r].g = J.g;
    hj[r].plog = B.plog[r];
    hj[r].acc = B.plog[r] ? static_cast<uint32_t*>(st.bacc.p) + B.aoff[r] : nullptr;
    hj[r].done = B.plog[r] ? hj[r].acc + J.n * J.g : nullptr;
  }
  const size_t jbytes = std::max<size_t>(nz, 1) * sizeof(hwc::JobDesc);
  if ((rc = order_begin(c, set, s))) return rc;
  const bool use_graph = !(flags & HWC_NO_GRAPH) && !c->profile;
  if (!use_graph) {
    // job descriptors through a ring of pinned staging buffers, copied on s
    JobSlot& sl = st.slots[st.next_slot];
    st.next_slot = (st.next_slot + 1) % kJobSlots;
    if (sl.used) HIPX(c, hipEventSynchronize(sl.done));
    if (!sl.done) HIPX(c, hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    if (sl.bytes < jbytes) {
      defer_free(c, sl.p, sl.bytes);
      if (sl.h) HIPX(c, hipHostFree(sl.h));
      sl.p = sl.h = nullptr;
      sl.bytes = 0;
      const size_t want = std::max<size_t>(jbytes, 64 * sizeof(hwc::JobDesc));
      HIPX(c, hipMalloc(&sl.p, want));
      HIPX(c, hipHostMalloc(&sl.h, want, hipHostMallocDefault));
      sl.bytes = want;
    }
    std::memcpy(sl.h, hj.data(), jbytes);
    HIPX(c, hipMemcpyAsync(sl.p, sl.h, jbytes, hipMemcpyHostToDevice, s));
    rc = enqueue_batch(c, jobs, B, static_cast<const hwc::JobDesc*>(sl.p), set, flags, s);
    if (rc) return rc;
    HIPX(c, hipEventRecord(sl.done, s));
    sl.used = true;
    return order_end(c, set, s);
  }
  std::vector<uint64_t> key = {2, njobs, flags, (uint64_t)set};
  for (size_t i = 0; i < njobs; ++i) {
    const hwc_job& J = jobs[i];
    for (uint64_t v : {(uint64_t)J.q, (uint64_t)J.g, (uint64_t)(uintptr_t)J.d_coeffs, (uint64_t)J.coeff_bytes, J.n,
                       (uint64_t)(uintptr_t)J.d_out_N, (uint64_t)(uintptr_t)J.d_hist_keys,
                       (uint64_t)(uintptr_t)J.d_hist_counts, J.hist_capacity, (uint64_t)(uintptr_t)J.d_hist_len,
                       (uint64_t)(uintptr_t)B.plans[i]})
      key.push_back(v);
  }
  for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it) {
    if (it->key == key) {
      c->graphs.splice(c->graphs.begin(), c->graphs, it);
      HIPX(c, hipGraphLaunch(c->graphs.front().exec, s));
      return order_end(c, set, s);
    }
  }
  if (s != c->stream) HIPX(c, hipStreamSynchronize(c->stream));
  GraphEntry ge;
  ge.key = key;
  ge.set = set;
  ge.plans.assign(B.plans.begin(), B.plans.end());
  HIPX(c, hipMalloc(&ge.jobs, jbytes));
  hipError_t me = hipMemcpy(ge.jobs, hj.data(), jbytes, hipMemcpyHostToDevice);
  if (me != hipSuccess) {
    (void)hipFree(ge.jobs);
    return fail(c, HWC_ERR_DEVICE, std::string("job copy: ") + hipGetErrorString(me));
  }
  HIPX(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  rc = enqueue_batch(c, jobs, B, static_cast<const hwc::JobDesc*>(ge.jobs), set, flags, c->stream);
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(c->stream, &graph);
  ge.graph = graph;
  if (rc || ee != hipSuccess) {
    destroy_graph(c, ge);
    return rc ? rc : fail(c, HWC_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(ee));
  }
  hipError_t ie = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    destroy_graph(c, ge);
    return fail(c, HWC_ERR_DEVICE, std::string("instantiate: ") + hipGetErrorString(ie));
  }
  c->graphs.push_front(ge);
  while (c->graphs.size() > kMaxGraphs) {
    destroy_graph(c, c->graphs.back());
    c->graphs.pop_back();
  }
  HIPX(c, hipGraphLaunch(c->graphs.front().exec, s));
  return order_end(c, set, s);
}

// square-free test over F_q with the level-1 tables (codes are packed values)
bool squarefree_host(const hwc::Field& F, const int16_t* row, int nc) {
  const uint32_t p = F.p, M = (uint32_t)F.M;
  const uint32_t e = F.n;
  auto add = [&](uint32_t a, uint32_t b) {
    uint32_t out = 0, pw = 1;
    for (uint32_t i = 0; i < e; ++i) {
      out += ((a % p + b % p) % p) * pw;
      a /= p; b /= p; pw *= p;
    }
    return out;
  };
  auto neg = [&](uint32_t a) {
    uint32_t out = 0, pw = 1;
    for (uint32_t i = 0; i < e; ++i) { out += ((p - a % p) % p) * pw; a /= p; pw *= p; }
    return out;
  };
  auto mul = [&](uint32_t a, uint32_t b) -> uint32_t {
    if (!a || !b) return 0;
    return F.exp[(F.log[a] + F.log[b]) % M];
  };
  auto inv = [&](uint32_t a) -> uint32_t { return F.exp[(M - F.log[a]) % M]; };
  std::vector<uint32_t> A(row, row + nc), B(nc, 0);
  auto deg = [](const std::vector<uint32_t>& v, int n) { for (int i = n - 1; i >= 0; --i) if (v[i]) return i; return -1; };
  int da = deg(A, nc);
  if (da < 1) return false;
  for (int i = 1; i <= da; ++i) {
    uint32_t v = 0;
    for (uint32_t t = 0; t < (uint32_t)i % p; ++t) v = add(v, A[i]);
    B[i - 1] = v;
  }
  int db = deg(B, nc);
  if (db < 0) return false;
  while (db >= 0) {
    const uint32_t il = inv(B[db]);
    while (da >= db) {
      const uint32_t cf = neg(mul(A[da], il));
      for (int i = 0; i <= db; ++i) A[da - db + i] = add(A[da - db + i], mul(cf, B[i]));
      da = deg(A, da);
      if (da < 0) break;
    }
    std::swap(A, B);
    std::swap(da, db);
  }
  return da == 0;
}

int set_tuning_field(hwc_ctx* c, Tuning& T, int opt, int64_t value) {
  switch (opt) {
    case HWC_OPT_SPLIT: T.split = value != 0; break;
    case HWC_OPT_BLOCK:
      if (value != 0 && value != 256 && value != 512 && value != 1024)
        return fail(c, HWC_ERR_ARG, "block must be 0, 256, 512 or 1024");
      T.block = (uint32_t)value;
      break;
    case HWC_OPT_WG_PER_CU:
      if (value < 0 || value > 64) return fail(c, HWC_ERR_ARG, "workgroups per CU must be in 0..64");
      T.wg_per_cu = (uint32_t)value;
      break;
    case HWC_OPT_MFMA:
      if (value != 0 && value != 1) return fail(c, HWC_ERR_ARG, "mfma must be 0 or 1");
      T.mfma = value != 0;
      break;
    case HWC_OPT_SHIFT:
      if (value != 0 && value != 1) return fail(c, HWC_ERR_ARG, "shift must be 0 or 1");
      T.shift = value != 0;
      break;
    case HWC_OPT_SPLIT_MIN_M:
      if (value < 0 || value > (1 << 24)) return fail(c, HWC_ERR_ARG, "split threshold must be in 0..2^24");
      T.split_min_m = (uint32_t)value;
      break;
    case HWC_OPT_DEVICE_TABLES:
      if (value < 0 || value > 15) return fail(c, HWC_ERR_ARG, "device table mask must be in 0..15");
      T.device_tables = (uint32_t)value;
      break;
    case HWC_OPT_WAVES_PER_SIMD:
      if (value != 0 && value != 1 && value != 6 && value != 8)
        return fail(c, HWC_ERR_ARG, "waves per SIMD must be 0, 1, 6 or 8");
      T.wpe = (uint32_t)value;
      break;
    default: return fail(c, HWC_ERR_ARG, "unknown option");
  }
  return HWC_OK;
}

// drop cached plans (all, or the one of key) and every graph
int drop_plans(hwc_ctx* c, const std::tuple<uint32_t, uint32_t, uint32_t>* key) {
  if (c->device < 0) return HWC_OK;
  for (auto it = c->plans.begin(); it != c->plans.end();) {
    if (!key || it->first == *key) {
      c->table_bytes -= it->second->dev_bytes;
      free_plan(c, it->second.get());
      it = c->plans.erase(it);
    } else {
      ++it;
    }
  }
  return HWC_OK;
}

// ---- the map N_{g,q} of eq. (1.2) by Algorithm 1 ----
//
// Classes of reduced representatives (Sec. 1.2-1.3), per degree d:
//  * p does not divide d: a translation makes c_{d-1} = 0; i is the highest
//    nonzero position below d (i <= d-2), j the next one (or none); scalings
//    X -> aX and f -> f / e^2 put c_j / c_i in R_{i-j} and c_i in R_2.  The
//    number of polynomials behind a representative is q (q-1)^2 / (2
//    gcd(q-1, i-j)), or q (q-1) / 2 without j.  The paper's list leaves out
//    the rows c_d X^d + c_1 X (i = 1, no j); they are a class like the others.
//  * p divides d: the translation step does not reduce every row, so only
//    the scalings are used: i <= d-1, multiplicities (q-1)^2 / (2 gcd(q-1,
//    i-j)) and (q-1) / 2.
// The twist-reduced set fixes c_i = 1; each representative also stands for
// its twist n f (n a nonsquare) with the same multiplicity, whose counts
// follow from the corrected twist relation: N_k(nf) = 2(q^k+1) - N_k(f) for
// odd k, N_k(f) for even k.  Rows that are not square-free are dropped on the
// device (factorization code 0).

struct RepClass {
  uint32_t d, i;
  int32_t j;                  // -1: no j
  uint64_t nrep, mult;
  std::vector<uint32_t> cj;   // codes of R_{i-j}
};

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

std::vector<RepClass> rep_classes(const hwc::Field& Fq, uint32_t q, uint32_t p, uint32_t g) {
  std::vector<RepClass> out;
  const uint64_t qm = q - 1;
  for (uint32_t d = 2 * g + 1; d <= 2 * g + 2; ++d) {
    const bool trans = d % p != 0;
    const uint32_t imax = trans ? d - 2 : d - 1;
    for (uint32_t i = 0; i <= imax; ++i) {
      out.push_back(RepClass{d, i, -1, qm, trans ? (uint64_t)q * qm / 2 : qm / 2, {}});
      uint64_t qj = 1;
      for (uint32_t j = 0; j < i; ++j) {
        const uint64_t gk = gcd64(qm, i - j);
        RepClass c{d, i, (int32_t)j, qm * gk * qj, (trans ? (uint64_t)q : 1u) * qm * qm / (2 * gk), {}};
        for (uint64_t L = 0; L < gk; ++L) c.cj.push_back(Fq.exp[L]);   // gamma^L: codes of R_{i-j}
        out.push_back(std::move(c));
        qj *= q;
      }
    }
  }
  return out;
}

int run_map(hwc_ctx* c, uint32_t q, uint32_t g, int32_t* keys, uint64_t* counts, uint64_t capacity,
            uint64_t* out_len, uint64_t* out_reps, uint32_t flags) {
  uint32_t p, e;
  int rc = check_args(c, q, g, flags);
  if (rc) return rc;
  hwc::factor_odd_prime_power(q, &p, &e);
  if (q > hwc::kFormAMaxM + 1) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "the map needs q <= 10923");
  HIPX(c, hipSetDevice(c->device));
  auto fe = get_field(c, p, e, 1, &rc);
  if (!fe) return rc;
  const uint32_t nc = 2 * g + 3, cb = q <= 127 ? 1 : 2;
  // host key: N_1..N_g and the code in mixed radix (as the device histogram)
  std::vector<uint64_t> radix(g + 1);
  std::vector<int64_t> qpow(g);
  double bits = hwc::kLamBits;
  uint64_t qk = 1;
  for (uint32_t k = 0; k < g; ++k) {
    qk *= q;
    qpow[k] = (int64_t)qk;
    radix[k] = 2 * qk + 3;
    bits += std::log2((double)radix[k]);
  }
  radix[g] = 1ull << hwc::kLamBits;
  if (bits > 63.0) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "map key wider than 63 bits");
  const uint64_t kChunk = 1ull << 22;
  if ((rc = ensure_sync(c, c->mcodes, kChunk * nc * cb))) return rc;
  if ((rc = ensure_sync(c, c->mN, kChunk * g * 4))) return rc;
  if ((rc = ensure_sync(c, c->mlam, kChunk * 4))) return rc;
  if ((rc = ensure_sync(c, c->mhk, kChunk * (g + 1) * 4))) return rc;
  if ((rc = ensure_sync(c, c->mhc, kChunk * 8 + 64))) return rc;
  if ((rc = ensure_sync(c, c->mcj, 4096 * 4))) return rc;
  const std::vector<RepClass> classes = rep_classes(fe->F, q, p, g);
  std::unordered_map<uint64_t, uint64_t> acc;
  std::vector<int32_t> hk;
  std::vector<uint64_t> hcnt;
  uint64_t reps = 0;
  uint64_t* d_len = reinterpret_cast<uint64_t*>(static_cast<uint8_t*>(c->mhc.p) + kChunk * 8);
  HIPX(c, hwc::launch_fill(c->d_err, 0, 1, c->stream));
  for (const RepClass& cl : classes) {
    if (cl.j >= 0) {
      if (cl.cj.size() > 4096) return fail(c, HWC_ERR_ARG, "too many representatives of R_k");
      HIPX(c, hipMemcpyAsync(c->mcj.p, cl.cj.data(), cl.cj.size() * 4, hipMemcpyHostToDevice, c->stream));
    }
    for (uint64_t start = 0; start < cl.nrep; start += kChunk) {
      const uint64_t cnt = std::min(kChunk, cl.nrep - start);
      HIPX(c, hwc::launch_gen_reps((int)cb, q, nc, cl.d, cl.i, cl.j, static_cast<const uint32_t*>(c->mcj.p),
                                   (uint32_t)cl.cj.size(), start, cnt, c->mcodes.p, c->stream));
      rc = run_dev(c, q, g, c->mcodes.p, (int)cb, cnt, static_cast<int32_t*>(c->mN.p),
                   static_cast<int32_t*>(c->mhk.p), static_cast<uint64_t*>(c->mhc.p), cnt, d_len,
                   flags | HWC_NO_GRAPH | kFlagSqf, c->stream, static_cast<uint32_t*>(c->mlam.p));
      if (rc) return rc;
      uint64_t len = 0;
      HIPX(c, hipMemcpyAsync(&len, d_len, 8, hipMemcpyDeviceToHost, c->stream));
      HIPX(c, hipStreamSynchronize(c->stream));
      hk.resize(len * (g + 1));
      hcnt.resize(len);
      if (len) {
        HIPX(c, hipMemcpyAsync(hk.data(), c->mhk.p, len * (g + 1) * 4, hipMemcpyDeviceToHost, c->stream));
        HIPX(c, hipMemcpyAsync(hcnt.data(), c->mhc.p, len * 8, hipMemcpyDeviceToHost, c->stream));
        HIPX(c, hipStreamSynchronize(c->stream));
      }
      for (uint64_t r = 0; r < len; ++r) {
        const int32_t* row = hk.data() + r * (g + 1);
        const uint32_t code = (uint32_t)row[g];
        if (code == 0) continue;                       // not square-free
        const uint64_t w = hcnt[r] * cl.mult;
        uint64_t k1 = 0, k2 = 0;
        for (uint32_t k = 0; k < g; ++k) {
          const int64_t Nk = row[k];
          const int64_t Nt = (k % 2 == 0) ? 2 * (qpow[k] + 1) - Nk : Nk;   // k = 0 holds N_1 (odd degree)
          if (Nt < 0 || (uint64_t)Nt >= radix[k]) return fail(c, HWC_ERR_DEVICE, "twisted count outside its range");
          k1 = k1 * radix[k] + (uint64_t)Nk;
          k2 = k2 * radix[k] + (uint64_t)Nt;
        }
        k1 = k1 * radix[g] + code;
        k2 = k2 * radix[g] + code;
        acc[k1] += w;
        acc[k2] += w;
      }
      reps += cnt;
    }
  }
  uint32_t derr = 0;
  HIPX(c, hipMemcpy(&derr, c->d_err, 4, hipMemcpyDeviceToHost));
  if (derr & 4u) return fail(c, HWC_ERR_DEVICE, "a representative's counts or partition fall outside the key range");
  // (a_1..a_g, code) with a_k = q^k + 1 - N_k, in lexicographic order
  std::vector<std::pair<std::vector<int64_t>, uint64_t>> rows;
  rows.reserve(acc.size());
  for (const auto& kv : acc) {
    std::vector<int64_t> t(g + 1);
    uint64_t key = kv.first;
    t[g] = (int64_t)(key % radix[g]);
    key /= radix[g];
    for (int k = (int)g - 1; k >= 0; --k) {
      t[k] = qpow[k] + 1 - (int64_t)(key % radix[k]);
      key /= radix[k];
    }
    rows.emplace_back(std::move(t), kv.second);
  }
  std::sort(rows.begin(), rows.end());
  if (out_len) *out_len = rows.size();
  if (out_reps) *out_reps = reps;
  if (rows.size() > capacity) return fail(c, HWC_ERR_HIST_CAPACITY, "map longer than the capacity");
  for (size_t r = 0; r < rows.size(); ++r) {
    for (uint32_t k = 0; k <= g; ++k) keys[r * (g + 1) + k] = (int32_t)rows[r].first[k];
    counts[r] = rows[r].second;
  }
  return HWC_OK;
}

// ---- one curve over large fields (Table 1): lane-per-x ----

int single_tables(hwc_ctx* c, uint32_t p, uint32_t e, uint32_t k, std::shared_ptr<FieldEntry>* fe_out,
                  SingleTabs** out, double* build_ms, double* upload_ms) {
  int rc = HWC_OK;
  const auto t0 = std::chrono::steady_clock::now();
  auto fe = get_field(c, p, e, k, &rc);
  if (!fe) return rc;
  const auto t1 = std::chrono::steady_clock::now();
  *build_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
  *fe_out = fe;
  auto key = std::make_tuple(p, e, k);
  auto it = c->single.find(key);
  if (it != c->single.end()) {
    it->second.last_use = ++c->tick;
    *out = &it->second;
    return HWC_OK;
  }
  // keep the tables of a few fields only (each can be tens of MB)
  constexpr size_t kMaxSingleFields = 8;
  while (c->single.size() >= kMaxSingleFields) {
    HIPX(c, hipDeviceSynchronize());
    auto victim = c->single.begin();
    for (auto v = c->single.begin(); v != c->single.end(); ++v)
      if (v->second.last_use < victim->second.last_use) victim = v;
    (void)hipFree(victim->second.d_zech);
    (void)hipFree(victim->second.d_reps);
    c->single.erase(victim);
  }
  SingleTabs T;
  const hwc::Field& F = fe->F;
  HIPX(c, hipMalloc(&T.d_zech, std::max<size_t>(F.zech.size(), 1) * 4));
  HIPX(c, hipMemcpy(T.d_zech, F.zech.data(), F.zech.size() * 4, hipMemcpyHostToDevice));
  T.nreps = F.prim_reps.size();
  HIPX(c, hipMalloc(&T.d_reps, std::max<size_t>(T.nreps, 1) * 4));
  if (T.nreps) HIPX(c, hipMemcpy(T.d_reps, F.prim_reps.data(), T.nreps * 4, hipMemcpyHostToDevice));
  *upload_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
  T.last_use = ++c->tick;
  auto ins = c->single.emplace(key, T);
  *out = &ins.first->second;
  return HWC_OK;
}

int run_single(hwc_ctx* c, uint32_t q, uint32_t g, const int16_t* coeffs, uint32_t kmax, int64_t* out_N,
               double* timings, uint32_t flags) {
  if (flags & ~(HWC_FULL_SWEEP)) return fail(c, HWC_ERR_ARG, "unknown flag");
  int rc = check_args(c, q, g, flags);
  if (rc) return rc;
  if (!coeffs || !out_N) return fail(c, HWC_ERR_ARG, "null pointer");
  if (kmax < 1 || kmax > 24) return fail(c, HWC_ERR_ARG, "k must be in 1..24");
  uint32_t p, e;
  hwc::factor_odd_prime_power(q, &p, &e);
  const uint32_t nc = 2 * g + 3;
  for (uint32_t j = 0; j < nc; ++j)
    if (coeffs[j] < 0 || (uint32_t)coeffs[j] >= q) return fail(c, HWC_ERR_COEFF_RANGE, "coefficient code out of range");
  if (coeffs[nc - 1] == 0 && coeffs[nc - 2] == 0) return fail(c, HWC_ERR_DEGREE, "degree below 2g+1");
  double Qk = 1;
  for (uint32_t j = 0; j < kmax; ++j) Qk *= q;
  if (Qk > 16777216.0) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "F_{q^k} larger than 2^24 elements");
  HIPX(c, hipSetDevice(c->device));
  const bool orbit = !(flags & HWC_FULL_SWEEP);
  const uint32_t d = coeffs[nc - 1] ? nc - 1 : nc - 2;
  if ((rc = ensure_sync(c, c->hout, 64))) return rc;
  unsigned long long* d_cnt = static_cast<unsigned long long*>(c->hout.p);
  std::vector<uint64_t> z(kmax + 1), ns(kmax + 1), nx(kmax + 1);
  double build_ms = 0, upload_ms = 0, eval_ms = 0;
  hipEvent_t ev0, ev1;
  HIPX(c, hipEventCreate(&ev0));
  HIPX(c, hipEventCreate(&ev1));
  int out_rc = HWC_OK;
  for (uint32_t j = 1; j <= kmax && out_rc == HWC_OK; ++j) {
    std::shared_ptr<FieldEntry> fe;
    SingleTabs* T = nullptr;
    if ((out_rc = single_tables(c, p, e, j, &fe, &T, &build_ms, &upload_ms))) break;
    const hwc::Field& F = fe->F;
    hwc::SingleDesc f{};
    f.M = (uint32_t)F.M;
    f.d = d;
    for (uint32_t i = 0; i < nc; ++i) f.lc[i] = F.emb[(uint32_t)coeffs[i]];
    const uint64_t n = orbit ? T->nreps : F.M;
    nx[j] = n;
    unsigned long long host[2] = {0, 0};
    if (hipMemsetAsync(d_cnt, 0, 16, c->stream) != hipSuccess ||
        hipEventRecord(ev0, c->stream) != hipSuccess ||
        hwc::launch_single(T->d_zech, orbit ? T->d_reps : nullptr, n, f, d_cnt, c->stream) != hipSuccess ||
        hipEventRecord(ev1, c->stream) != hipSuccess ||
        hipMemcpyAsync(host, d_cnt, 16, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      out_rc = fail(c, HWC_ERR_DEVICE, "single-curve count failed");
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    eval_ms += ms;
    z[j] = host[0];
    ns[j] = host[1];
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (out_rc) return out_rc;
  // N_k (Sec. 1.1): affine points from the levels j | k (orbit sweep: weight j,
  // and a nonsquare of F_{q^j} is a square in F_{q^k} when k/j is even), plus
  // x = 0 and the points at infinity
  auto fq = get_field(c, p, e, 1, &rc);
  if (!fq) return rc;
  const uint32_t l0 = fq->F.emb[(uint32_t)coeffs[0]], lt = fq->F.emb[(uint32_t)coeffs[nc - 1]];
  for (uint32_t k = 1; k <= kmax; ++k) {
    int64_t N = 0;
    for (uint32_t j = 1; j <= k; ++j) {
      if (orbit ? (k % j) : (j != k)) continue;
      const uint64_t s = nx[j] - z[j] - ns[j];
      const uint64_t sq = ((k / j) % 2 == 0) ? s + ns[j] : s;
      N += (int64_t)(orbit ? j : 1) * (int64_t)(z[j] + 2 * sq);
    }
    const bool keven = k % 2 == 0;
    N += coeffs[0] == 0 ? 1 : (keven || (l0 & 1u) == 0 ? 2 : 0);
    N += coeffs[nc - 1] == 0 ? 1 : (keven || (lt & 1u) == 0 ? 2 : 0);
    out_N[k - 1] = N;
  }
  if (timings) {
    timings[0] = build_ms;
    timings[1] = upload_ms;
    timings[2] = eval_ms;
  }
  return HWC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

static thread_local std::string g_create_error;

static int create_fail(hipError_t e, const char* what) {
  g_create_error = std::string(what) + ": " + hipGetErrorString(e);
  return HWC_ERR_DEVICE;
}

int hwc_ctx_create(int device, uint64_t hbm_budget_bytes, hwc_ctx** out) {
  if (!out) return HWC_ERR_ARG;
  g_create_error.clear();
  *out = nullptr;
  auto c = std::make_unique<hwc_ctx>();
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (device >= 0) {
    int ndev = 0;
    hipError_t e;
    if ((e = hipGetDeviceCount(&ndev)) != hipSuccess) return create_fail(e, "hipGetDeviceCount");
    if (device >= ndev) return create_fail(hipErrorInvalidDevice, "device index");
    if ((e = hipSetDevice(device)) != hipSuccess) return create_fail(e, "hipSetDevice");
    if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess)
      return create_fail(e, "hipStreamCreate");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return create_fail(e, "hipGetDeviceProperties");
    c->cus = prop.multiProcessorCount;
    if ((e = hwc::prepare_kernels()) != hipSuccess) return create_fail(e, "kernel attributes");
    if ((e = hwc::prepare_vcount()) != hipSuccess) return create_fail(e, "kernel attributes");
    if ((e = hipMalloc(reinterpret_cast<void**>(&c->d_err), 256)) != hipSuccess) return create_fail(e, "hipMalloc");
    for (auto& st : c->sets)
      if ((e = hipEventCreateWithFlags(&st.ev, hipEventDisableTiming)) != hipSuccess)
        return create_fail(e, "hipEventCreate");
    if ((e = hipMemset(c->d_err, 0, 256)) != hipSuccess) return create_fail(e, "hipMemset");
    if ((e = hipEventCreateWithFlags(&c->static_ev, hipEventDisableTiming)) != hipSuccess)
      return create_fail(e, "hipEventCreate");
    if ((e = setup_static_scratch(device)) != hipSuccess) return create_fail(e, "hipGetSymbolAddress(scratch)");
  }
  *out = c.release();
  return HWC_OK;
}

void hwc_ctx_destroy(hwc_ctx* c) {
  if (!c) return;
  if (c->device >= 0) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < kSets; ++k) wait_set(c, k);
    if (c->static_ev_valid) (void)hipEventSynchronize(c->static_ev);
    drop_graphs(c);
    for (auto& kv : c->plans) free_plan(c, kv.second.get());
    (void)reap(c, true);
    for (Buf* b : {&c->N, &c->codes, &c->hout, &c->mcodes, &c->mN, &c->mlam, &c->mhk, &c->mhc, &c->mcj})
      if (b->p) (void)hipFree(b->p);
    for (auto& st : c->sets) {
      for (Buf* b : {&st.pid, &st.small, &st.tiles, &st.perm, &st.lv, &st.hist, &st.tcodes, &st.acc, &st.bpid,
                     &st.bperm, &st.btiles, &st.bsmall, &st.btcodes, &st.bacc})
        if (b->p) (void)hipFree(b->p);
      for (auto& sl : st.slots) {
        if (sl.p) (void)hipFree(sl.p);
        if (sl.h) (void)hipHostFree(sl.h);
        if (sl.done) (void)hipEventDestroy(sl.done);
      }
      if (st.ev) (void)hipEventDestroy(st.ev);
    }
    for (auto& kv : c->single) {
      if (kv.second.d_zech) (void)hipFree(kv.second.d_zech);
      if (kv.second.d_reps) (void)hipFree(kv.second.d_reps);
    }
    if (c->d_err) (void)hipFree(c->d_err);
    for (auto& ev : c->prof)
      for (auto e : ev) (void)hipEventDestroy(e);
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    if (c->static_ev) (void)hipEventDestroy(c->static_ev);
    (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

const char* hwc_last_error(const hwc_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int hwc_build_field(hwc_ctx* c, uint32_t p, uint32_t e, uint32_t k, hwc_field** out) {
  if (!c || !out) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  *out = nullptr;
  uint32_t pp, ee;
  if (!hwc::factor_odd_prime_power(p, &pp, &ee) || ee != 1) return fail(c, HWC_ERR_NOT_ODD_PRIME_POWER, "p must be an odd prime");
  if (e < 1 || k < 1) return fail(c, HWC_ERR_ARG, "e and k must be positive");
  int rc = HWC_OK;
  auto fe = get_field(c, p, e, k, &rc);
  if (!fe) return rc;
  *out = new hwc_field{fe};
  return HWC_OK;
}

int hwc_field_info(const hwc_field* f, hwc_field_desc* out) {
  if (!f || !out) return HWC_ERR_ARG;
  const hwc::Field& F = f->e->F;
  std::memset(out, 0, sizeof(*out));
  out->p = F.p; out->e = F.e; out->k = F.k; out->n = F.n;
  out->q = F.q; out->Q = F.Q;
  for (size_t i = 0; i < F.modulus.size() && i < 41; ++i) out->modulus[i] = F.modulus[i];
  for (size_t i = 0; i < F.qmodulus.size() && i < 41; ++i) out->qmodulus[i] = F.qmodulus[i];
  out->root_log = F.root_log;
  out->nprim_orbits = F.prim_reps.size();
  out->table_bytes = 4ull * (F.exp.size() + F.log.size() + F.zech.size() + F.emb.size() + F.prim_reps.size());
  return HWC_OK;
}

int hwc_field_tables(const hwc_field* f, uint32_t* exp, uint32_t* log, uint32_t* zech, uint32_t* emb,
                     uint32_t* prim_reps) {
  if (!f) return HWC_ERR_ARG;
  const hwc::Field& F = f->e->F;
  if (exp) std::memcpy(exp, F.exp.data(), F.exp.size() * 4);
  if (log) std::memcpy(log, F.log.data(), F.log.size() * 4);
  if (zech) std::memcpy(zech, F.zech.data(), F.zech.size() * 4);
  if (emb) std::memcpy(emb, F.emb.data(), F.emb.size() * 4);
  if (prim_reps) std::memcpy(prim_reps, F.prim_reps.data(), F.prim_reps.size() * 4);
  return HWC_OK;
}

void hwc_field_release(hwc_field* f) { delete f; }

int hwc_count_curves(hwc_ctx* c, uint32_t q, uint32_t g, const int16_t* coeffs, uint64_t n, int32_t* out_N,
                     hwc_hist* out_hist, uint32_t flags) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  int rc = check_args(c, q, g, flags);
  if (rc) return rc;
  if (n > 0 && !coeffs) return fail(c, HWC_ERR_ARG, "null coefficients");
  if (out_hist && (out_hist->g != g || (out_hist->capacity && (!out_hist->keys || !out_hist->counts))))
    return fail(c, HWC_ERR_ARG, "bad histogram descriptor");
  const uint32_t nc = 2 * g + 3;
  // row checks on the host: range and degree
  for (uint64_t i = 0; i < n; ++i) {
    const int16_t* r = coeffs + i * nc;
    for (uint32_t j = 0; j < nc; ++j)
      if (r[j] < 0 || (uint32_t)r[j] >= q) return fail(c, HWC_ERR_COEFF_RANGE, "coefficient code out of range");
    if (r[nc - 1] == 0 && r[nc - 2] == 0) return fail(c, HWC_ERR_DEGREE, "degree below 2g+1");
  }
  HIPX(c, hipSetDevice(c->device));
  if (flags & HWC_VALIDATE) {
    uint32_t p, e;
    hwc::factor_odd_prime_power(q, &p, &e);
    auto fe = get_field(c, p, e, 1, &rc);
    if (!fe) return rc;
    for (uint64_t i = 0; i < n; ++i)
      if (!squarefree_host(fe->F, coeffs + i * nc, (int)nc)) return fail(c, HWC_ERR_SINGULAR, "row is not square-free");
  }
  if ((rc = ensure_sync(c, c->codes, std::max<uint64_t>(n, 1) * nc * 2))) return rc;
  if ((rc = ensure_sync(c, c->N, std::max<uint64_t>(n, 1) * g * 4))) return rc;
  const bool want_hist = out_hist != nullptr;
  uint64_t cap = want_hist ? out_hist->capacity : 0;
  uint64_t* d_len = nullptr;
  if (want_hist) {
    // device histogram sized to n (the most it can need), copied back up to cap
    if ((rc = ensure_sync(c, c->hout, std::max<uint64_t>(n, 1) * (g * 4 + 8) + 64))) return rc;
  }
  if (n) HIPX(c, hipMemcpyAsync(c->codes.p, coeffs, n * nc * 2, hipMemcpyHostToDevice, c->stream));
  HIPX(c, hwc::launch_fill(c->d_err, 0, 1, c->stream));
  int32_t* dN = static_cast<int32_t*>(c->N.p);
  int32_t* dK = nullptr;
  uint64_t* dC = nullptr;
  if (want_hist) {
    uint8_t* base = static_cast<uint8_t*>(c->hout.p);
    dC = reinterpret_cast<uint64_t*>(base);
    d_len = reinterpret_cast<uint64_t*>(base + std::max<uint64_t>(n, 1) * 8);
    dK = reinterpret_cast<int32_t*>(base + std::max<uint64_t>(n, 1) * 8 + 64);
  }
  rc = run_dev(c, q, g, c->codes.p, 2, n, dN, dK, dC, std::max<uint64_t>(n, 1), d_len, flags | HWC_NO_GRAPH,
               c->stream);
  if (rc) return rc;
  uint32_t derr = 0;
  HIPX(c, hipMemcpyAsync(&derr, c->d_err, 4, hipMemcpyDeviceToHost, c->stream));
  if (out_N && n) HIPX(c, hipMemcpyAsync(out_N, dN, n * g * 4, hipMemcpyDeviceToHost, c->stream));
  uint64_t len = 0;
  if (want_hist) HIPX(c, hipMemcpyAsync(&len, d_len, 8, hipMemcpyDeviceToHost, c->stream));
  HIPX(c, hipStreamSynchronize(c->stream));
  if (derr & 1u) return fail(c, HWC_ERR_COEFF_RANGE, "coefficient code out of range");
  if (derr & 2u) return fail(c, HWC_ERR_DEGREE, "degree below 2g+1");
  if (derr & 4u) return fail(c, HWC_ERR_DEVICE, "point count outside its histogram radix");
  if (want_hist) {
    out_hist->len = len;
    const uint64_t m = std::min(len, cap);
    if (m) {
      HIPX(c, hipMemcpyAsync(out_hist->keys, dK, m * g * 4, hipMemcpyDeviceToHost, c->stream));
      HIPX(c, hipMemcpyAsync(out_hist->counts, dC, m * 8, hipMemcpyDeviceToHost, c->stream));
      HIPX(c, hipStreamSynchronize(c->stream));
    }
    if (len > cap) return fail(c, HWC_ERR_HIST_CAPACITY, "histogram capacity too small");
  }
  return HWC_OK;
}

int hwc_count_curves_dev(hwc_ctx* c, uint32_t q, uint32_t g, const void* d_coeffs, int coeff_bytes, uint64_t n,
                         int32_t* d_out_N, int32_t* d_hist_keys, uint64_t* d_hist_counts, uint64_t hist_capacity,
                         uint64_t* d_hist_len, uint32_t flags, void* stream) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (flags & HWC_VALIDATE) return fail(c, HWC_ERR_ARG, "HWC_VALIDATE needs host rows");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  return run_dev(c, q, g, d_coeffs, coeff_bytes, n, d_out_N, d_hist_keys, d_hist_counts, hist_capacity, d_hist_len,
                 flags, s);
}

int hwc_count_curves_dev_noalloc(hwc_ctx* c, uint32_t q, uint32_t g, const void* d_coeffs, int coeff_bytes,
                                 uint64_t n, int32_t* d_out_N, int32_t* d_hist_keys, uint64_t* d_hist_counts,
                                 uint64_t hist_capacity, uint64_t* d_hist_len, uint32_t flags, void* stream) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (flags & HWC_VALIDATE) return fail(c, HWC_ERR_ARG, "HWC_VALIDATE needs host rows");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  return run_dev_noalloc(c, q, g, d_coeffs, coeff_bytes, n, d_out_N, d_hist_keys, d_hist_counts, hist_capacity,
                         d_hist_len, flags, s);
}

int hwc_count_lambda_dev(hwc_ctx* c, uint32_t q, uint32_t g, const void* d_coeffs, int coeff_bytes, uint64_t n,
                         int32_t* d_out_N, uint32_t* d_out_lambda, int32_t* d_hist_keys, uint64_t* d_hist_counts,
                         uint64_t hist_capacity, uint64_t* d_hist_len, uint32_t flags, void* stream) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (flags & HWC_VALIDATE) return fail(c, HWC_ERR_ARG, "HWC_VALIDATE needs host rows");
  if (!d_out_lambda) return fail(c, HWC_ERR_ARG, "null device pointer");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  return run_dev(c, q, g, d_coeffs, coeff_bytes, n, d_out_N, d_hist_keys, d_hist_counts, hist_capacity, d_hist_len,
                 flags, s, d_out_lambda);
}

int hwc_translate_dev(hwc_ctx* c, uint32_t q, uint32_t g, const void* d_coeffs, int coeff_bytes, uint64_t n,
                      void* d_out, void* stream) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  int rc = check_args(c, q, g, 0);
  if (rc) return rc;
  if (coeff_bytes != 1 && coeff_bytes != 2) return fail(c, HWC_ERR_ARG, "coeff_bytes must be 1 or 2");
  if (coeff_bytes == 1 && q > 127) return fail(c, HWC_ERR_ARG, "int8 codes need q <= 127");
  if (n == 0) return HWC_OK;
  if (!d_coeffs || !d_out) return fail(c, HWC_ERR_ARG, "null device pointer");
  const uint64_t bytes = n * (2 * g + 3) * (uint64_t)coeff_bytes;
  const char* a = static_cast<const char*>(d_coeffs);
  const char* b = static_cast<const char*>(d_out);
  if (a < b + bytes && b < a + bytes) return fail(c, HWC_ERR_ARG, "d_out overlaps d_coeffs");
  HIPX(c, hipSetDevice(c->device));
  DevPlan* P = nullptr;
  if ((rc = get_plan(c, q, g, 1u, &P))) return rc;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  if (P->d_shift) HIPX(c, hwc::launch_shift(coeff_bytes, g, d_coeffs, n, q, P->d_shift, d_out, nullptr, nullptr, nullptr, s));
  else HIPX(c, hipMemcpyAsync(d_out, d_coeffs, bytes, hipMemcpyDeviceToDevice, s));
  return HWC_OK;
}

int hwc_count_map(hwc_ctx* c, uint32_t q, uint32_t g, int32_t* keys, uint64_t* counts, uint64_t capacity,
                  uint64_t* len, uint64_t* reps, uint32_t flags) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (flags & HWC_VALIDATE) return fail(c, HWC_ERR_ARG, "HWC_VALIDATE does not apply to the map");
  if (capacity && (!keys || !counts)) return fail(c, HWC_ERR_ARG, "null output buffer");
  return run_map(c, q, g, keys, counts, capacity, len, reps, flags);
}

int hwc_count_single(hwc_ctx* c, uint32_t q, uint32_t g, const int16_t* coeffs, uint32_t kmax, int64_t* out_N,
                     double* timings, uint32_t flags) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  return run_single(c, q, g, coeffs, kmax, out_N, timings, flags);
}

int hwc_lds_gather_rate(hwc_ctx* c, uint32_t table_entries, uint32_t chains, double* lookups_per_s) {
  if (!c || !lookups_per_s) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (c->device < 0) return fail(c, HWC_ERR_NO_DEVICE, "host-only context");
  if (table_entries < 64 || table_entries > hwc::kLdsImageLimit / 2) return fail(c, HWC_ERR_ARG, "table size");
  if (chains != 1 && chains != 2 && chains != 4) return fail(c, HWC_ERR_ARG, "chains must be 1, 2 or 4");
  HIPX(c, hipSetDevice(c->device));
  int rc;
  if ((rc = ensure_sync(c, c->hout, 64))) return rc;
  int ncu = 0;
  HIPX(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  const uint32_t grid = (uint32_t)ncu * 32, steps = 4096;
  uint32_t* sink = static_cast<uint32_t*>(c->hout.p);
  hipEvent_t e0, e1;
  HIPX(c, hipEventCreate(&e0));
  HIPX(c, hipEventCreate(&e1));
  float best = 0;
  for (int rep = 0; rep < 3; ++rep) {   // warm-up, then the best of two
    if (hipEventRecord(e0, c->stream) != hipSuccess ||
        hwc::launch_lds_gather(table_entries, chains, steps, grid, sink, c->stream) != hipSuccess ||
        hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(c, HWC_ERR_DEVICE, "gather benchmark failed");
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && (best == 0 || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *lookups_per_s = (double)grid * 256.0 * steps * chains / (best * 1e-3);
  return HWC_OK;
}

int hwc_valu_issue_rate(hwc_ctx* c, double* insts_per_s) {
  if (!c || !insts_per_s) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (c->device < 0) return fail(c, HWC_ERR_NO_DEVICE, "host-only context");
  HIPX(c, hipSetDevice(c->device));
  int rc;
  if ((rc = ensure_sync(c, c->hout, 64))) return rc;
  int ncu = 0;
  HIPX(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  const uint32_t grid = (uint32_t)ncu * 8, iters = 4096;   // 8 waves per SIMD
  uint32_t* sink = static_cast<uint32_t*>(c->hout.p);
  hipEvent_t e0, e1;
  HIPX(c, hipEventCreate(&e0));
  HIPX(c, hipEventCreate(&e1));
  float best = 0;
  for (int rep = 0; rep < 3; ++rep) {   // warm-up, then the best of two
    if (hipEventRecord(e0, c->stream) != hipSuccess ||
        hwc::launch_valu_issue(iters, grid, sink, c->stream) != hipSuccess ||
        hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(c, HWC_ERR_DEVICE, "issue-rate benchmark failed");
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && (best == 0 || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // wave64 instructions: waves x iterations x 192
  *insts_per_s = (double)grid * (256 / hwc::kWave) * iters * 192.0 / (best * 1e-3);
  return HWC_OK;
}

int hwc_device_gather_rate(hwc_ctx* c, uint64_t table_entries, uint32_t chains, double* lookups_per_s) {
  if (!c || !lookups_per_s) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (c->device < 0) return fail(c, HWC_ERR_NO_DEVICE, "host-only context");
  if (table_entries < 64 || table_entries > (1ull << 26)) return fail(c, HWC_ERR_ARG, "table size");
  if (chains != 1 && chains != 2 && chains != 4) return fail(c, HWC_ERR_ARG, "chains must be 1, 2 or 4");
  HIPX(c, hipSetDevice(c->device));
  int rc;
  if ((rc = ensure_sync(c, c->hout, 64))) return rc;
  if ((rc = ensure_sync(c, c->N, table_entries * 4))) return rc;
  int ncu = 0;
  HIPX(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  const uint32_t grid = (uint32_t)ncu * 32, steps = 256, n = (uint32_t)table_entries;
  uint32_t* tab = static_cast<uint32_t*>(c->N.p);
  uint32_t* sink = static_cast<uint32_t*>(c->hout.p);
  HIPX(c, hwc::launch_dev_table_fill(tab, n, c->stream));
  hipEvent_t e0, e1;
  HIPX(c, hipEventCreate(&e0));
  HIPX(c, hipEventCreate(&e1));
  float best = 0;
  for (int rep = 0; rep < 3; ++rep) {   // warm-up, then the best of two
    if (hipEventRecord(e0, c->stream) != hipSuccess ||
        hwc::launch_dev_gather(tab, n, chains, steps, grid, sink, c->stream) != hipSuccess ||
        hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(c, HWC_ERR_DEVICE, "gather benchmark failed");
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && (best == 0 || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *lookups_per_s = (double)grid * 256.0 * steps * chains / (best * 1e-3);
  return HWC_OK;
}

int hwc_count_batch(hwc_ctx* c, const hwc_job* jobs, size_t njobs, uint32_t flags, void* stream) {
  if (!c || (njobs && !jobs)) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (flags & HWC_VALIDATE) return fail(c, HWC_ERR_ARG, "HWC_VALIDATE needs host rows");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  return run_batch(c, jobs, njobs, flags, s);
}

int hwc_ctx_status(hwc_ctx* c, void* stream) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->device < 0) return HWC_OK;
  HIPX(c, hipSetDevice(c->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  HIPX(c, hipStreamSynchronize(s));
  HIPX(c, hipStreamSynchronize(c->stream));
  uint32_t derr = 0;
  HIPX(c, hipMemcpy(&derr, c->d_err, 4, hipMemcpyDeviceToHost));
  HIPX(c, hwc::launch_fill(c->d_err, 0, 1, c->stream));
  HIPX(c, hipStreamSynchronize(c->stream));
  if (derr & 1u) return fail(c, HWC_ERR_COEFF_RANGE, "coefficient code out of range");
  if (derr & 2u) return fail(c, HWC_ERR_DEGREE, "degree below 2g+1");
  if (derr & 4u) return fail(c, HWC_ERR_DEVICE, "point count outside its histogram radix");
  return HWC_OK;
}

int hwc_ctx_profile(hwc_ctx* c, int enable) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->profile = enable != 0;
  return HWC_OK;
}

int hwc_ctx_profile_read(hwc_ctx* c, double* prep_ms, double* count_ms, double* hist_ms, uint64_t* calls) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  double t[3] = {0, 0, 0};
  for (auto& ev : c->prof) {
    HIPX(c, hipEventSynchronize(ev[3]));
    for (int i = 0; i < 3; ++i) {
      float ms = 0;
      HIPX(c, hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      t[i] += ms;
    }
    for (auto e : ev) c->event_pool.push_back(e);
  }
  if (calls) *calls = c->prof.size();
  c->prof.clear();
  if (prep_ms) *prep_ms = t[0];
  if (count_ms) *count_ms = t[1];
  if (hist_ms) *hist_ms = t[2];
  return HWC_OK;
}

int hwc_ctx_set_option(hwc_ctx* c, int opt, int64_t value) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  int rc = set_tuning_field(c, c->defaults, opt, value);
  if (rc) return rc;
  return drop_plans(c, nullptr);
}

int hwc_ctx_set_plan_option(hwc_ctx* c, uint32_t q, uint32_t g, uint32_t flags, int opt, int64_t value) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  const auto key = std::make_tuple(q, g, (flags & HWC_FULL_SWEEP) ? 0u : 1u);
  auto it = c->tuned.find(key);
  Tuning T = it != c->tuned.end() ? it->second : c->defaults;
  int rc = set_tuning_field(c, T, opt, value);
  if (rc) return rc;
  c->tuned[key] = T;
  return drop_plans(c, &key);
}

int hwc_plan_info(hwc_ctx* c, uint32_t q, uint32_t g, uint32_t flags, hwc_level_desc* levels) {
  if (!c || !levels) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  int rc = check_args(c, q, g, flags);
  if (rc) return rc;
  HIPX(c, hipSetDevice(c->device));
  DevPlan* P = nullptr;
  if ((rc = get_plan(c, q, g, (flags & HWC_FULL_SWEEP) ? 0u : 1u, &P))) return rc;
  for (uint32_t j = 0; j < g; ++j) {
    const hwc::LevelDesc& L = P->desc.lv[j];
    levels[j].M = L.M;
    levels[j].form = L.form;
    levels[j].nx = L.nx;
    levels[j].weight = L.weight;
    levels[j].msplit = L.msplit;
    levels[j].nt = L.nt;
    levels[j].ns = L.ns;
    uint32_t vmax = 0;
    for (const auto& v : P->vpasses) vmax = std::max(vmax, v.desc.image_bytes);
    levels[j].lds_bytes = P->vpath ? vmax : P->desc.image_bytes;
    levels[j].mfma = 0;
    for (const auto& v : P->vpasses)
      if (P->vpath && v.lo <= j && j <= v.hi) levels[j].mfma = v.desc.bal ? 2u : 1u;
  }
  return HWC_OK;
}

int hwc_ctx_stats(const hwc_ctx* c, uint64_t* plans_resident, uint64_t* table_bytes, uint64_t* cache_hits,
                  uint64_t* cache_misses, uint64_t* evictions, uint64_t* pending_free_bytes) {
  if (!c) return HWC_ERR_ARG;
  if (plans_resident) *plans_resident = c->plans.size();
  if (table_bytes) *table_bytes = c->table_bytes;
  if (cache_hits) *cache_hits = c->hits;
  if (cache_misses) *cache_misses = c->misses;
  if (evictions) *evictions = c->evictions;
  if (pending_free_bytes) *pending_free_bytes = c->grave_bytes;
  return HWC_OK;
}

int hwc_ctx_reserve(hwc_ctx* c, uint64_t max_curves, uint32_t max_jobs, void* stream) {
  if (!c) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (c->device < 0) return fail(c, HWC_ERR_NO_DEVICE, "host-only context");
  if (max_curves >= (1ull << 31) || max_jobs < 1 || max_jobs > 65535) return fail(c, HWC_ERR_ARG, "reserve sizes");
  HIPX(c, hipSetDevice(c->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  const int set = set_for(c, s);
  ScratchSet& st = c->sets[set];
  const uint64_t N = std::max<uint64_t>(max_curves, 1), J = max_jobs;
  // one request of N rows at the largest genus and code width, every optional part
  const ScratchSizes z = scratch_sizes(N, hwc::kMaxG, 2, true, true, true, true);
  int rc;
  if ((rc = ensure(c, set, st.pid, z.pid))) return rc;
  if ((rc = ensure(c, set, st.small, z.small))) return rc;
  if ((rc = ensure(c, set, st.tiles, z.tiles))) return rc;
  if ((rc = ensure(c, set, st.perm, z.perm))) return rc;
  if ((rc = ensure(c, set, st.lv, z.lv))) return rc;
  if ((rc = ensure(c, set, st.hist, z.hist))) return rc;
  if ((rc = ensure(c, set, st.tcodes, z.tcodes))) return rc;
  if ((rc = ensure(c, set, st.acc, z.acc))) return rc;
  // a multi-plan batch of N rows over at most J jobs (run_batch's sizes, bounded
  // with every job at the largest genus)
  const uint64_t tiles = N / hwc::kWave + J * (hwc::pattern_count(hwc::kMaxG) + 1);
  if ((rc = ensure(c, set, st.bpid, N * 2))) return rc;
  if ((rc = ensure(c, set, st.bperm, N * 4))) return rc;
  if ((rc = ensure(c, set, st.btiles, tiles * 8))) return rc;
  if ((rc = ensure(c, set, st.bsmall, J * kSmallStride * 4))) return rc;
  if ((rc = ensure(c, set, st.btcodes, N * (2 * hwc::kMaxG + 3) * 2 + J * 256))) return rc;
  if ((rc = ensure(c, set, st.bacc, (N * hwc::kMaxG + tiles) * 4))) return rc;
  const size_t jbytes = std::max<size_t>(J, 64) * sizeof(hwc::JobDesc);
  for (auto& sl : st.slots) {
    if (sl.bytes >= jbytes) continue;
    if (sl.used) HIPX(c, hipEventSynchronize(sl.done));
    if (!sl.done) HIPX(c, hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    defer_free(c, sl.p, sl.bytes);
    if (sl.h) HIPX(c, hipHostFree(sl.h));
    sl.p = sl.h = nullptr;
    sl.bytes = 0;
    HIPX(c, hipMalloc(&sl.p, jbytes));
    HIPX(c, hipHostMalloc(&sl.h, jbytes, hipHostMallocDefault));
    sl.bytes = jbytes;
  }
  return HWC_OK;
}

}  // extern "C"
