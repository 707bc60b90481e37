// C ABI of libhwcount.so (declared in include/hwcount.h).
//
// A context owns a HIP stream, a cache of built fields, a cache of device
// plans (one per (q, g, sweep mode): the LDS image of all level tables plus
// the x lists), scratch buffers and captured HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hwcount.h"
#include "field.h"
#include "plan.h"

namespace hwc {
hipError_t launch_count(const PlanDesc& P, int coeff_bytes, const void* codes, const uint32_t* perm,
                        const uint64_t* tiles, const uint32_t* ntiles, uint32_t* queue, uint32_t lo, uint32_t hi,
                        int32_t* outN, uint32_t* outLv, uint32_t grid, uint32_t block, hipStream_t s);
hipError_t occupancy_count(uint32_t g, int coeff_bytes, uint32_t block, uint32_t lds_bytes, int* blocks_per_cu);
hipError_t prepare_kernels();
hipError_t launch_assemble(const PlanDesc& P, int coeff_bytes, const void* codes, uint64_t n, const uint32_t* lv,
                           int32_t* outN, hipStream_t s);
hipError_t launch_fill(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t launch_bucket(int coeff_bytes, const void* codes, uint64_t n, uint32_t q, uint32_t g, uint16_t* pid,
                         uint32_t* counts, uint32_t* err, uint32_t* bucket_start, uint32_t* tile_start,
                         uint32_t* cursor, uint32_t* ntiles, uint32_t* queue, uint64_t* tiles, uint32_t* perm,
                         uint64_t max_tiles, hipStream_t s);
uint64_t hist_scratch_bytes(uint64_t n);
hipError_t hist_run(const int32_t* N, uint64_t n, uint32_t g, uint32_t q, void* scratch, int32_t* out_keys,
                    uint64_t* out_counts, uint64_t cap, uint64_t* out_len, uint32_t* err, hipStream_t s);
}  // namespace hwc

namespace {

constexpr uint32_t kLdsLimit = 160 * 1024;
constexpr size_t kMaxGraphs = 8;

struct FieldEntry {
  hwc::Field F;
};

struct DevPlan {
  uint32_t q = 0, g = 0, orbit = 0;
  std::vector<std::shared_ptr<FieldEntry>> fields;
  std::vector<uint32_t> image;  // dwords
  hwc::PlanDesc desc{};
  void* d_image = nullptr;
  std::vector<uint32_t*> d_reps;
  uint64_t dev_bytes = 0;
  uint64_t last_use = 0;
  uint32_t block = 256, grid = 0;
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct GraphKey {
  const DevPlan* plan;
  uint64_t n;
  int cb;
  const void* codes;
  const int32_t* N;
  const int32_t* hk;
  const uint64_t* hc;
  uint64_t hcap;
  const uint64_t* hlen;
  uint32_t flags;
  bool operator==(const GraphKey& o) const {
    return plan == o.plan && n == o.n && cb == o.cb && codes == o.codes && N == o.N && hk == o.hk && hc == o.hc &&
           hcap == o.hcap && hlen == o.hlen && flags == o.flags;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

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
  uint64_t table_bytes = 0, hits = 0, misses = 0, tick = 0;
  int cus = 0;
  // scratch
  Buf pid, small, tiles, perm, lv, N, hist, codes, hout;
  uint32_t* d_err = nullptr;
  std::list<GraphEntry> graphs;
  // profiling: events around the phases of each direct (non-graph) call
  bool profile = false;
  std::vector<std::array<hipEvent_t, 4>> prof;
  std::vector<hipEvent_t> event_pool;
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

void drop_graphs(hwc_ctx* c) {
  for (auto& g : c->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  c->graphs.clear();
}

int ensure(hwc_ctx* c, Buf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return HWC_OK;
  drop_graphs(c);  // captured graphs may hold the old pointer
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

void free_plan(DevPlan* P) {
  if (P->d_image) (void)hipFree(P->d_image);
  for (auto* r : P->d_reps)
    if (r) (void)hipFree(r);
  P->d_image = nullptr;
  P->d_reps.clear();
}

uint32_t align16(uint32_t v) { return (v + 15u) & ~15u; }

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
  if (q > 32768) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "q too large");
  // sizes first, so oversize requests fail before any table is built
  uint64_t Mj = 1, lds = 0;
  for (uint32_t j = 1; j <= g; ++j) {
    Mj = Mj * q;
    const uint64_t M = Mj - 1;
    if (M > hwc::kFormCMaxM) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "F_{q^g} is too large for the LDS-resident tables");
    lds += align16((uint32_t)((M <= hwc::kFormAMaxM ? 5 * M : 2 * M) * 2)) + align16((uint32_t)(2 * q));
  }
  if (lds > kLdsLimit) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "tables of F_q..F_{q^g} exceed 160 KiB of LDS");
  auto P = std::make_unique<DevPlan>();
  P->q = q; P->g = g; P->orbit = orbit;
  int rc = HWC_OK;
  for (uint32_t j = 1; j <= g; ++j) {
    auto fe = get_field(c, p, e, j, &rc);
    if (!fe) return rc;
    P->fields.push_back(fe);
  }
  // LDS image: level tables, then embedding tables
  std::vector<uint16_t> img;
  auto put = [&](const std::vector<uint16_t>& v) {
    uint32_t off = (uint32_t)img.size() * 2;
    img.insert(img.end(), v.begin(), v.end());
    while ((img.size() * 2) % 16) img.push_back(0);
    return off;
  };
  hwc::PlanDesc& D = P->desc;
  D.q = q; D.g = g; D.ncoef = 2 * g + 3; D.orbit = orbit;
  for (uint32_t j = 0; j < g; ++j) {
    const hwc::Field& F = P->fields[j]->F;
    const uint32_t M = (uint32_t)F.M;
    hwc::LevelDesc& L = D.lv[j];
    L.M = M;
    std::vector<uint16_t> tab;
    if (M <= hwc::kFormAMaxM) {
      L.form = hwc::kFormA;
      tab.assign(5 * (size_t)M, 0);
      for (uint32_t i = 0; i < 3 * M; ++i) {
        const uint32_t z = F.zech[i % M];
        tab[i] = (uint16_t)(z == M ? 6 * M : 2 * z);
      }
    } else {
      L.form = hwc::kFormC;
      tab.resize(2 * (size_t)M);
      for (uint32_t i = 0; i < 2 * M; ++i) tab[i] = (uint16_t)F.zech[i % M];
    }
    L.tab_off = put(tab);
    if (orbit) {
      L.nx = (uint32_t)F.prim_reps.size();
      L.weight = j + 1;
    } else {
      L.nx = M;
      L.weight = 1;
    }
  }
  for (uint32_t j = 0; j < g; ++j) {
    const hwc::Field& F = P->fields[j]->F;
    std::vector<uint16_t> emb(F.emb.begin(), F.emb.end());
    D.lv[j].emb_off = put(emb);
  }
  D.image_bytes = (uint32_t)img.size() * 2;
  if (D.image_bytes > kLdsLimit) return fail(c, HWC_ERR_FIELD_TOO_LARGE, "LDS image too large");
  P->image.assign(img.size() / 2, 0);
  std::memcpy(P->image.data(), img.data(), img.size() * 2);
  // device memory for the plan, admitted against the budget
  uint64_t bytes = D.image_bytes;
  if (orbit)
    for (uint32_t j = 0; j < g; ++j) bytes += P->fields[j]->F.prim_reps.size() * 4;
  if (c->budget) {
    while (c->table_bytes + bytes > c->budget && !c->plans.empty()) {
      auto victim = c->plans.begin();
      for (auto i2 = c->plans.begin(); i2 != c->plans.end(); ++i2)
        if (i2->second->last_use < victim->second->last_use) victim = i2;
      drop_graphs(c);
      HIPX(c, hipStreamSynchronize(c->stream));
      c->table_bytes -= victim->second->dev_bytes;
      free_plan(victim->second.get());
      c->plans.erase(victim);
    }
    if (c->table_bytes + bytes > c->budget)
      return fail(c, HWC_ERR_OOM_BUDGET, "tables exceed the context's HBM budget");
  }
  HIPX(c, hipMalloc(&P->d_image, D.image_bytes));
  HIPX(c, hipMemcpy(P->d_image, P->image.data(), D.image_bytes, hipMemcpyHostToDevice));
  D.image = static_cast<const uint32_t*>(P->d_image);
  P->d_reps.assign(g, nullptr);
  for (uint32_t j = 0; j < g; ++j) {
    if (!orbit) { D.lv[j].xs = nullptr; continue; }
    const auto& reps = P->fields[j]->F.prim_reps;
    HIPX(c, hipMalloc(&P->d_reps[j], std::max<size_t>(reps.size(), 1) * 4));
    if (!reps.empty()) HIPX(c, hipMemcpy(P->d_reps[j], reps.data(), reps.size() * 4, hipMemcpyHostToDevice));
    D.lv[j].xs = P->d_reps[j];
  }
  P->dev_bytes = bytes;
  c->table_bytes += bytes;
  // launch shape: many waves per CU; one large block when the tables fill LDS
  P->block = D.image_bytes > 80 * 1024 ? 1024 : 256;
  int bpc = 0;
  HIPX(c, hwc::occupancy_count(g, 1, P->block, D.image_bytes, &bpc));
  if (bpc < 1) bpc = 1;
  P->grid = (uint32_t)(c->cus * bpc);
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
  uint64_t max_tiles;
};

int get_scratch(hwc_ctx* c, uint64_t n, uint32_t g, bool plain, bool hist, Scratch* s) {
  const uint32_t npat = hwc::pattern_count(g);
  s->max_tiles = n / hwc::kWave + npat + 1;
  int rc;
  if ((rc = ensure(c, c->pid, std::max<uint64_t>(n, 1) * 2))) return rc;
  if ((rc = ensure(c, c->small, (size_t)(4 * npat + 16) * 4))) return rc;
  if ((rc = ensure(c, c->tiles, s->max_tiles * 8))) return rc;
  if ((rc = ensure(c, c->perm, std::max<uint64_t>(n, 1) * 4))) return rc;
  if (plain && (rc = ensure(c, c->lv, std::max<uint64_t>(n, 1) * g * 4))) return rc;
  if (hist && (rc = ensure(c, c->hist, hwc::hist_scratch_bytes(n)))) return rc;
  s->pid = static_cast<uint16_t*>(c->pid.p);
  uint32_t* sm = static_cast<uint32_t*>(c->small.p);
  s->counts = sm;
  s->bucket_start = sm + npat;
  s->tile_start = sm + 2 * npat;
  s->cursor = sm + 3 * npat;
  s->ntiles = sm + 4 * npat;
  s->queue = sm + 4 * npat + 4;
  s->tiles = static_cast<uint64_t*>(c->tiles.p);
  s->perm = static_cast<uint32_t*>(c->perm.p);
  s->lv = plain ? static_cast<uint32_t*>(c->lv.p) : nullptr;
  s->hist = hist ? c->hist.p : nullptr;
  return HWC_OK;
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
            int32_t* hk, uint64_t* hc, uint64_t hcap, uint64_t* hlen, uint32_t flags, hipStream_t s,
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
  HIPX(c, hwc::launch_bucket(cb, codes, n, P->q, g, S.pid, S.counts, c->d_err, S.bucket_start, S.tile_start,
                             S.cursor, S.ntiles, S.queue, S.tiles, S.perm, S.max_tiles, s));
  if (record) HIPX(c, hipEventRecord(ev[1], s));
  if (n > 0) {
    if (flags & HWC_PLAIN) {
      for (uint32_t j = 0; j < g; ++j)
        HIPX(c, hwc::launch_count(P->desc, cb, codes, S.perm, S.tiles, S.ntiles, nullptr, j, j, nullptr, S.lv,
                                  P->grid, P->block, s));
      HIPX(c, hwc::launch_assemble(P->desc, cb, codes, n, S.lv, N, s));
    } else {
      HIPX(c, hwc::launch_count(P->desc, cb, codes, S.perm, S.tiles, S.ntiles, S.queue, 0, g - 1, N, nullptr,
                                P->grid, P->block, s));
    }
  }
  if (record) HIPX(c, hipEventRecord(ev[2], s));
  if (hk) HIPX(c, hwc::hist_run(N, n, g, P->q, S.hist, hk, hc, hcap, hlen, c->d_err, s));
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

int run_dev(hwc_ctx* c, uint32_t q, uint32_t g, const void* codes, int cb, uint64_t n, int32_t* N, int32_t* hk,
            uint64_t* hc, uint64_t hcap, uint64_t* hlen, uint32_t flags, hipStream_t s) {
  int rc = check_args(c, q, g, flags);
  if (rc) return rc;
  if (cb != 1 && cb != 2) return fail(c, HWC_ERR_ARG, "coeff_bytes must be 1 or 2");
  if (cb == 1 && q > 127) return fail(c, HWC_ERR_ARG, "int8 codes need q <= 127");
  if (n > 0 && (!codes || !N)) return fail(c, HWC_ERR_ARG, "null device pointer");
  if (hk && (!hc || !hlen)) return fail(c, HWC_ERR_ARG, "histogram needs counts and length pointers");
  if (n >= (1ull << 31)) return fail(c, HWC_ERR_ARG, "n too large");
  HIPX(c, hipSetDevice(c->device));
  DevPlan* P = nullptr;
  if ((rc = get_plan(c, q, g, (flags & HWC_FULL_SWEEP) ? 0u : 1u, &P))) return rc;
  Scratch S;
  if ((rc = get_scratch(c, n, g, (flags & HWC_PLAIN) != 0, hk != nullptr, &S))) return rc;
  const bool use_graph = !(flags & (HWC_PLAIN | HWC_NO_GRAPH)) && n > 0 && !c->profile;
  if (!use_graph) return enqueue(c, P, S, codes, cb, n, N, hk, hc, hcap, hlen, flags, s, c->profile);
  GraphKey key{P, n, cb, codes, N, hk, hc, hcap, hlen, flags};
  for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it) {
    if (it->key == key) {
      c->graphs.splice(c->graphs.begin(), c->graphs, it);
      HIPX(c, hipGraphLaunch(c->graphs.front().exec, s));
      return HWC_OK;
    }
  }
  // capture on the context stream, replay on s
  if (s != c->stream) HIPX(c, hipStreamSynchronize(c->stream));
  GraphEntry ge;
  ge.key = key;
  HIPX(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  rc = enqueue(c, P, S, codes, cb, n, N, hk, hc, hcap, hlen, flags, c->stream);
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
    auto& b = c->graphs.back();
    (void)hipGraphExecDestroy(b.exec);
    (void)hipGraphDestroy(b.graph);
    c->graphs.pop_back();
  }
  HIPX(c, hipGraphLaunch(c->graphs.front().exec, s));
  return HWC_OK;
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

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

int hwc_ctx_create(int device, uint64_t hbm_budget_bytes, hwc_ctx** out) {
  if (!out) return HWC_ERR_ARG;
  *out = nullptr;
  auto c = std::make_unique<hwc_ctx>();
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (device >= 0) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return HWC_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return HWC_ERR_DEVICE;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return HWC_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HWC_ERR_DEVICE;
    c->cus = prop.multiProcessorCount;
    if (hwc::prepare_kernels() != hipSuccess) return HWC_ERR_DEVICE;
    if (hipMalloc(reinterpret_cast<void**>(&c->d_err), 256) != hipSuccess) return HWC_ERR_DEVICE;
    if (hipMemset(c->d_err, 0, 256) != hipSuccess) return HWC_ERR_DEVICE;
  }
  *out = c.release();
  return HWC_OK;
}

void hwc_ctx_destroy(hwc_ctx* c) {
  if (!c) return;
  if (c->device >= 0) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (auto& kv : c->plans) free_plan(kv.second.get());
    for (Buf* b : {&c->pid, &c->small, &c->tiles, &c->perm, &c->lv, &c->N, &c->hist, &c->codes, &c->hout})
      if (b->p) (void)hipFree(b->p);
    if (c->d_err) (void)hipFree(c->d_err);
    for (auto& ev : c->prof)
      for (auto e : ev) (void)hipEventDestroy(e);
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

const char* hwc_last_error(const hwc_ctx* c) { return c ? c->err.c_str() : "null context"; }

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
  if ((rc = ensure(c, c->codes, std::max<uint64_t>(n, 1) * nc * 2))) return rc;
  if ((rc = ensure(c, c->N, std::max<uint64_t>(n, 1) * g * 4))) return rc;
  const bool want_hist = out_hist != nullptr;
  uint64_t cap = want_hist ? out_hist->capacity : 0;
  uint64_t* d_len = nullptr;
  if (want_hist) {
    // device histogram sized to n (the most it can need), copied back up to cap
    if ((rc = ensure(c, c->hout, std::max<uint64_t>(n, 1) * (g * 4 + 8) + 64))) return rc;
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

int hwc_count_batch(hwc_ctx* c, const hwc_job* jobs, size_t njobs, uint32_t flags, void* stream) {
  if (!c || (njobs && !jobs)) return HWC_ERR_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (flags & HWC_VALIDATE) return fail(c, HWC_ERR_ARG, "HWC_VALIDATE needs host rows");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  for (size_t i = 0; i < njobs; ++i) {
    const hwc_job& J = jobs[i];
    int rc = run_dev(c, J.q, J.g, J.d_coeffs, J.coeff_bytes, J.n, J.d_out_N, J.d_hist_keys, J.d_hist_counts,
                     J.hist_capacity, J.d_hist_len, flags, s);
    if (rc) return rc;
  }
  return HWC_OK;
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

int hwc_ctx_stats(const hwc_ctx* c, uint64_t* plans_resident, uint64_t* table_bytes, uint64_t* cache_hits,
                  uint64_t* cache_misses) {
  if (!c) return HWC_ERR_ARG;
  if (plans_resident) *plans_resident = c->plans.size();
  if (table_bytes) *table_bytes = c->table_bytes;
  if (cache_hits) *cache_hits = c->hits;
  if (cache_misses) *cache_misses = c->misses;
  return HWC_OK;
}

}  // extern "C"
