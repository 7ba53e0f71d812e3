// C-ABI of libpmc (declared in include/pmc.h): contexts, payoff loading,
// pricing launches (single, batched persistent with graph replay), parity
// hooks and the batch autotuner.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pmc.h"
#include "codegen.h"
#include "ctx.h"
#include "ilc.h"
#include "kernels.h"

using namespace pmc;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  ~DevBuf() { if (p) (void)hipFree(p); }
  hipError_t ensure(size_t n) {
    if (n <= cap) return hipSuccess;
    if (p) { (void)hipFree(p); p = nullptr; cap = 0; }
    size_t want = std::max<size_t>(n, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) cap = want;
    return e;
  }
};

struct HostPinned {
  void* p = nullptr;
  void* dev = nullptr;   // the device's address of the same memory
  size_t cap = 0;
  unsigned flags = hipHostMallocDefault;
  ~HostPinned() { if (p) (void)hipHostFree(p); }
  hipError_t ensure(size_t n) {
    if (n <= cap) return hipSuccess;
    if (p) { (void)hipHostFree(p); p = nullptr; dev = nullptr; cap = 0; }
    size_t want = std::max<size_t>(n, 4096);
    hipError_t e = hipHostMalloc(&p, want, flags);
    if (e != hipSuccess) return e;
    cap = want;
    return hipHostGetDevicePointer(&dev, p, 0);
  }
};

// A packed upload: several host arrays placed at aligned offsets of one
// device blob, copied with a single async H2D transfer.
struct Pack {
  std::vector<uint8_t> bytes;
  size_t add(const void* src, size_t n) {
    size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + n);
    if (n) std::memcpy(bytes.data() + off, src, n);
    return off;
  }
};

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  std::vector<uint8_t> key;
  ~GraphCache() { if (exec) (void)hipGraphExecDestroy(exec); }
};

// A batched launch, ready to run: launch arguments, grid and tile, and what
// the results need.
struct BatchPlan {
  McLaunch L;
  int grid = 0, block = 256, ppt = 1, n_inst = 0, mode = PMC_MODE_FUSED, full = 0;
  int lanes = 1;                // paths per lane (streamed paths only)
  bool stream = false;          // paths generated as a stream
  bool spec = false;            // one template environment shared by all instances:
  std::vector<int32_t> tenv;   // that environment (and a trailing 0)
  std::vector<uint64_t> n_paths;
  std::vector<int> n_slots;
  int64_t path_dates = 0;
};

}  // namespace

struct pmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  DevBuf blob, partial, bad, counters, paths, sobol, chol, sobol_hi;
  // Results, written by the kernels straight into coherent host memory:
  // n_inst (sum, sum of squares) pairs, then n_inst Cholesky status words.
  HostPinned results{nullptr, nullptr, 0, hipHostMallocCoherent | hipHostMallocMapped};
  int sobol_hi_rows = 0, sobol_hi_dims = 0, sobol_hi_bits = 0;
  std::vector<uint8_t> last_upload;   // bytes the blob holds (skip identical uploads)
  HostPinned staging;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evk[3] = {nullptr, nullptr, nullptr};   // around the generation and pricing kernels
  int sobol_dims = 0;
  int n_cu = 0;
  std::string device_name;
  GraphCache graph;
  struct Tile { int block, ppt, lanes; };
  std::map<std::string, Tile> tuned;  // batch shape -> tile
  std::map<std::string, int> occupancy;   // kernel variant and block size -> resident blocks per CU
  // Bumped whenever the device tables change content: an upload that
  // rewrites the blob, new direction numbers, a rebuilt Sobol high table.
  uint64_t table_gen = 0;
  // The last fused single-instrument pricing's host-side preparation
  // (tables, launch arguments, kernel and grid), reused by a call whose
  // inputs are byte-identical while the tables and buffers are unchanged.
  // Every kernel still runs; only the marshalling is skipped.
  struct Prepared {
    bool valid = false;
    std::vector<uint8_t> key;     // the call's inputs, serialized
    uint64_t gen = 0;             // table_gen it was built under
    const void* bufs[8] = {};     // device buffers its launch arguments point into
    pmc::McLaunch L{};
    pmc::EngineLaunch e{};
    uint64_t n_paths = 0;
    int n_slots = 0;
    int engine = 0;
  } prepared;
  // The same for the last batch: a call whose inputs and tile are
  // byte-identical, with the tables and buffers unchanged since, replays its
  // graph without rebuilding the instance tables.
  struct PreparedBatch {
    bool valid = false;
    std::vector<uint8_t> key;
    uint64_t gen = 0;
    const void* bufs[8] = {};
    BatchPlan bp;
  } prepared_batch;
  std::vector<uint8_t> key_buf;   // scratch for a call's key
  // The device address of the allocation-free call's scratch on this
  // device (null, with the reason, if the lookup failed).
  void* scratch = nullptr;
  std::string scratch_err;
};

static uint64_t next_payoff_serial() {
  static std::atomic<uint64_t> n{0};
  return ++n;
}

struct pmc_payoff {
  Program prog;
  uint64_t hash = 0;
  // Never reused (unlike the object's address): prepared calls name their
  // payoff by it, so a freed payoff's kernels can never be launched again.
  const uint64_t serial = next_payoff_serial();
  mutable JitCache jit;   // compiled-engine kernels, built on first use
  mutable std::map<std::vector<int32_t>, int64_t> fused_cost;   // per template environment
  // per template environment (and start of the simulation): whether the
  // expression's reads go strictly forward, so paths can be streamed
  mutable std::map<std::vector<int32_t>, bool> streamable;
};

// Errors of calls made without a context (payoff loading may run before
// any device is opened) are kept per thread.
static thread_local std::string g_err;

static int fail(pmc_ctx* c, int st, const std::string& m) {
  if (c) c->err = m;
  else g_err = m;
  return st;
}

#define HIP_TRY(ctx, expr)                                                           \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(ctx, e_ == hipErrorOutOfMemory ? PMC_E_OOM : PMC_E_HIP,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                \
  } while (0)

namespace pmc {
hipStream_t ctx_stream(const pmc_ctx* c) { return c->stream; }
int ctx_device(const pmc_ctx* c) { return c->device; }
int ctx_fail(pmc_ctx* c, int status, const std::string& msg) { return fail(c, status, msg); }
}  // namespace pmc

extern "C" const char* pmc_version(void) { return "pmc 1.0 (gfx950)"; }

extern "C" int pmc_ctx_create(int device, void* stream, pmc_ctx** out) {
  if (!out) return fail(nullptr, PMC_E_ARG, "null out");
  auto hip_fail = [](const char* what, hipError_t e) {
    return fail(nullptr, PMC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail("hipGetDeviceCount", e);
  if (device < 0 || device >= n)
    return fail(nullptr, PMC_E_ARG, "device " + std::to_string(device) + " of " + std::to_string(n));
  auto c = std::make_unique<pmc_ctx>();
  c->device = device;
  c->stream = (hipStream_t)stream;
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail("hipSetDevice", e);
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail("hipGetDeviceProperties", e);
  c->n_cu = prop.multiProcessorCount;
  c->device_name = prop.gcnArchName;
  // Set-up of the allocation-free call: the scratch's address on this
  // device, looked up (once per device) while the device is current.
  if ((e = scratch_address(device, &c->scratch)) != hipSuccess) {
    c->scratch = nullptr;
    c->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
  }
  // Start and intermediate markers only take times: no system-scope cache
  // write-back and invalidation when they are reached (which would also
  // leave the following kernel a cold L2).  The end marker, which the host
  // waits on before reading results, keeps the default fence.
  if ((e = hipEventCreateWithFlags(&c->ev0, hipEventDisableSystemFence)) != hipSuccess ||
      (e = hipEventCreate(&c->ev1)) != hipSuccess)
    return hip_fail("hipEventCreate", e);
  for (auto& ev : c->evk)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence)) != hipSuccess)
      return hip_fail("hipEventCreate", e);
  *out = c.release();
  return PMC_OK;
}

extern "C" void pmc_ctx_destroy(pmc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (auto e : c->evk)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

extern "C" const char* pmc_last_error(const pmc_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

static std::vector<std::string> names(const char* const* a, int n) {
  std::vector<std::string> v;
  for (int i = 0; i < n; ++i) v.emplace_back(a[i] ? a[i] : "");
  return v;
}

extern "C" int pmc_payoff_load(pmc_ctx* c, const char* text, size_t len, const char* const* assets,
                               int n_assets, const char* const* params, int n_params,
                               const char* const* tvars, int n_tvars, pmc_payoff** out) {
  if (!out || (!text && len)) return fail(c, PMC_E_ARG, "null argument");
  if (n_assets < 1 || n_assets > PMC_MAX_ASSETS) return fail(c, PMC_E_UNSUPPORTED, "1..4 assets supported");
  if (n_params < 0 || n_tvars < 0 || (n_params && !params) || (n_tvars && !tvars) || !assets)
    return fail(c, PMC_E_ARG, "bad label arrays");
  auto p = std::make_unique<pmc_payoff>();
  std::string err;
  int st = compile(text, len, names(assets, n_assets), names(params, n_params), names(tvars, n_tvars), p->prog, err);
  if (st != PMC_OK) return fail(c, st, err);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < len; ++i) h = (h ^ (uint8_t)text[i]) * 1099511628211ull;
  p->hash = h;
  *out = p.release();
  return PMC_OK;
}

extern "C" void pmc_payoff_free(pmc_payoff* p) { delete p; }

extern "C" int pmc_payoff_cut(pmc_ctx* c, const pmc_payoff* in, pmc_payoff** out) {
  if (!in || !out) return fail(c, PMC_E_ARG, "null argument");
  auto p = std::make_unique<pmc_payoff>();
  std::string err;
  int st = cut_payoff(in->prog, p->prog, err);
  if (st != PMC_OK) return fail(c, st, err);
  p->hash = (in->hash ^ 0x9E3779B97F4A7C15ull) * 1099511628211ull;
  *out = p.release();
  return PMC_OK;
}

namespace pmc {
namespace {
#include "engine_src.inc"
}  // namespace
}  // namespace pmc

extern "C" int pmc_payoff_source(const pmc_payoff* p, const int32_t* tenv, char* buf, size_t cap, size_t* len) {
  if (!p || !len) return PMC_E_ARG;
  pmc::Grid g;
  const pmc::Grid* gp = nullptr;
  bool fixed = false;
  if (tenv) {
    std::string err;
    const int st = pmc::plan(p->prog, tenv, g, err);
    if (st != PMC_OK) return st;
    fixed = pmc::unrolled_size(p->prog, g, p->prog.root, pmc::kMaxUnrolled + 1) <= pmc::kMaxUnrolled;
    if (fixed) gp = &g;   // else the generic function serves this environment too
  }
  const std::string s = std::string(pmc::kEngineSource) + "\n" + generate_payoff(p->prog, gp, fixed);
  *len = s.size();
  if (buf && cap) {
    const size_t n = std::min(cap - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return PMC_OK;
}

extern "C" int pmc_payoff_get_info(const pmc_payoff* p, pmc_payoff_info* o) {
  if (!p || !o) return PMC_E_ARG;
  o->n_instr = (int)p->prog.code.size();
  o->n_regs = p->prog.n_regs;
  o->loop_depth = p->prog.loop_depth;
  o->n_time_exprs = (int)p->prog.tt.size();
  o->n_parties = (int)p->prog.parties.size();
  o->n_assets = (int)p->prog.assets.size();
  o->n_params = (int)p->prog.params.size();
  o->n_tvars = (int)p->prog.tvars.size();
  return PMC_OK;
}

extern "C" int pmc_payoff_grid(const pmc_payoff* p, const int32_t* tenv, int32_t* days, int max_days,
                               int* n_slots, int* horizon) {
  if (!p || (!tenv && !p->prog.tvars.empty()) || !n_slots) return PMC_E_ARG;
  Grid g;
  std::string err;
  int st = plan(p->prog, tenv, g, err);
  if (st != PMC_OK) return st;
  *n_slots = (int)g.days.size();
  if (horizon) *horizon = g.horizon;
  if (days) {
    if (max_days < (int)g.days.size()) return PMC_E_ARG;
    std::copy(g.days.begin(), g.days.end(), days);
  }
  return PMC_OK;
}

extern "C" int pmc_payoff_streams(const pmc_payoff* p, const int32_t* tenv, int32_t sim_from, int* streams) {
  if (!p || (!tenv && !p->prog.tvars.empty()) || !streams || sim_from < 0) return PMC_E_ARG;
  Grid g;
  std::string err;
  const int st = plan(p->prog, tenv, g, err, sim_from);
  if (st != PMC_OK) return st;
  *streams = stream_reads(p->prog, g, int64_t(1) << 22) ? 1 : 0;
  return PMC_OK;
}

extern "C" int pmc_cholesky(pmc_ctx* c, const double* a, int n, int m, double* l) {
  if (!c || !a || !l || n < 1 || m < 1 || m > 16) return fail(c, PMC_E_ARG, "bad cholesky arguments");
  HIP_TRY(c, hipSetDevice(c->device));
  size_t bytes = (size_t)n * m * m * sizeof(double);
  HIP_TRY(c, c->blob.ensure(bytes));
  c->last_upload.clear();   // the blob is reused for the input below
  HIP_TRY(c, c->chol.ensure(bytes));
  HIP_TRY(c, c->bad.ensure((size_t)n * sizeof(int)));
  HIP_TRY(c, hipMemcpyAsync(c->blob.p, a, bytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_prep((const double*)c->blob.p, (double*)c->chol.p, (int*)c->bad.p, nullptr, 0, n, m, c->stream));
  std::vector<int> status(n);
  HIP_TRY(c, hipMemcpyAsync(status.data(), c->bad.p, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(l, c->chol.p, bytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int bad = -1;
  for (int i = 0; i < n && bad < 0; ++i)
    if (status[i]) bad = i;
  if (bad >= 0) return fail(c, PMC_E_NOT_PD, "matrix " + std::to_string(bad) + " is not positive definite");
  return PMC_OK;
}

// ---------------------------------------------------------------------------
namespace {

bool finite(double x) { return std::isfinite(x); }

struct InstanceIn {
  const int32_t* tenv;
  const double* params;
  const double* spot;
  const double* vol;
  const double* corr;  // may be null (identity)
  uint32_t instance;
};

int check_model(pmc_ctx* c, const Program& P, const pmc_gbm* m) {
  if (!m) return fail(c, PMC_E_ARG, "null model");
  if (m->n_assets != (int)P.assets.size()) return fail(c, PMC_E_ARG, "model asset count differs from the payoff's");
  if (!finite(m->rate) || !finite(m->years_per_day) || m->years_per_day <= 0)
    return fail(c, PMC_E_ARG, "rate and years_per_day must be finite, years_per_day > 0");
  return PMC_OK;
}

int check_instance(pmc_ctx* c, const Program& P, const InstanceIn& in) {
  const int A = (int)P.assets.size();
  if (!in.spot || !in.vol) return fail(c, PMC_E_ARG, "null spot or vol");
  for (int a = 0; a < A; ++a) {
    if (!finite(in.spot[a]) || in.spot[a] <= 0) return fail(c, PMC_E_ARG, "spot must be finite and > 0");
    if (!finite(in.vol[a]) || in.vol[a] < 0) return fail(c, PMC_E_ARG, "vol must be finite and >= 0");
  }
  if (in.corr)
    for (int i = 0; i < A * A; ++i)
      if (!finite(in.corr[i])) return fail(c, PMC_E_ARG, "correlation must be finite");
  if (!P.params.empty() && !in.params) return fail(c, PMC_E_ARG, "null params");
  for (size_t q = 0; q < P.params.size(); ++q)
    if (!finite(in.params[q])) return fail(c, PMC_E_ARG, "parameter '" + P.params[q] + "' is not finite");
  if (!P.tvars.empty() && !in.tenv) return fail(c, PMC_E_ARG, "null tenv");
  return PMC_OK;
}

int check_opts(pmc_ctx* c, const pmc_opts* o) {
  if (!o) return fail(c, PMC_E_ARG, "null opts");
  if (o->n_paths < 1 || o->n_paths > (1ull << 32)) return fail(c, PMC_E_ARG, "n_paths must be in 1..2^32");
  if (o->rng != PMC_RNG_PHILOX && o->rng != PMC_RNG_SOBOL) return fail(c, PMC_E_ARG, "bad rng");
  if (o->precision != PMC_FP32 && o->precision != PMC_FP64) return fail(c, PMC_E_ARG, "bad precision");
  if (!o->party_from || !o->party_to) return fail(c, PMC_E_ARG, "null party name");
  if (o->block != 0 && (o->block % 64 != 0 || o->block > 256 || o->block < 64))
    return fail(c, PMC_E_ARG, "block must be 64, 128, 192 or 256");
  if (o->history && (o->history_len < 1 || o->history_len > (1 << 20) || o->t_now < 0))
    return fail(c, PMC_E_ARG, "a price history needs 1 <= history_len <= 2^20 and t_now >= 0");
  if (o->mode < 0 || o->mode > 2) return fail(c, PMC_E_ARG, "bad mode");
  if (o->engine < 0 || o->engine > 2) return fail(c, PMC_E_ARG, "bad engine");
  return PMC_OK;
}

// Host-side tables of one launch (all instances), before upload.
template <typename T>
struct Tables {
  std::vector<int32_t> itab;
  std::vector<T> rtab;
  std::vector<double> corr;  // Cholesky inputs, A x A per instance
  std::vector<InstDesc> desc;
  int max_dims = 0;          // largest slots * assets
  int64_t path_dates = 0;
  std::vector<int> n_slots;
  int32_t hist_off = -1;     // a given price history, shared by the instances
};

// Tables shared by every instance with the same template environment
// (folded template values, party signs, day map, discount per day, per-slot
// dt): built once per distinct tenv of a launch.
struct GridTables {
  int32_t tt_off, sign_off, daymap_off, horizon, n_slots, dense_first, disc_off, slot_off;
};

template <typename T>
int build_instance(pmc_ctx* c, const Program& P, const pmc_gbm& m, const pmc_opts& o,
                   const InstanceIn& in, int idx, Tables<T>& tb,
                   std::map<std::vector<int32_t>, GridTables>* memo = nullptr) {
  const int A = (int)P.assets.size();
  std::vector<int32_t> key(in.tenv, in.tenv + P.tvars.size());
  GridTables gt{};
  auto hit = memo ? memo->find(key) : decltype(memo->end()){};
  if (memo && hit != memo->end()) {
    gt = hit->second;
  } else {
    Grid g;
    std::string err;
    int st = plan(P, in.tenv, g, err, o.history ? o.t_now : 0);
    if (st != PMC_OK) return fail(c, st, err);
    gt.tt_off = (int32_t)tb.itab.size();
    tb.itab.insert(tb.itab.end(), g.tt.begin(), g.tt.end());
    gt.sign_off = (int32_t)tb.itab.size();
    for (auto& pr : P.pairs) {
      const std::string& f = P.parties[pr.first];
      const std::string& t = P.parties[pr.second];
      int sg = 0;
      if (f == o.party_from && t == o.party_to) sg = 1;
      else if (f == o.party_to && t == o.party_from) sg = -1;
      tb.itab.push_back(sg);
    }
    gt.daymap_off = (int32_t)tb.itab.size();
    tb.itab.insert(tb.itab.end(), g.daymap.begin(), g.daymap.end());
    gt.horizon = g.horizon;
    gt.n_slots = (int32_t)g.days.size();
    gt.dense_first = 0;
    if (!g.days.empty() && g.days.back() - g.days.front() + 1 == (int32_t)g.days.size()) gt.dense_first = g.days.front();
    // d(day) = exp(-r * day * years_per_day)
    gt.disc_off = (int32_t)tb.rtab.size();
    for (int32_t day = 0; day <= g.horizon; ++day) tb.rtab.push_back((T)std::exp(-m.rate * (double)day * m.years_per_day));
    // per slot: dt, sqrt(dt) with dt = (day_s - day_{s-1}) * years_per_day,
    // from the day the simulation starts
    gt.slot_off = (int32_t)tb.rtab.size();
    int32_t prev = g.sim_from;
    for (int32_t day : g.days) {
      const double dt = (double)(day - prev) * m.years_per_day;
      tb.rtab.push_back((T)dt);
      tb.rtab.push_back((T)std::sqrt(dt));
      prev = day;
    }
    if (memo) (*memo)[key] = gt;
  }
  InstDesc d{};
  d.tt_off = gt.tt_off;
  d.sign_off = gt.sign_off;
  d.daymap_off = gt.daymap_off;
  d.horizon = gt.horizon;
  d.n_slots = gt.n_slots;
  d.dense_first = gt.dense_first;
  d.disc_off = gt.disc_off;
  d.slot_off = gt.slot_off;
  d.t_now = o.t_now;
  d.param_off = (int32_t)tb.rtab.size();
  for (size_t q = 0; q < P.params.size(); ++q) tb.rtab.push_back((T)in.params[q]);
  d.model_off = (int32_t)tb.rtab.size();
  for (int a = 0; a < A; ++a) tb.rtab.push_back((T)(m.rate - 0.5 * in.vol[a] * in.vol[a]));
  for (int a = 0; a < A; ++a) tb.rtab.push_back((T)in.vol[a]);
  // the prices the simulation starts from: the spot, or the history's last
  const int32_t L = o.history_len;
  for (int a = 0; a < A; ++a) tb.rtab.push_back((T)(o.history ? o.history[(size_t)a * L + L - 1] : in.spot[a]));
  if (o.history) {
    if (tb.hist_off < 0) {
      for (size_t i = 0; i < (size_t)A * L; ++i)
        if (!finite(o.history[i]) || !(o.history[i] > 0)) return fail(c, PMC_E_ARG, "history prices must be finite and > 0");
      tb.hist_off = (int32_t)tb.rtab.size();
      for (size_t i = 0; i < (size_t)A * L; ++i) tb.rtab.push_back((T)o.history[i]);
    }
    d.sim_from = o.t_now;
    d.hist_off = tb.hist_off;
    d.hist_first = o.t_now - L + 1;
    d.n_hist = L;
  } else {   // days up to 0 read the spot
    d.sim_from = 0;
    d.hist_off = d.model_off + 2 * A;
    d.hist_first = 0;
    d.n_hist = 1;
  }
  d.chol_off = (int32_t)tb.corr.size();
  for (int i = 0; i < A; ++i)
    for (int j = 0; j < A; ++j) tb.corr.push_back(in.corr ? in.corr[i * A + j] : (i == j ? 1.0 : 0.0));
  d.instance = in.instance;
  d.n_paths = (uint32_t)std::min<uint64_t>(o.n_paths, 0xFFFFFFFFull);
  if (o.n_paths == (1ull << 32)) return fail(c, PMC_E_UNSUPPORTED, "n_paths = 2^32 is not supported per instance");
  if (tb.rtab.size() > 0x7fffffffu || tb.itab.size() > 0x7fffffffu)
    return fail(c, PMC_E_UNSUPPORTED, "batch tables exceed 2^31 entries");
  tb.max_dims = std::max(tb.max_dims, (int)gt.n_slots * A);
  tb.path_dates += (int64_t)o.n_paths * (int64_t)gt.n_slots;
  tb.n_slots.push_back((int)gt.n_slots);
  tb.desc.push_back(d);
  (void)idx;
  return PMC_OK;
}

int ensure_sobol(pmc_ctx* c, int dims) {
  if (dims <= c->sobol_dims) return PMC_OK;
  if (dims > 20000) return fail(c, PMC_E_UNSUPPORTED, "Sobol needs more than 20000 dimensions");
  const unsigned int* v = nullptr;
  if (rocrand_get_direction_vectors32(&v, ROCRAND_DIRECTION_VECTORS_32_JOEKUO6) != ROCRAND_STATUS_SUCCESS || !v)
    return fail(c, PMC_E_HIP, "Sobol direction numbers unavailable");
  const int want = std::max(dims, 64);
  HIP_TRY(c, c->sobol.ensure((size_t)want * 32 * sizeof(uint32_t)));
  HIP_TRY(c, hipMemcpyAsync(c->sobol.p, v, (size_t)want * 32 * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->sobol_dims = want;
  ++c->table_gen;
  return PMC_OK;
}

// Per-wave high-part table of the Sobol points 0 .. n-1 (kept while the
// shape is unchanged; limited to 64 MB).
int ensure_sobol_hi(pmc_ctx* c, uint64_t n, int dims, int bits, const uint32_t** out) {
  *out = nullptr;
  const uint64_t rows = (n + 63) / 64;
  const uint64_t bytes = rows * (uint64_t)dims * 4u;
  if (bytes > (64ull << 20)) return PMC_OK;
  if (c->sobol_hi_rows >= (int)rows && c->sobol_hi_dims == dims && c->sobol_hi_bits == bits) {
    *out = (const uint32_t*)c->sobol_hi.p;
    return PMC_OK;
  }
  HIP_TRY(c, c->sobol_hi.ensure((size_t)bytes));
  HIP_TRY(c, launch_sobol_hi((const uint32_t*)c->sobol.p, (uint32_t*)c->sobol_hi.p, (int)rows, dims, bits, c->stream));
  ++c->table_gen;
  c->sobol_hi_rows = (int)rows;
  c->sobol_hi_dims = dims;
  c->sobol_hi_bits = bits;
  *out = (const uint32_t*)c->sobol_hi.p;
  return PMC_OK;
}

int sobol_bits(uint64_t n) {
  int b = 1;
  while (b < 32 && ((n - 1) >> b) != 0) ++b;
  return b;
}

// Uploads the tables and fills the launch arguments (except work items).
template <typename T>
int upload(pmc_ctx* c, const Program& P, const Tables<T>& tb, const pmc_opts& o, McLaunch& L,
           const std::vector<int>* order) {
  Pack pk;
  std::vector<T> consts(P.consts.size());
  for (size_t i = 0; i < consts.size(); ++i) consts[i] = (T)P.consts[i];
  const size_t o_code = pk.add(P.code.data(), P.code.size() * sizeof(Instr));
  const size_t o_consts = pk.add(consts.data(), consts.size() * sizeof(T));
  const size_t o_desc = pk.add(tb.desc.data(), tb.desc.size() * sizeof(InstDesc));
  const size_t o_itab = pk.add(tb.itab.data(), tb.itab.size() * sizeof(int32_t));
  const size_t o_rtab = pk.add(tb.rtab.data(), tb.rtab.size() * sizeof(T));
  const size_t o_corr = pk.add(tb.corr.data(), tb.corr.size() * sizeof(double));
  size_t o_order = 0;
  if (order) o_order = pk.add(order->data(), order->size() * sizeof(int));
  void* old_blob = c->blob.p;
  HIP_TRY(c, c->blob.ensure(pk.bytes.size()));
  if (c->blob.p != old_blob || c->last_upload != pk.bytes) {
    HIP_TRY(c, c->staging.ensure(pk.bytes.size()));
    // the previous call may still read the staging buffer's last copy
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::memcpy(c->staging.p, pk.bytes.data(), pk.bytes.size());
    HIP_TRY(c, hipMemcpyAsync(c->blob.p, c->staging.p, pk.bytes.size(), hipMemcpyHostToDevice, c->stream));
    c->last_upload.swap(pk.bytes);
    ++c->table_gen;
  }
  HIP_TRY(c, c->chol.ensure(std::max<size_t>(tb.corr.size(), 1) * sizeof(double)));
  uint8_t* b = (uint8_t*)c->blob.p;
  L = McLaunch{};
  L.code = (const Instr*)(b + o_code);
  L.consts = b + o_consts;
  L.desc = (const InstDesc*)(b + o_desc);
  L.itab = (const int32_t*)(b + o_itab);
  L.rtab = b + o_rtab;
  L.chol = (const double*)c->chol.p;
  L.order = order ? (const int*)(b + o_order) : nullptr;
  L.k0 = (uint32_t)(o.seed & 0xFFFFFFFFull);
  L.k1 = (uint32_t)(o.seed >> 32);
  L.n_assets = (int)P.assets.size();
  L.n_regs = P.n_regs;
  L.ppt = 1;
  if (o.rng == PMC_RNG_SOBOL) {
    // at least one dimension, so that the direction-number table exists even
    // for an expression that simulates no day (the kernels read it regardless)
    int st = ensure_sobol(c, std::max(1, tb.max_dims));
    if (st != PMC_OK) return st;
    L.sobol = (const uint32_t*)c->sobol.p;
    L.sobol_bits = sobol_bits(o.n_paths);
    const int dims = std::max(1, tb.max_dims);
    st = ensure_sobol_hi(c, o.n_paths, dims, L.sobol_bits, &L.sobol_hi);
    if (st != PMC_OK) return st;
    L.sobol_dims = dims;
  }
  L.chol_in = (const double*)(b + o_corr);
  return PMC_OK;
}

// Result and counter buffers for n_inst instances; fills the launch's
// result, done and (persistent launches) queue pointers.
int bind_results(pmc_ctx* c, McLaunch& L, int n_inst, bool persistent) {
  HIP_TRY(c, c->results.ensure((size_t)n_inst * (sizeof(double2) + sizeof(int))));
  HIP_TRY(c, c->counters.ensure((size_t)(n_inst + 1) * sizeof(uint32_t)));
  L.result = (double2*)c->results.dev;
  L.done = (uint32_t*)c->counters.p;
  L.queue = persistent ? L.done + n_inst : nullptr;
  return PMC_OK;
}

int* status_dev(pmc_ctx* c, int n_inst) { return (int*)((double2*)c->results.dev + n_inst); }
const int* status_host(pmc_ctx* c, int n_inst) { return (const int*)((const double2*)c->results.p + n_inst); }

// Zeroes the counters and factors the instances' correlation matrices.
int prep(pmc_ctx* c, const McLaunch& L, int n_inst, int A) {
  HIP_TRY(c, launch_prep(L.chol_in, (double*)c->chol.p, status_dev(c, n_inst), L.done, n_inst + 1, n_inst, A,
                         c->stream));
  return PMC_OK;
}

int first_bad(pmc_ctx* c, int n_inst) {
  const int* st = status_host(c, n_inst);
  for (int i = 0; i < n_inst; ++i)
    if (st[i]) return i;
  return -1;
}

// One instrument's result from its FP64 path sums.
pmc_result make_result(double2 sums, uint64_t n_paths, int n_slots, int mode_used, double ms, double gen_ms,
                       double eval_ms) {
  const double N = (double)n_paths;
  pmc_result r{};
  r.sum = sums.x;
  r.sum_sq = sums.y;
  r.n_paths = n_paths;
  r.price = r.sum / N;
  const double var = N > 1 ? std::max(0.0, (r.sum_sq - r.sum * r.sum / N) / (N - 1.0)) : 0.0;
  r.std_err = std::sqrt(var / N);
  r.n_slots = n_slots;
  r.path_dates = n_paths * (uint64_t)n_slots;
  r.mode_used = mode_used;
  r.ms = ms;
  r.gen_ms = gen_ms;
  r.eval_ms = eval_ms;
  return r;
}

// Reads the results the kernels wrote to host memory; the caller has
// synchronized with the launch.
int finish(pmc_ctx* c, int n_inst, const uint64_t* n_paths, const int* n_slots, int mode_used, double ms,
           pmc_result* out, double gen_ms = 0.0, double eval_ms = 0.0) {
  const int bad = first_bad(c, n_inst);
  if (bad >= 0) return fail(c, PMC_E_NOT_PD, "correlation matrix of instance " + std::to_string(bad) + " is not positive definite");
  const double2* res = (const double2*)c->results.p;
  for (int i = 0; i < n_inst; ++i)
    out[i] = make_result(res[i], n_paths[i], n_slots[i], mode_used, ms, gen_ms, eval_ms);
  return PMC_OK;
}

// Simulated asset-dates per path up to which a single-instrument launch
// counts as short.
constexpr int64_t kShortItem = 64;

// A fixed-stride grid for `items` work items on at most `cap` resident
// blocks: the fewest blocks that still take ceil(items / cap) items each, so
// that every block strides over the same number of items (a grid of cap
// blocks would leave some with one item fewer, and the kernel waits for the
// blocks with the most).
int balanced_grid(int items, int cap) {
  cap = std::max(1, cap);
  if (items <= cap) return std::max(1, items);
  const int per = (items + cap - 1) / cap;
  return (items + per - 1) / per;
}

// Chooses the Monte Carlo kernel for the requested payoff engine and its
// grid.  lanes: paths per lane (compiled engine with stored paths only);
// full, tenv: whole-path capacity and the template environment a compiled
// kernel is generated for.  Without a work queue the kernel strides over
// the items.  Short items (few simulated asset-dates per path) run on a grid
// capped at the blocks that fit on the chip at once, so per-block set-up
// (tables, factor, partial) is paid once per resident block; long items keep
// one block per item, whose dispatch balances the load better than a fixed
// stride.
int resolve_engine(pmc_ctx* c, const pmc_payoff* p, const pmc_opts* o, int prec, bool mem, const McLaunch& L,
                   int grid, int block, int lanes, int64_t asset_dates, int full, const int32_t* tenv,
                   EngineLaunch& e, bool stream = false) {
  const int A = (int)p->prog.assets.size();
  const bool cap = !L.queue && asset_dates <= kShortItem;
  e = EngineLaunch{};
  e.prec = prec;
  e.rng = o->rng;
  e.mem = mem;
  e.block = block;
  if (o->engine == PMC_ENGINE_INTERPRETER) {
    if (cap) {
      const std::string key = "interp/" + std::to_string(prec) + "/" + std::to_string(o->rng) + "/" +
                              std::to_string(A) + "/" + std::to_string(p->prog.n_regs <= 7 ? 8 : 32) + "/" +
                              std::to_string(block);
      auto it = c->occupancy.find(key);
      if (it == c->occupancy.end()) it = c->occupancy.emplace(key, mc_occupancy(prec, o->rng, A, p->prog.n_regs, block)).first;
      grid = balanced_grid(grid, c->n_cu * it->second);
    }
    e.grid = grid;
    return PMC_OK;
  }
  hipFunction_t f = nullptr;
  std::string err;
  const bool single = !L.queue && !L.order;
  const bool own = !mem && L.factor != 0;
  int st = p->jit.get(p->prog, c->device, prec, o->rng, A, mem, &f, err, lanes, full, tenv, single, own, stream);
  if (st != PMC_OK) return fail(c, st, err);
  if (cap) {
    char kb[64];
    std::snprintf(kb, sizeof kb, "jit/%p/%d", (const void*)f, block);
    const std::string key = kb;
    auto it = c->occupancy.find(key);
    if (it == c->occupancy.end()) it = c->occupancy.emplace(key, mc_occupancy_jit(f, block)).first;
    grid = balanced_grid(grid, c->n_cu * it->second);
  }
  e.jit = true;
  e.f = f;
  e.grid = grid;
  return PMC_OK;
}

// Enqueues a resolved launch; one instrument (no work queue): the
// per-block partials are summed by a second kernel, and `mid` (optional)
// marks the end of the pricing kernel itself.
int run_engine(pmc_ctx* c, const EngineLaunch& e, const McLaunch& L, hipEvent_t mid = nullptr) {
  if (e.jit) HIP_TRY(c, launch_mc_jit(e.f, e.prec, L, e.grid, e.block, c->stream));
  else HIP_TRY(c, launch_mc(e.prec, e.rng, e.mem, L, e.grid, e.block, c->stream));
  if (!L.queue) {
    if (mid) HIP_TRY(c, hipEventRecord(mid, c->stream));
    HIP_TRY(c, launch_finish(L.partial, e.grid, L.result, c->stream));
  }
  return PMC_OK;
}

int launch_engine(pmc_ctx* c, const pmc_payoff* p, const pmc_opts* o, int prec, bool mem, const McLaunch& L,
                  int grid, int block, int lanes = 1, int64_t asset_dates = 0, int full = 0,
                  const int32_t* tenv = nullptr, bool stream = false) {
  EngineLaunch e;
  const int st = resolve_engine(c, p, o, prec, mem, L, grid, block, lanes, asset_dates, full, tenv, e, stream);
  return st != PMC_OK ? st : run_engine(c, e, L);
}

// Whole-path capacity of the compiled engine's generated paths for at most
// `values` (= slots x assets) prices per path: the smallest power of two that
// holds them, or 0 (the sliding window) above 32 values in FP32 or 16 in
// FP64 (32 registers either way).
int full_capacity(const pmc_opts* o, int64_t values, int prec) {
  if (o->engine == PMC_ENGINE_INTERPRETER || values > (prec ? 16 : 32)) return 0;
  int cap = 1;
  while (cap < values) cap <<= 1;
  return cap;
}

// Whether the payoff's reads for this template environment (simulation
// from day sim_from) never go back to an earlier slot, memoized per payoff:
// its generated paths can then be streamed (compiled engine, Philox).
bool streamable(const pmc_payoff* p, const int32_t* tenv, int32_t sim_from) {
  const size_t nv = p->prog.tvars.size();
  std::vector<int32_t> key(tenv, tenv + (tenv ? nv : 0));
  key.push_back(sim_from);
  auto it = p->streamable.find(key);
  if (it != p->streamable.end()) return it->second;
  Grid g;
  std::string err;
  const bool ok = (nv == 0 || tenv) && plan(p->prog, tenv, g, err, sim_from) == PMC_OK &&
                  stream_reads(p->prog, g, int64_t(1) << 22);
  p->streamable.emplace(key, ok);
  return ok;
}

// A launch that can stream its paths: compiled engine, Philox words, no
// whole-path window.
bool stream_launch(const pmc_opts* o, int full) {
  return o->engine != PMC_ENGINE_INTERPRETER && o->rng == PMC_RNG_PHILOX && full == 0;
}

int engine_used(const pmc_opts* o) {
  return o->engine == PMC_ENGINE_INTERPRETER ? PMC_ENGINE_INTERPRETER : PMC_ENGINE_COMPILED;
}

// ---------------------------------------------- prepared single calls ---
template <typename X>
void put(std::vector<uint8_t>& k, const X& x) {
  const uint8_t* b = reinterpret_cast<const uint8_t*>(&x);
  k.insert(k.end(), b, b + sizeof(X));
}
void put_bytes(std::vector<uint8_t>& k, const void* p, size_t n) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  k.insert(k.end(), b, b + n);
}

// Serializes everything a fused single pricing depends on; false if an
// input pointer is missing (the call then takes the checked path).
bool call_key(std::vector<uint8_t>& k, const pmc_payoff* p, int real_size, const int32_t* tenv,
              const double* params, const pmc_gbm* m, const pmc_opts* o) {
  const Program& P = p->prog;
  const size_t A = P.assets.size();
  if ((!tenv && !P.tvars.empty()) || (!params && !P.params.empty()) || !m->spot || !m->vol || !o->party_from ||
      !o->party_to)
    return false;
  k.clear();
  put(k, p->serial);
  put(k, real_size);
  if (!P.tvars.empty()) put_bytes(k, tenv, P.tvars.size() * sizeof(int32_t));
  if (!P.params.empty()) put_bytes(k, params, P.params.size() * sizeof(double));
  put(k, m->rate);
  put(k, m->years_per_day);
  put_bytes(k, m->spot, A * sizeof(double));
  put_bytes(k, m->vol, A * sizeof(double));
  put(k, (uint8_t)(m->corr != nullptr));
  if (m->corr) put_bytes(k, m->corr, A * A * sizeof(double));
  put(k, o->n_paths); put(k, o->rng); put(k, o->seed); put(k, o->instance); put(k, o->precision);
  put(k, o->t_now); put(k, o->mode); put(k, o->payoffs_dev); put(k, o->block); put(k, o->engine);
  put_bytes(k, o->party_from, std::strlen(o->party_from) + 1);
  put_bytes(k, o->party_to, std::strlen(o->party_to) + 1);
  put(k, (uint8_t)(o->history != nullptr));
  if (o->history) {
    put(k, o->history_len);
    put_bytes(k, o->history, A * (size_t)o->history_len * sizeof(double));
  }
  return true;
}

// Serializes everything a batched pricing depends on, with its tile; false
// if an input pointer is missing (the call then takes the checked path).
bool batch_call_key(std::vector<uint8_t>& k, const pmc_payoff* p, const pmc_batch* b, const pmc_gbm* m,
                    const pmc_opts* o, int block, int ppt, int lanes) {
  const Program& P = p->prog;
  const size_t A = P.assets.size(), I = (size_t)b->n_inst, nv = P.tvars.size(), nq = P.params.size();
  const bool per = b->per_instance_model != 0;
  const double* sp = per ? b->spot : m->spot;
  const double* vo = per ? b->vol : m->vol;
  const double* co = per ? b->corr : m->corr;
  if ((nv && !b->tenv) || (nq && !b->params) || !sp || !vo || !o->party_from || !o->party_to) return false;
  const size_t rows = per ? I : 1;
  k.clear();
  put(k, p->serial);
  put(k, block); put(k, ppt); put(k, lanes); put(k, b->n_inst);
  if (nv) put_bytes(k, b->tenv, I * nv * sizeof(int32_t));
  if (nq) put_bytes(k, b->params, I * nq * sizeof(double));
  put(k, (uint8_t)per);
  put_bytes(k, sp, rows * A * sizeof(double));
  put_bytes(k, vo, rows * A * sizeof(double));
  put(k, (uint8_t)(co != nullptr));
  if (co) put_bytes(k, co, rows * A * A * sizeof(double));
  put(k, (uint8_t)(b->instance_ids != nullptr));
  if (b->instance_ids) put_bytes(k, b->instance_ids, I * sizeof(uint32_t));
  put(k, m->rate); put(k, m->years_per_day);
  put(k, o->n_paths); put(k, o->rng); put(k, o->seed); put(k, o->instance); put(k, o->precision);
  put(k, o->t_now); put(k, o->mode); put(k, o->block); put(k, o->engine);
  put_bytes(k, o->party_from, std::strlen(o->party_from) + 1);
  put_bytes(k, o->party_to, std::strlen(o->party_to) + 1);
  put(k, (uint8_t)(o->history != nullptr));
  if (o->history) {
    put(k, o->history_len);
    put_bytes(k, o->history, A * (size_t)o->history_len * sizeof(double));
  }
  return true;
}

// The device buffers a prepared launch points into (reallocation of any of
// them invalidates it).
void buffer_snapshot(const pmc_ctx* c, const void* (&b)[8]) {
  b[0] = c->blob.p; b[1] = c->partial.p; b[2] = c->results.dev; b[3] = c->counters.p;
  b[4] = c->chol.p; b[5] = c->sobol.p; b[6] = c->sobol_hi.p; b[7] = c->staging.p;
}

bool prepared_hit(const pmc_ctx* c) {
  const auto& pr = c->prepared;
  if (!pr.valid || pr.gen != c->table_gen || pr.key != c->key_buf) return false;
  const void* b[8];
  buffer_snapshot(c, b);
  return std::memcmp(b, pr.bufs, sizeof b) == 0;
}

// Waits for the end marker and reports one instrument's result.
int complete_single(pmc_ctx* c, uint64_t N, int n_slots, int mode, bool two_phase, int engine, pmc_result* out) {
  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  HIP_TRY(c, hipEventSynchronize(c->ev1));
  float ms = 0, gen_ms = 0, eval_ms = 0;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (two_phase) {
    HIP_TRY(c, hipEventElapsedTime(&gen_ms, c->evk[0], c->evk[1]));
    HIP_TRY(c, hipEventElapsedTime(&eval_ms, c->evk[1], c->ev1));
  } else {
    HIP_TRY(c, hipEventElapsedTime(&eval_ms, c->ev0, c->evk[2]));   // the pricing kernel, before k_finish
  }
  const int st = finish(c, 1, &N, &n_slots, mode, ms, out, gen_ms, eval_ms);
  if (st == PMC_OK) out->engine_used = engine;
  return st;
}

template <typename T>
int price_one(pmc_ctx* c, const pmc_payoff* p, const int32_t* tenv, const double* params, const pmc_gbm* m,
              const pmc_opts* o, pmc_result* out, const void* given_paths, bool eval_only) {
  const Program& P = p->prog;
  // A fused call identical to the previous one, with the tables untouched
  // since: launch straight away.
  const bool keyed = !eval_only && !given_paths && call_key(c->key_buf, p, (int)sizeof(T), tenv, params, m, o);
  if (keyed && prepared_hit(c)) {
    const auto& pr = c->prepared;
    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    int st = run_engine(c, pr.e, pr.L, c->evk[2]);
    if (st != PMC_OK) return st;
    return complete_single(c, pr.n_paths, pr.n_slots, PMC_MODE_FUSED, false, pr.engine, out);
  }
  c->prepared.valid = false;
  InstanceIn in{tenv, params, m->spot, m->vol, m->corr, o->instance};
  int st = check_instance(c, P, in);
  if (st != PMC_OK) return st;
  Tables<T> tb;
  st = build_instance<T>(c, P, *m, *o, in, 0, tb);
  if (st != PMC_OK) return st;
  const int A = (int)P.assets.size();
  const int block = o->block ? o->block : 256;
  const uint64_t N = o->n_paths;
  const int n_slots = tb.desc[0].n_slots;
  const int prec = sizeof(T) == 8 ? 1 : 0;
  const int full = full_capacity(o, (int64_t)n_slots * A, prec);
  int mode = o->mode;
  const int32_t sim_from = o->history ? o->t_now : 0;
  const bool stream = !eval_only && stream_launch(o, full) && streamable(p, tenv, sim_from);
  if (eval_only) {
    mode = PMC_MODE_TWO_PHASE;
  } else if (mode == PMC_MODE_AUTO && (full > 0 || stream)) {
    mode = PMC_MODE_FUSED;   // the whole path is generated once
  } else if (mode == PMC_MODE_AUTO) {
    // fused unless the window would regenerate much more than one path
    std::vector<int32_t> key(tenv, tenv + P.tvars.size());
    key.push_back(o->history ? o->t_now : 0);   // the grid starts after the history
    auto it = p->fused_cost.find(key);
    if (it == p->fused_cost.end()) {
      Grid g;
      std::string err;
      plan(P, tenv, g, err, o->history ? o->t_now : 0);
      it = p->fused_cost.emplace(key, fused_generation_cost(P, g, A, 1 << 22)).first;
    }
    const int64_t cost = it->second;
    mode = (cost >= 0 && cost <= 2 * (int64_t)std::max(1, n_slots)) ? PMC_MODE_FUSED : PMC_MODE_TWO_PHASE;
  }
  // The compiled evaluator of stored paths gives each lane P consecutive
  // paths (one or more 16-byte loads per slot) when the path count and the
  // buffer's alignment allow it: 16 bytes' worth always, and up to 64 bytes
  // while the launch keeps at least one wave per SIMD (2^16 lanes), since the
  // wave-uniform work per slot is shared by more paths.
  // A fused launch that streams its paths gives each lane two paths once
  // the launch keeps at least one wave per SIMD (2^16 lanes): the paths
  // share each read's wave-uniform work (slot lookup, loop control), which
  // halves the scalar instructions per path-date; every path's payoff is
  // the same bit for bit.
  int lanes = 1;
  if (mode == PMC_MODE_TWO_PHASE && o->engine != PMC_ENGINE_INTERPRETER && n_slots > 0) {
    const int base_p = 16 / (int)sizeof(T);
    for (int want = 4 * base_p; want >= base_p; want /= 2) {
      const bool aligned = !given_paths || ((uintptr_t)given_paths % (want * sizeof(T))) == 0;
      const bool waves = want == base_p || N / (uint64_t)want >= (1u << 16);
      if (N % (uint64_t)want == 0 && aligned && waves) {
        lanes = want;
        break;
      }
    }
  } else if (mode == PMC_MODE_FUSED && stream && N >= (1u << 17)) {
    lanes = 2;
  }
  const uint64_t tile_paths = (uint64_t)block * (uint64_t)lanes;
  const uint32_t tiles = (uint32_t)((N + tile_paths - 1) / tile_paths);
  tb.desc[0].n_tiles = tiles;
  tb.desc[0].first_item = 0;
  McLaunch L;
  st = upload<T>(c, P, tb, *o, L, nullptr);
  if (st != PMC_OK) return st;
  HIP_TRY(c, c->partial.ensure((size_t)tiles * sizeof(double2)));
  st = bind_results(c, L, 1, false);
  if (st != PMC_OK) return st;
  L.partial = (double2*)c->partial.p;
  L.n_work = (int)tiles;
  L.payoff_out = o->payoffs_dev;
  // Timing markers: ev0 (start), evk[0] (generation start) and evk[1] (MC
  // kernel start) in the two-phase sequence, evk[2] (pricing kernel end,
  // before its finishing reduction) in the fused one, ev1 (end); each is a
  // queue entry, so only the ones a reported time needs are recorded.  (Events
  // attached to the launches themselves cost more: each such launch waits
  // on its own.)
  const bool two_phase = mode == PMC_MODE_TWO_PHASE;
  // the pricing kernel is generated for this template environment (a
  // program without template variables has one, the empty one)
  // (with a price history, the generic kernel: a generated one fixes the
  // grid, which then also depends on the current day)
  static const int32_t kNoTenv[1] = {0};
  const int32_t* env = o->history ? nullptr : tenv ? tenv : kNoTenv;
  HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  if (two_phase) {
    st = prep(c, L, 1, A);
    if (st != PMC_OK) return st;
    HIP_TRY(c, hipEventRecord(c->evk[0], c->stream));
    if (given_paths) {
      L.paths = given_paths;
    } else {
      const size_t bytes = (size_t)n_slots * A * N * sizeof(T);
      HIP_TRY(c, c->paths.ensure(std::max<size_t>(bytes, 4)));
      HIP_TRY(c, launch_pathgen(prec, o->rng, L, c->paths.p, nullptr, nullptr, (uint32_t)N, 256, c->stream));
      L.paths = c->paths.p;
    }
    if (n_slots == 0) L.paths = nullptr;
    HIP_TRY(c, hipEventRecord(c->evk[1], c->stream));
    st = launch_engine(c, p, o, prec, n_slots > 0, L, (int)tiles, block, lanes, (int64_t)n_slots * A, 0, env);
  } else {
    // Fused: the pricing kernel factors the correlation matrix itself (one
    // thread per block, into LDS) and reports its status; no preparation
    // kernel runs.
    L.factor = 1;
    L.status = status_dev(c, 1);
    EngineLaunch e;
    st = resolve_engine(c, p, o, prec, false, L, (int)tiles, block, lanes, (int64_t)n_slots * A, full, env, e,
                        stream);
    if (st != PMC_OK) return st;
    if (keyed) {   // the next identical call can reuse all of this
      auto& pr = c->prepared;
      pr.key = c->key_buf;
      pr.gen = c->table_gen;
      buffer_snapshot(c, pr.bufs);
      pr.L = L;
      pr.e = e;
      pr.n_paths = N;
      pr.n_slots = n_slots;
      pr.engine = engine_used(o);
      pr.valid = true;
    }
    st = run_engine(c, e, L, c->evk[2]);
  }
  if (st != PMC_OK) return st;
  return complete_single(c, N, n_slots, mode, two_phase, engine_used(o), out);
}

}  // namespace

extern "C" int pmc_price(pmc_ctx* c, const pmc_payoff* p, const int32_t* tenv, const double* params,
                         const pmc_gbm* m, const pmc_opts* o, pmc_result* out) {
  if (!c || !p || !out) return fail(c, PMC_E_ARG, "null argument");
  int st = check_model(c, p->prog, m);
  if (st == PMC_OK) st = check_opts(c, o);
  if (st != PMC_OK) return st;
  HIP_TRY(c, hipSetDevice(c->device));
  return o->precision == PMC_FP64 ? price_one<double>(c, p, tenv, params, m, o, out, nullptr, false)
                                  : price_one<float>(c, p, tenv, params, m, o, out, nullptr, false);
}

extern "C" int pmc_eval_paths(pmc_ctx* c, const pmc_payoff* p, const int32_t* tenv, const double* params,
                              const pmc_gbm* m, const pmc_opts* o, const void* paths_dev, pmc_result* out) {
  if (!c || !p || !out || !paths_dev) return fail(c, PMC_E_ARG, "null argument");
  int st = check_model(c, p->prog, m);
  if (st == PMC_OK) st = check_opts(c, o);
  if (st != PMC_OK) return st;
  HIP_TRY(c, hipSetDevice(c->device));
  return o->precision == PMC_FP64 ? price_one<double>(c, p, tenv, params, m, o, out, paths_dev, true)
                                  : price_one<float>(c, p, tenv, params, m, o, out, paths_dev, true);
}

// ------------------------------------------------ allocation-free call ---
namespace {

// One fused pricing by the precompiled interpreter kernel, with every
// device buffer in the per-device scratch: the tables are copied into its
// table area, the kernel writes its per-block partials and factorisation
// status there, the finishing kernel the (sum, sum of squares), which is
// copied back to the host.  Nothing in the scratch has to start at zero.
template <typename T>
int price_noalloc_one(pmc_ctx* c, const pmc_payoff* p, const int32_t* tenv, const double* params,
                      const pmc_gbm* m, const pmc_opts* o, pmc_result* out) {
  const Program& P = p->prog;
  InstanceIn in{tenv, params, m->spot, m->vol, m->corr, o->instance};
  int st = check_instance(c, P, in);
  if (st != PMC_OK) return st;
  Tables<T> tb;
  st = build_instance<T>(c, P, *m, *o, in, 0, tb);
  if (st != PMC_OK) return st;
  const int A = (int)P.assets.size();
  const int block = o->block ? o->block : 256;
  const uint64_t N = o->n_paths;
  const int n_slots = tb.desc[0].n_slots;
  const uint32_t tiles = (uint32_t)((N + (uint64_t)block - 1) / (uint64_t)block);
  tb.desc[0].n_tiles = tiles;
  tb.desc[0].first_item = 0;
  Pack pk;
  std::vector<T> consts(P.consts.size());
  for (size_t i = 0; i < consts.size(); ++i) consts[i] = (T)P.consts[i];
  const size_t o_code = pk.add(P.code.data(), P.code.size() * sizeof(Instr));
  const size_t o_consts = pk.add(consts.data(), consts.size() * sizeof(T));
  const size_t o_desc = pk.add(tb.desc.data(), tb.desc.size() * sizeof(InstDesc));
  const size_t o_itab = pk.add(tb.itab.data(), tb.itab.size() * sizeof(int32_t));
  const size_t o_rtab = pk.add(tb.rtab.data(), tb.rtab.size() * sizeof(T));
  const size_t o_corr = pk.add(tb.corr.data(), tb.corr.size() * sizeof(double));
  const int dims = std::max(1, tb.max_dims);
  size_t o_sobol = 0;
  if (o->rng == PMC_RNG_SOBOL) {
    if (dims > 20000) return fail(c, PMC_E_UNSUPPORTED, "Sobol needs more than 20000 dimensions");
    const unsigned int* v = nullptr;
    if (rocrand_get_direction_vectors32(&v, ROCRAND_DIRECTION_VECTORS_32_JOEKUO6) != ROCRAND_STATUS_SUCCESS || !v)
      return fail(c, PMC_E_HIP, "Sobol direction numbers unavailable");
    o_sobol = pk.add(v, (size_t)std::max(dims, 64) * 32 * sizeof(uint32_t));
  }
  if (pk.bytes.size() > kScratchTables)
    return fail(c, PMC_E_UNSUPPORTED, "the allocation-free call's tables need " + std::to_string(pk.bytes.size()) +
                                          " bytes; its scratch holds " + std::to_string(kScratchTables));
  uint8_t* const sc = (uint8_t*)c->scratch;
  uint8_t* const tab = sc + kScratchHead + (size_t)kScratchPartials * sizeof(double2);
  McLaunch L{};
  L.code = (const Instr*)(tab + o_code);
  L.consts = tab + o_consts;
  L.desc = (const InstDesc*)(tab + o_desc);
  L.itab = (const int32_t*)(tab + o_itab);
  L.rtab = tab + o_rtab;
  L.chol_in = (const double*)(tab + o_corr);
  L.chol = L.chol_in;   // not read: every block factors the matrix itself
  L.factor = 1;
  L.status = (int*)(sc + sizeof(double2));
  L.result = (double2*)sc;
  L.partial = (double2*)(sc + kScratchHead);
  L.k0 = (uint32_t)(o->seed & 0xFFFFFFFFull);
  L.k1 = (uint32_t)(o->seed >> 32);
  L.n_assets = A;
  L.n_regs = P.n_regs;
  L.ppt = 1;
  L.n_work = (int)tiles;
  L.payoff_out = o->payoffs_dev;
  if (o->rng == PMC_RNG_SOBOL) {
    L.sobol = (const uint32_t*)(tab + o_sobol);
    L.sobol_bits = sobol_bits(N);
    L.sobol_dims = dims;   // no high-part table: words come from the direction numbers
  }
  // the interpreter's grid of pmc_price, within the scratch's partials
  pmc_opts oi = *o;
  oi.engine = PMC_ENGINE_INTERPRETER;
  EngineLaunch e;
  st = resolve_engine(c, p, &oi, sizeof(T) == 8 ? 1 : 0, false, L, (int)tiles, block, 1, (int64_t)n_slots * A, 0,
                      nullptr, e);
  if (st != PMC_OK) return st;
  if (e.grid > kScratchPartials) e.grid = balanced_grid(e.grid, kScratchPartials);
  HIP_TRY(c, hipMemcpyAsync(tab, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  st = run_engine(c, e, L, c->evk[2]);
  if (st != PMC_OK) return st;
  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  struct { double2 sums; int status; } head{};
  HIP_TRY(c, hipMemcpyAsync(&head, sc, sizeof(double2) + sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (head.status) return fail(c, PMC_E_NOT_PD, "correlation matrix is not positive definite");
  float ms = 0, eval_ms = 0;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  HIP_TRY(c, hipEventElapsedTime(&eval_ms, c->ev0, c->evk[2]));
  *out = make_result(head.sums, N, n_slots, PMC_MODE_FUSED, ms, 0.0, eval_ms);
  out->engine_used = PMC_ENGINE_INTERPRETER;
  return PMC_OK;
}

}  // namespace

extern "C" int pmc_price_noalloc(pmc_ctx* c, const pmc_payoff* p, const int32_t* tenv, const double* params,
                                 const pmc_gbm* m, const pmc_opts* o, pmc_result* out) {
  if (!c || !p || !out) return fail(c, PMC_E_ARG, "null argument");
  int st = check_model(c, p->prog, m);
  if (st == PMC_OK) st = check_opts(c, o);
  if (st != PMC_OK) return st;
  if (o->mode == PMC_MODE_TWO_PHASE)
    return fail(c, PMC_E_UNSUPPORTED, "the allocation-free call generates paths in registers (fused) only");
  if (o->engine == PMC_ENGINE_COMPILED)
    return fail(c, PMC_E_UNSUPPORTED, "the allocation-free call runs the precompiled interpreter only");
  if (!c->scratch) return fail(c, PMC_E_HIP, c->scratch_err);
  HIP_TRY(c, hipSetDevice(c->device));
  return o->precision == PMC_FP64 ? price_noalloc_one<double>(c, p, tenv, params, m, o, out)
                                  : price_noalloc_one<float>(c, p, tenv, params, m, o, out);
}

namespace {
template <typename T>
int gen_paths(pmc_ctx* c, const pmc_payoff* p, const int32_t* tenv, const pmc_gbm* m, const pmc_opts* o,
              void* paths, uint32_t* words, void* normals) {
  const Program& P = p->prog;
  static const double zero_params[64] = {0};
  std::vector<double> params(P.params.size(), 0.0);
  InstanceIn in{tenv, params.empty() ? zero_params : params.data(), m->spot, m->vol, m->corr, o->instance};
  int st = check_instance(c, P, in);
  if (st != PMC_OK) return st;
  Tables<T> tb;
  st = build_instance<T>(c, P, *m, *o, in, 0, tb);
  if (st != PMC_OK) return st;
  McLaunch L;
  st = upload<T>(c, P, tb, *o, L, nullptr);
  if (st != PMC_OK) return st;
  st = bind_results(c, L, 1, false);
  if (st == PMC_OK) st = prep(c, L, 1, (int)P.assets.size());
  if (st != PMC_OK) return st;
  HIP_TRY(c, launch_pathgen(sizeof(T) == 8 ? 1 : 0, o->rng, L, paths, words, normals, (uint32_t)o->n_paths, 256, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (first_bad(c, 1) >= 0) return fail(c, PMC_E_NOT_PD, "correlation matrix is not positive definite");
  return PMC_OK;
}
}  // namespace

extern "C" int pmc_gen_paths(pmc_ctx* c, const pmc_payoff* p, const int32_t* tenv, const pmc_gbm* m,
                             const pmc_opts* o, void* paths_dev, uint32_t* words_dev, void* normals_dev) {
  if (!c || !p || !paths_dev) return fail(c, PMC_E_ARG, "null argument");
  int st = check_model(c, p->prog, m);
  if (st == PMC_OK) st = check_opts(c, o);
  if (st != PMC_OK) return st;
  HIP_TRY(c, hipSetDevice(c->device));
  return o->precision == PMC_FP64 ? gen_paths<double>(c, p, tenv, m, o, paths_dev, words_dev, normals_dev)
                                  : gen_paths<float>(c, p, tenv, m, o, paths_dev, words_dev, normals_dev);
}

// ------------------------------------------------------------ batched ------
namespace {

// The template environment a batch's kernel is generated for, or null.
const int32_t* spec_tenv(const BatchPlan& bp) { return bp.spec ? bp.tenv.data() : nullptr; }

template <typename T>
int batch_prepare(pmc_ctx* c, const pmc_payoff* p, const pmc_batch* b, const pmc_gbm* m, const pmc_opts* o,
                  int block, int ppt, int lanes, BatchPlan& bp) {
  const Program& P = p->prog;
  const int A = (int)P.assets.size();
  const int I = b->n_inst;
  Tables<T> tb;
  tb.desc.reserve(I);
  std::map<std::vector<int32_t>, GridTables> memo;
  for (int i = 0; i < I; ++i) {
    InstanceIn in;
    in.tenv = b->tenv ? b->tenv + (size_t)i * P.tvars.size() : nullptr;
    in.params = b->params ? b->params + (size_t)i * P.params.size() : nullptr;
    if (b->per_instance_model) {
      in.spot = b->spot + (size_t)i * A;
      in.vol = b->vol + (size_t)i * A;
      in.corr = b->corr ? b->corr + (size_t)i * A * A : nullptr;
    } else {
      in.spot = m->spot; in.vol = m->vol; in.corr = m->corr;
    }
    in.instance = b->instance_ids ? b->instance_ids[i] : (uint32_t)i;
    int st = check_instance(c, P, in);
    if (st != PMC_OK) return st;
    st = build_instance<T>(c, P, *m, *o, in, i, tb, &memo);
    if (st != PMC_OK) return st;
  }
  // Streamed paths if every template environment of the batch reads
  // strictly forward (then `lanes` paths per lane, else one).
  const int full = full_capacity(o, tb.max_dims, sizeof(T) == 8 ? 1 : 0);
  bool stream = stream_launch(o, full);
  for (auto it = memo.begin(); stream && it != memo.end(); ++it)
    stream = streamable(p, it->first.data(), o->history ? o->t_now : 0);
  const uint64_t N = o->n_paths;
  if (!stream || N < (uint64_t)lanes) lanes = 1;
  if (ppt == 0) {
    // untuned: enough paths per thread to keep the item count (and the
    // partial-sum buffer) below 2^22, and for short paths enough that a
    // thread's tile simulates at least 128 asset-dates (per-tile set-up and
    // sums otherwise dominate: the surrogate's label batches, 3 assets and
    // at most 5 dates, took 52 ms per chunk at 2 paths per thread and 36.6 at
    // 16), while each instance keeps at least 8 tiles and the batch at
    // least 8 items per CU
    ppt = 1;
    while (ppt < 1024 && (uint64_t)I * ((N + (uint64_t)block * ppt - 1) / ((uint64_t)block * ppt)) > (1ull << 22))
      ppt *= 2;
    const int64_t dims = std::max<int64_t>(1, tb.max_dims);
    for (;;) {
      const uint64_t next_tile = (uint64_t)block * lanes * ppt * 2;
      if (ppt >= 1024 || (int64_t)ppt * dims >= 128 || N < next_tile * 8 ||
          (uint64_t)I * (N / next_tile) < 8ull * (uint64_t)std::max(1, c->n_cu))
        break;
      ppt *= 2;
    }
  }
  // work items (instance, tile), instances with the most slots first; the
  // item list is implicit: item i is tile i % tiles of instance order[i / tiles]
  const uint32_t tile_paths = (uint32_t)block * (uint32_t)ppt * (uint32_t)lanes;
  const uint32_t tiles = (uint32_t)((N + tile_paths - 1) / tile_paths);
  const size_t n_work = (size_t)I * tiles;
  if (n_work > (1u << 26))
    return fail(c, PMC_E_UNSUPPORTED, "batch needs more than 2^26 work items; raise paths per thread");
  std::vector<int> order(I);
  for (int i = 0; i < I; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tb.n_slots[x] > tb.n_slots[y]; });
  for (int i = 0; i < I; ++i) {
    tb.desc[i].n_tiles = tiles;
    tb.desc[i].first_item = (int32_t)((size_t)i * tiles);
  }
  McLaunch L;
  int st = upload<T>(c, P, tb, *o, L, &order);
  if (st != PMC_OK) return st;
  L.tiles = (int)tiles;
  HIP_TRY(c, c->partial.ensure(n_work * sizeof(double2)));
  st = bind_results(c, L, I, true);
  if (st != PMC_OK) return st;
  L.partial = (double2*)c->partial.p;
  L.n_work = (int)n_work;
  L.ppt = ppt;
  L.payoff_out = nullptr;
  bp.L = L;
  bp.lanes = lanes;
  bp.stream = stream;
  if (memo.size() == 1 && !o->history) {
    bp.spec = true;
    bp.tenv = memo.begin()->first;
    bp.tenv.push_back(0);
  }
  int occ = 1;
  if (o->engine == PMC_ENGINE_INTERPRETER) {
    occ = mc_occupancy(sizeof(T) == 8 ? 1 : 0, o->rng, A, P.n_regs, block);
  } else {   // the generated kernel's own register and LDS use
    hipFunction_t f = nullptr;
    std::string err;
    st = p->jit.get(P, c->device, sizeof(T) == 8 ? 1 : 0, o->rng, A, false, &f, err, lanes, full, spec_tenv(bp),
                    false, false, stream);
    if (st != PMC_OK) return fail(c, st, err);
    occ = mc_occupancy_jit(f, block);
  }
  bp.grid = std::max(1, std::min<int>((int)n_work, c->n_cu * occ));
  bp.block = block; bp.ppt = ppt; bp.n_inst = I; bp.full = full;
  bp.n_paths.assign(I, N);
  bp.n_slots = tb.n_slots;
  bp.path_dates = tb.path_dates;
  return PMC_OK;
}

// Enqueue the batched sequence: counter reset and Cholesky factors, then the
// persistent MC kernel (which also reduces each instance).  Captured once
// into a graph.
int batch_enqueue(pmc_ctx* c, const pmc_payoff* p, const pmc_opts* o, const BatchPlan& bp, int prec, int A) {
  int st = prep(c, bp.L, bp.n_inst, A);
  if (st != PMC_OK) return st;
  return launch_engine(c, p, o, prec, false, bp.L, bp.grid, bp.block, bp.lanes, 0, bp.full, spec_tenv(bp),
                       bp.stream);
}

// Everything a captured batch graph bakes in: the kernel variant, the grid,
// and every launch argument (pointers and values alike: the Philox key, the
// Sobol shape, tile counts).  A replay is valid only for an identical key.
void batch_graph_key(std::vector<uint8_t>& k, const pmc_ctx* c, const pmc_payoff* p, const BatchPlan& bp,
                     const pmc_opts* o, int prec) {
  const McLaunch& L = bp.L;
  k.clear();
  put(k, p->serial);   // never reused: a freed payoff's kernels are never replayed
  put(k, prec); put(k, o->rng); put(k, o->engine);
  put(k, bp.n_inst); put(k, bp.grid); put(k, bp.block); put(k, bp.ppt); put(k, bp.full); put(k, bp.spec);
  put(k, bp.lanes); put(k, bp.stream);
  put(k, bp.tenv.size());
  if (!bp.tenv.empty()) put_bytes(k, bp.tenv.data(), bp.tenv.size() * sizeof(int32_t));
  put(k, L.code); put(k, L.consts); put(k, L.desc); put(k, L.itab); put(k, L.rtab); put(k, L.chol);
  put(k, L.chol_in); put(k, L.status); put(k, L.factor); put(k, L.sobol); put(k, L.sobol_bits);
  put(k, L.sobol_hi); put(k, L.sobol_dims); put(k, L.order); put(k, L.tiles); put(k, L.n_work);
  put(k, L.queue); put(k, L.partial); put(k, L.done); put(k, L.result); put(k, L.payoff_out);
  put(k, L.paths); put(k, L.k0); put(k, L.k1); put(k, L.ppt); put(k, L.n_assets); put(k, L.n_regs);
  // buffers the preparation kernel writes
  put(k, c->chol.p); put(k, c->results.dev); put(k, c->counters.p);
}

int batch_run(pmc_ctx* c, const pmc_payoff* p, const BatchPlan& bp, const pmc_opts* o, float* ms_out) {
  const int prec = o->precision == PMC_FP64 ? 1 : 0;
  const int A = (int)p->prog.assets.size();
  std::vector<uint8_t> key;
  batch_graph_key(key, c, p, bp, o, prec);
  if (c->graph.key != key) {
    if (c->graph.exec) { (void)hipGraphExecDestroy(c->graph.exec); c->graph.exec = nullptr; }
    c->graph.key.clear();
    hipStream_t cap = c->stream;
    bool own = false;
    if (!cap) {  // the null stream cannot be captured: use a private one
      HIP_TRY(c, hipStreamCreate(&cap));
      own = true;
    }
    hipStream_t saved = c->stream;
    c->stream = cap;
    if (o->engine != PMC_ENGINE_INTERPRETER) {   // compile outside the capture
      hipFunction_t f = nullptr;
      std::string err;
      int jst = p->jit.get(p->prog, c->device, prec, o->rng, A, false, &f, err, bp.lanes, bp.full, spec_tenv(bp),
                           false, false, bp.stream);
      if (jst != PMC_OK) { c->stream = saved; if (own) (void)hipStreamDestroy(cap); return fail(c, jst, err); }
    }
    HIP_TRY(c, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    int st = batch_enqueue(c, p, o, bp, prec, A);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &graph);
    c->stream = saved;
    if (st != PMC_OK) { if (graph) (void)hipGraphDestroy(graph); if (own) (void)hipStreamDestroy(cap); return st; }
    if (e != hipSuccess) { if (own) (void)hipStreamDestroy(cap); return fail(c, PMC_E_HIP, std::string("graph capture: ") + hipGetErrorString(e)); }
    e = hipGraphInstantiate(&c->graph.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (own) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(c, PMC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    c->graph.key = key;
  }
  HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  HIP_TRY(c, hipGraphLaunch(c->graph.exec, c->stream));
  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  HIP_TRY(c, hipEventSynchronize(c->ev1));
  HIP_TRY(c, hipEventElapsedTime(ms_out, c->ev0, c->ev1));
  return PMC_OK;
}

// A batch tile the kernels can run: whole waves, at most the 256 threads the
// kernels are compiled for, 1 .. 1024 rounds per thread, and 1, 2 or 4
// paths per lane per round.
bool valid_tile(int block, int ppt, int lanes) {
  return block >= 64 && block <= 256 && block % 64 == 0 && ppt >= 1 && ppt <= 1024 &&
         (lanes == 1 || lanes == 2 || lanes == 4);
}

std::string tune_key(pmc_ctx* c, const pmc_payoff* p, const pmc_batch* b, const pmc_opts* o) {
  std::ostringstream k;
  k << c->device_name << '/' << std::hex << p->hash << std::dec << '/' << b->n_inst << '/' << o->n_paths << '/'
    << o->precision << '/' << o->rng << '/' << o->engine;
  return k.str();
}

int check_batch(pmc_ctx* c, const pmc_payoff* p, const pmc_batch* b, const pmc_gbm* m, const pmc_opts* o) {
  if (!c || !p || !b) return fail(c, PMC_E_ARG, "null argument");
  if (b->n_inst < 1) return fail(c, PMC_E_ARG, "n_inst must be >= 1");
  if (b->per_instance_model && (!b->spot || !b->vol)) return fail(c, PMC_E_ARG, "per-instance model needs spot and vol");
  int st = check_model(c, p->prog, m);
  if (st == PMC_OK) st = check_opts(c, o);
  if (st != PMC_OK) return st;
  if (o->payoffs_dev) return fail(c, PMC_E_UNSUPPORTED, "per-path payoff output is not supported for batches");
  if ((uint64_t)b->n_inst * ((o->n_paths + 63) / 64) > (1ull << 31)) return fail(c, PMC_E_UNSUPPORTED, "batch too large");
  return PMC_OK;
}

}  // namespace

extern "C" int pmc_price_batch(pmc_ctx* c, const pmc_payoff* p, const pmc_batch* b, const pmc_gbm* m,
                               const pmc_opts* o, pmc_result* out) {
  int st = check_batch(c, p, b, m, o);
  if (st != PMC_OK) return st;
  if (!out) return fail(c, PMC_E_ARG, "null out");
  HIP_TRY(c, hipSetDevice(c->device));
  int block = o->block ? o->block : 256, ppt = 1, lanes = 1;
  auto it = c->tuned.find(tune_key(c, p, b, o));
  if (it != c->tuned.end() && !o->block) {
    block = it->second.block;
    ppt = it->second.ppt;
    lanes = it->second.lanes;
  } else {
    // untuned: the paths per thread are chosen with the batch's tables
    // (ppt 0), and two paths per lane where paths are streamed (the launch
    // falls back to one otherwise; with one, the batched down-and-out
    // headline ran 1.36x longer)
    ppt = 0;
    if (!o->block && o->n_paths >= (uint64_t)block * 2) lanes = 2;
  }
  // A call identical to the previous batch, with the tables and buffers
  // untouched since: its plan (and graph) serve again; the kernels all run.
  auto& pb = c->prepared_batch;
  const bool keyed = batch_call_key(c->key_buf, p, b, m, o, block, ppt, lanes);
  bool hit = keyed && pb.valid && pb.gen == c->table_gen && pb.key == c->key_buf;
  if (hit) {
    const void* bufs[8];
    buffer_snapshot(c, bufs);
    hit = std::memcmp(bufs, pb.bufs, sizeof bufs) == 0;
  }
  if (!hit) {
    pb.valid = false;
    BatchPlan fresh;
    st = o->precision == PMC_FP64 ? batch_prepare<double>(c, p, b, m, o, block, ppt, lanes, fresh)
                                  : batch_prepare<float>(c, p, b, m, o, block, ppt, lanes, fresh);
    if (st != PMC_OK) return st;
    pb.bp = std::move(fresh);
    if (keyed) {
      pb.key = c->key_buf;
      pb.gen = c->table_gen;
      buffer_snapshot(c, pb.bufs);
      pb.valid = true;
    }
  }
  const BatchPlan& bp = pb.bp;
  float ms = 0;
  st = batch_run(c, p, bp, o, &ms);
  if (st != PMC_OK) return st;
  st = finish(c, bp.n_inst, bp.n_paths.data(), bp.n_slots.data(), PMC_MODE_FUSED, ms, out, 0.0, ms);
  if (st == PMC_OK)
    for (int i = 0; i < bp.n_inst; ++i) out[i].engine_used = engine_used(o);
  return st;
}

extern "C" int pmc_autotune_batch(pmc_ctx* c, const pmc_payoff* p, const pmc_batch* b, const pmc_gbm* m,
                                  const pmc_opts* o, const char* cache_path, int* block_out, int* ppt_out,
                                  int* lanes_out) {
  int st = check_batch(c, p, b, m, o);
  if (st != PMC_OK) return st;
  HIP_TRY(c, hipSetDevice(c->device));
  const std::string key = tune_key(c, p, b, o);
  auto report = [&](int bl, int pp, int ln) {
    c->tuned[key] = {bl, pp, ln};
    if (block_out) *block_out = bl;
    if (ppt_out) *ppt_out = pp;
    if (lanes_out) *lanes_out = ln;
  };
  if (cache_path) {  // cache file: one "key block ppt lanes" line per entry
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      std::istringstream ls(line);
      std::string k;
      int bl = 0, pp = 0, ln = 0;
      if (!(ls >> k >> bl >> pp >> ln)) continue;
      if (k == key && valid_tile(bl, pp, ln)) {   // an entry that is not a launchable tile is ignored
        report(bl, pp, ln);
        return PMC_OK;
      }
    }
  }
  // Candidates: threads per block x rounds per thread x paths per lane (more
  // than one only where the batch streams its paths).  A candidate whose
  // paths per lane the batch cannot use is the one-path tile, timed already.
  const int blocks[] = {64, 128, 256};
  const int ppts[] = {1, 2, 4};
  const int lanes_c[] = {1, 2};
  float best = 1e30f;
  int bb = 256, bpp = 1, bln = 1;
  for (int ln : lanes_c)
    for (int bl : blocks)
      for (int pp : ppts) {
        const uint64_t tile = (uint64_t)bl * pp * ln;
        if ((uint64_t)b->n_inst * ((o->n_paths + tile - 1) / tile) > (1ull << 24)) continue;
        BatchPlan bp;
        st = o->precision == PMC_FP64 ? batch_prepare<double>(c, p, b, m, o, bl, pp, ln, bp)
                                      : batch_prepare<float>(c, p, b, m, o, bl, pp, ln, bp);
        if (st != PMC_OK) return st;
        if (bp.lanes != ln) continue;
        float t = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          float ms = 0;
          st = batch_run(c, p, bp, o, &ms);
          if (st != PMC_OK) return st;
          if (rep > 0) t = std::min(t, ms);   // first replay includes instantiation effects
        }
        if (t < best) { best = t; bb = bl; bpp = pp; bln = ln; }
      }
  report(bb, bpp, bln);
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << key << ' ' << bb << ' ' << bpp << ' ' << bln << '\n';
  }
  return PMC_OK;
}
