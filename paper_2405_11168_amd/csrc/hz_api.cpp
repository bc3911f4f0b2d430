// C ABI of the tetrahedral-stencil FFT homogenization solver: grid handles
// (one microstructure, a batch of load cases per call) and the solve server
// (continuous batching of requests on many grids).
//
// The library owns no device memory: a caller-bound workspace is carved into
// tables, per-load spectra and small status blocks.  All work is issued on the
// caller's stream by the executor (hz_engine.cpp); the stop rule runs on the
// device, so the host only reads status blocks once per tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hz_host.h"

using namespace hz;

namespace {

thread_local std::string g_err;

void check_opts(const hz_opts& o) {
  if (o.precision != HZ_FP64 && o.precision != HZ_FP32_REFINE) fail(HZ_EINVAL, "unknown precision");
  if (!(o.tol > 0) && o.fixed_iters < 0) fail(HZ_EINVAL, "tol must be > 0");
  if (o.max_iters < 0 || o.max_iters > kMaxIters) fail(HZ_EINVAL, "max_iters out of range [0, 1000000]");
  if (o.fixed_iters > kTraceCap - 1) fail(HZ_EINVAL, "fixed_iters out of range [0, 4096]");
  if (o.precision == HZ_FP32_REFINE && o.fixed_iters == 0) fail(HZ_EINVAL, "HZ_FP32_REFINE needs fixed_iters >= 1");
  if ((o.trace_residual || o.trace_mean) && o.fixed_iters < 0 && o.max_iters > kTraceCap - 1)
    fail(HZ_EINVAL, "a trace needs max_iters <= 4096");
  if (o.fields_on_device != 0 && o.fields_on_device != 1) fail(HZ_EINVAL, "fields_on_device must be 0 or 1");
  if (o.inner_max < 0 || o.inner_max > 100000) fail(HZ_EINVAL, "inner_max out of range");
  if (o.scheme < HZ_SCHEME_AUTO || o.scheme > HZ_SCHEME_STRAIN) fail(HZ_EINVAL, "unknown scheme");
  if (o.scheme == HZ_SCHEME_STRAIN && o.precision != HZ_FP64) fail(HZ_EINVAL, "the strain-based scheme needs HZ_FP64");
  if (o.loading != HZ_LOAD_STRAIN && o.loading != HZ_LOAD_STRESS) fail(HZ_EINVAL, "unknown loading");
  if (o.loading == HZ_LOAD_STRESS && o.precision != HZ_FP64) fail(HZ_EINVAL, "applied stress needs HZ_FP64");
  if ((o.u_init || o.Ebar_init) && (o.precision != HZ_FP64 || o.scheme == HZ_SCHEME_STRAIN))
    fail(HZ_EINVAL, "an initial guess needs HZ_FP64 and the spectral or stencil scheme");
  if (o.green < HZ_GREEN_TETRA || o.green > HZ_GREEN_CONTINUOUS) fail(HZ_EINVAL, "unknown Green operator");
  if (o.green != HZ_GREEN_TETRA && o.precision != HZ_FP64)
    fail(HZ_EINVAL, "the comparison Green operators need HZ_FP64");
  if (o.green != HZ_GREEN_TETRA && o.scheme != HZ_SCHEME_AUTO && o.scheme != HZ_SCHEME_SPECTRAL)
    fail(HZ_EINVAL, "the comparison Green operators run in the spectral scheme");
}
static_assert(HZ_GREEN_TETRA == GREEN_TETRA && HZ_GREEN_ROTATED == GREEN_ROTATED &&
                  HZ_GREEN_CONTINUOUS == GREEN_CONTINUOUS,
              "Green operator ids");

int pick_form(const Shape& sh, int scheme) {
  if (scheme == HZ_SCHEME_STENCIL && !sh.stencil) fail(HZ_EINVAL, "the stencil scheme does not fit this grid's x rows");
  if (scheme == HZ_SCHEME_SPECTRAL || scheme == HZ_SCHEME_STRAIN) return scheme;
  return sh.stencil ? HZ_SCHEME_STENCIL : HZ_SCHEME_SPECTRAL;
}

void check_loads(const double* E, int n) {
  for (int i = 0; i < 6 * n; ++i)
    if (!std::isfinite(E[i])) fail(HZ_EINVAL, "non-finite applied load");
}

// one load case ready for the executor
void setup_prob(Prob& p, int slot, const Shape* sh, const ShapeTables& tab, const MaterialTables& mt,
                const Material& m, const Reference& R, const ProbBuffers& b, const double* E, int load,
                const hz_opts& o) {
  p = Prob{};
  p.slot = slot;
  p.shape = sh;
  p.tab = tab;
  p.prec = o.precision;
  p.form = o.green != HZ_GREEN_TETRA ? HZ_SCHEME_SPECTRAL : pick_form(*sh, o.scheme);
  p.green = o.green;
  if (o.green == HZ_GREEN_CONTINUOUS && sh->subc == 0)
    fail(HZ_EINVAL, "N3 too large for the continuous-frequency operator's z kernels");
  p.loading = o.loading;
  for (int c = 0; c < 6; ++c) p.E[c] = E[c];
  if (o.loading == HZ_LOAD_STRESS && o.Ebar_init) {
    for (int c = 0; c < 6; ++c) p.Eb0[c] = o.Ebar_init[6 * (size_t)load + c];
  } else if (o.loading == HZ_LOAD_STRESS) {
    // initial mean strain lambda0^-1:sigma^a (Algorithm 1)
    for (int i = 0; i < 6; ++i) {
      double a = 0;
      for (int j = 0; j < 6; ++j) a += R.S0[i * 6 + j] * E[j];
      p.Eb0[i] = a;
    }
  } else {
    for (int c = 0; c < 6; ++c) p.Eb0[c] = E[c];
  }
  for (int c = 0; c < 6; ++c) p.Ebar[c] = p.Eb0[c];
  if (o.u_init) p.u_init = o.u_init + (size_t)load * 6 * sh->geo.S;  // 3 S complex = 6 S doubles
  p.tol = o.tol;
  p.max_iters = o.max_iters;
  p.fixed_iters = o.fixed_iters;
  // a fixed FP32 count is one round 0 of exactly that many updates, measured by one sweep
  p.inner_max = o.fixed_iters >= 0 ? o.fixed_iters : (o.inner_max > 0 ? o.inner_max : 400);
  p.rho = o.inner_rho > 0 ? o.inner_rho : 1e-3;
  Desc& d = p.base;
  d = Desc{};
  d.spec = b.spec;
  d.u[0] = b.u0;
  d.u[1] = b.u1;
  d.u64 = b.u64;
  d.r32 = b.r32;
  d.phase = mt.phase;
  d.C64 = mt.C64;
  d.C32 = mt.C32;
  d.iso = m.iso;
  d.c0_iso = R.iso;
  d.lam0 = R.lam0;
  d.mu0 = R.mu0;
  d.part_sig = b.part_sig;
  d.part_res = b.part_res;
  d.trace = b.trace;
  d.tau64 = mt.tau64;
  d.tau32 = mt.tau32;
  d.green = o.green;
  d.n_phases = m.n_phases;
  d.loading = o.loading;
  if (o.loading == HZ_LOAD_STRESS) {
    auto frob = [](const double* t) {
      return std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2] + 2.0 * (t[3] * t[3] + t[4] * t[4] + t[5] * t[5]));
    };
    for (int c = 0; c < 6; ++c) d.sig_a[c] = E[c];
    std::memcpy(d.S0, R.S0, sizeof(d.S0));
    // stop-rule scale: ||sigma^a||, else the eigenstress scale ||<lambda:eps0>||, else 1
    d.sref = frob(E);
    if (!(d.sref > 0)) d.sref = frob(m.tau_mean);
    if (!(d.sref > 0)) d.sref = 1.0;
  }
  std::memcpy(d.C0, R.C0t, sizeof(d.C0));
}

int worst_code(int worst, int code) {
  if (code < 0) return std::min(worst, code);
  if (worst >= 0) return std::max(worst, code);
  return worst;
}

void fill_info(const Prob& p, double t0_ms, double wall, hz_info& in) {
  in.status = p.code;
  in.iters = p.iters;
  in.outer_rounds = p.rounds;
  in.precision_used = p.fb ? HZ_FP64 : p.prec;
  in.residual = p.err;
  in.seconds = 1e-3 * (p.t_done - t0_ms);
  in.seconds_to_1e6 = p.t_1e6 >= 0 ? 1e-3 * (p.t_1e6 - t0_ms) : -1.0;
  in.wall_seconds = wall;
  for (int c = 0; c < 6; ++c) in.Ebar[c] = p.Ebar[c];
}

// first-fit allocator over a byte range, 256-byte granules, neighbours coalesced
struct Arena {
  std::map<size_t, size_t> free_;
  size_t total = 0;
  void init(size_t n) {
    free_.clear();
    total = n;
    if (n) free_[0] = n;
  }
  long long alloc(size_t n) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        const size_t off = it->first, rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        return (long long)off;
      }
    return -1;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }
};

}  // namespace

// ===========================================================================
// grid handle
// ===========================================================================
struct hz_grid_s {
  Shape shape;
  std::shared_ptr<Material> mat;
  // bound workspace
  char* ws = nullptr;
  int64_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int prec = -1;
  int cap = 0;
  struct Off {
    size_t shape_tab, mat_tab, engine, fields, probs, pb, total;
  } off{};
  ShapeTables tab{};
  MaterialTables mtab{};
  std::unique_ptr<Engine> eng;
  std::unique_ptr<Engine> seng;  // executor of hz_solve_static (pageable host mirrors)
  Prof prof;
  std::vector<Prob> probs;
  int last_prec = -1;
};

namespace {

void grid_layout(const hz_grid_s* g, int prec, int nl, hz_grid_s::Off& o) {
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t r = p;
    p = align_up(p + bytes);
    return r;
  };
  o.shape_tab = take(shape_table_bytes(g->shape));
  o.mat_tab = take(material_table_bytes(g->mat ? g->mat->n_phases : 1, g->shape.geo.N));
  o.engine = take(Engine::table_bytes(nl));
  o.fields = take((size_t)12 * g->shape.geo.N * 8);
  o.pb = prob_bytes(g->shape, prec, true);
  o.probs = take((size_t)nl * o.pb);
  o.total = p;
}

void check_bound(hz_grid g) {
  if (!g->mat) fail(HZ_ENOMATERIAL, "material not set");
  if (!g->ws) fail(HZ_EWORKSPACE, "workspace not bound");
}

int grid_solve(hz_grid g, int nl, const double* E, const hz_opts& o, double* sigma_mean, double* eps_out,
               double* sig_out, hz_info* info) {
  const auto t_call = std::chrono::steady_clock::now();
  const Reference R = make_reference(o, *g->mat);
  Engine& e = *g->eng;
  e.live.clear();  // a solve that failed part-way leaves nothing behind
  e.check_every = std::max(1, o.check_every);
  g->probs.assign(nl, Prob{});
  for (int b = 0; b < nl; ++b) {
    const ProbBuffers pb = carve_prob(g->shape, g->prec, true, g->ws + g->off.probs + (size_t)b * g->off.pb);
    setup_prob(g->probs[b], b, &g->shape, g->tab, g->mtab, *g->mat, R, pb, E + 6 * b, b, o);
    // the strain-based form keeps its 12 strain spectra in the block of load nl + b
    if (g->probs[b].form == HZ_SCHEME_STRAIN) g->probs[b].base.state = g->ws + g->off.probs + (size_t)(nl + b) * g->off.pb;
  }
  g->last_prec = -1;
  e.start_clock();
  for (auto& p : g->probs) e.add(&p);
  while (!e.live.empty()) e.tick();
  g->last_prec = o.precision;
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_call).count();
  int worst = HZ_OK;
  const int stride = (o.fixed_iters >= 0 ? o.fixed_iters : o.max_iters) + 1;
  for (int b = 0; b < nl; ++b) {
    const Prob& p = g->probs[b];
    worst = worst_code(worst, p.code);
    if (sigma_mean)
      for (int c = 0; c < 6; ++c) sigma_mean[6 * b + c] = p.mean[c];
    if (info) fill_info(p, 0.0, wall, info[b]);
    if (o.precision == HZ_FP64 && (o.trace_residual || o.trace_mean)) {
      const int ntr = (int)p.trace.size() / 7;
      for (int t = 0; t < ntr && t < stride; ++t) {
        if (o.trace_residual) o.trace_residual[(size_t)b * stride + t] = p.trace[(size_t)t * 7];
        if (o.trace_mean)
          for (int c = 0; c < 6; ++c) o.trace_mean[((size_t)b * stride + t) * 6 + c] = p.trace[(size_t)t * 7 + 1 + c];
      }
    }
  }
  if (eps_out || sig_out) {
    const size_t n6 = (size_t)6 * g->shape.geo.N;
    double* fe = reinterpret_cast<double*>(g->ws + g->off.fields);
    const bool dev = o.fields_on_device != 0;
    for (int b = 0; b < nl; ++b) {
      // device outputs are written by the field writer in place; host outputs (and an
      // output the caller did not ask for) go through the workspace's field buffer
      double* de = dev && eps_out ? eps_out + (size_t)b * n6 : fe;
      double* ds = dev && sig_out ? sig_out + (size_t)b * n6 : fe + n6;
      output_fields(e, g->probs[b], de, ds);
      if (dev) continue;
      if (eps_out)
        hip_check(hipMemcpy(eps_out + (size_t)b * n6, fe, n6 * 8, hipMemcpyDeviceToHost), "eps D2H");
      if (sig_out)
        hip_check(hipMemcpy(sig_out + (size_t)b * n6, fe + n6, n6 * 8, hipMemcpyDeviceToHost), "sigma D2H");
    }
  }
  return worst;
}

}  // namespace

// ===========================================================================
// solve server: requests (a grid's material + n loads) admitted while their
// buffers fit the arena, advanced together tick by tick, retired on completion
// ===========================================================================
namespace {

struct ShapeEntry {
  Shape shape;
  size_t off = 0, bytes = 0;
  ShapeTables tab{};
  int refs = 0;
};

struct MatEntry {
  std::shared_ptr<Material> mat;
  size_t off = 0, bytes = 0;
  MaterialTables tab{};
  int refs = 0;
};

struct Req {
  int64_t id = 0;
  int state = 0;  // 0 queued, 1 running, 2 finished
  std::shared_ptr<Material> mat;
  Shape shape;
  hz_opts opts{};
  Reference ref{};
  int n = 0;
  std::vector<double> E;
  ShapeEntry* se = nullptr;
  MatEntry* me = nullptr;
  size_t off = 0, bytes = 0, pb = 0;
  std::vector<Prob> probs;
  int remaining = 0;
  int code = HZ_OK;
  std::chrono::steady_clock::time_point t_submit, t_done;
};

}  // namespace

struct hz_server_s {
  char* ws = nullptr;
  int64_t bytes = 0;
  hipStream_t stream = nullptr;
  int max_problems = 0;
  Engine eng;
  Prof prof;
  Arena arena;
  size_t arena_base = 0;
  std::map<std::tuple<int, int, int>, std::unique_ptr<ShapeEntry>> shapes;
  std::map<const Material*, std::unique_ptr<MatEntry>> mats;
  std::deque<Req*> queue;
  std::map<int64_t, std::unique_ptr<Req>> reqs;
  std::vector<int> free_slots;
  int64_t next_id = 1;
  int running = 0;
};

namespace {

size_t request_bytes(const Shape& sh, const Material& m, int prec, int n) {
  return (size_t)n * prob_bytes(sh, prec, prec == HZ_FP64) + align_up(shape_table_bytes(sh)) +
         align_up(material_table_bytes(m));
}

void release_request_memory(hz_server s, Req* r) {
  s->arena.release(r->off, r->bytes);
  if (--r->se->refs == 0) {
    s->arena.release(r->se->off, r->se->bytes);
    s->shapes.erase(std::make_tuple(r->shape.geo.N1, r->shape.geo.N2, r->shape.geo.N3));
  }
  if (--r->me->refs == 0) {
    s->arena.release(r->me->off, r->me->bytes);
    s->mats.erase(r->mat.get());
  }
  r->se = nullptr;
  r->me = nullptr;
  for (auto& p : r->probs) s->free_slots.push_back(p.slot);
}

// admit queued requests in arrival order while their buffers and slots fit
void admit(hz_server s) {
  while (!s->queue.empty()) {
    Req* r = s->queue.front();
    if ((int)s->free_slots.size() < r->n) return;
    const auto key = std::make_tuple(r->shape.geo.N1, r->shape.geo.N2, r->shape.geo.N3);
    auto sit = s->shapes.find(key);
    auto mit = s->mats.find(r->mat.get());
    const long long off = s->arena.alloc(r->bytes);
    if (off < 0) return;
    long long soff = -1, moff = -1;
    const size_t sbytes = shape_table_bytes(r->shape), mbytes = material_table_bytes(*r->mat);
    if (sit == s->shapes.end() && (soff = s->arena.alloc(sbytes)) < 0) {
      s->arena.release((size_t)off, r->bytes);
      return;
    }
    if (mit == s->mats.end() && (moff = s->arena.alloc(mbytes)) < 0) {
      s->arena.release((size_t)off, r->bytes);
      if (soff >= 0) s->arena.release((size_t)soff, sbytes);
      return;
    }
    char* base = s->ws + s->arena_base;
    if (sit == s->shapes.end()) {
      auto se = std::make_unique<ShapeEntry>();
      se->shape = r->shape;
      se->off = (size_t)soff;
      se->bytes = sbytes;
      se->tab = upload_shape_tables(se->shape, base + soff, s->stream);
      sit = s->shapes.emplace(key, std::move(se)).first;
    }
    if (mit == s->mats.end()) {
      auto me = std::make_unique<MatEntry>();
      me->mat = r->mat;
      me->off = (size_t)moff;
      me->bytes = mbytes;
      me->tab = upload_material_tables(*r->mat, base + moff, s->stream);
      mit = s->mats.emplace(r->mat.get(), std::move(me)).first;
    }
    r->se = sit->second.get();
    r->me = mit->second.get();
    r->se->refs++;
    r->me->refs++;
    r->off = (size_t)off;
    r->probs.assign(r->n, Prob{});
    for (int b = 0; b < r->n; ++b) {
      const int slot = s->free_slots.back();
      s->free_slots.pop_back();
      const ProbBuffers pb = carve_prob(r->se->shape, r->opts.precision, r->opts.precision == HZ_FP64,
                                        base + r->off + (size_t)b * r->pb);
      setup_prob(r->probs[b], slot, &r->se->shape, r->se->tab, r->me->tab, *r->mat, r->ref, pb, r->E.data() + 6 * b,
                 b, r->opts);
      r->probs[b].owner = r;
    }
    for (auto& p : r->probs) s->eng.add(&p);
    r->remaining = r->n;
    r->state = 1;
    s->running++;
    s->queue.pop_front();
  }
}

}  // namespace

// ===========================================================================
// Static device workspace of hz_solve_static
// ===========================================================================
namespace {

// One array per GPU the library runs on, held until the process ends.  In host code
// its name is only a stand-in: kernels receive the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's array, looked up once per device
char* scratch_address() {
  int dev = -1;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) fail(HZ_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) fail(HZ_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

// The grid's own binding, set aside while a solve runs on the static workspace and
// put back afterwards (also when the solve fails).
struct BindingSwap {
  hz_grid g;
  char* ws;
  int64_t ws_bytes;
  hipStream_t stream;
  int prec, cap, last_prec;
  hz_grid_s::Off off;
  ShapeTables tab;
  MaterialTables mtab;
  std::unique_ptr<Engine> eng;
  std::vector<Prob> probs;
  explicit BindingSwap(hz_grid gg)
      : g(gg), ws(gg->ws), ws_bytes(gg->ws_bytes), stream(gg->stream), prec(gg->prec), cap(gg->cap),
        last_prec(gg->last_prec), off(gg->off), tab(gg->tab), mtab(gg->mtab), eng(std::move(gg->eng)),
        probs(std::move(gg->probs)) {}
  ~BindingSwap() {
    g->seng = std::move(g->eng);
    g->eng = std::move(eng);
    g->probs = std::move(probs);
    g->ws = ws;
    g->ws_bytes = ws_bytes;
    g->stream = stream;
    g->prec = prec;
    g->cap = cap;
    g->last_prec = last_prec;
    g->off = off;
    g->tab = tab;
    g->mtab = mtab;
  }
};

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
#define HZ_GUARD_BEGIN try {
#define HZ_GUARD_END                \
  }                                 \
  catch (const HzError& e) {        \
    g_err = e.msg;                  \
    return e.code;                  \
  }                                 \
  catch (const std::exception& e) { \
    g_err = e.what();               \
    return HZ_EINVAL;               \
  }

extern "C" {

void hz_default_opts(hz_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->max_iters = 2000;
  o->precision = HZ_FP64;
  o->ref_mode = 0;
  o->fixed_iters = -1;
  o->check_every = 8;
  o->inner_rho = 1e-3;
  o->inner_max = 400;
  o->scheme = HZ_SCHEME_AUTO;
  o->loading = HZ_LOAD_STRAIN;
  o->green = HZ_GREEN_TETRA;
}

const char* hz_last_error(void) { return g_err.c_str(); }

int hz_create_grid(int32_t n1, int32_t n2, int32_t n3, hz_grid* out) {
  HZ_GUARD_BEGIN
  if (!out) fail(HZ_EINVAL, "out is NULL");
  *out = nullptr;
  if (n1 < 2 || n2 < 2 || n3 < 2) fail(HZ_EINVAL, "grid sizes must be >= 2");
  if ((n1 | n2 | n3) & 1) fail(HZ_EODD, "grid sizes must be even");
  if (n1 > 4096 || n2 > 2048 || n3 > 2048) fail(HZ_EINVAL, "grid too large");
  if (!factor_ok(n1) || !factor_ok(n2) || !factor_ok(n3))
    fail(HZ_EINVAL, "grid sizes must have prime factors in {2,3,5,7}");
  auto g = std::make_unique<hz_grid_s>();
  g->shape.init(n1, n2, n3);
  *out = g.release();
  return HZ_OK;
  HZ_GUARD_END
}

int hz_set_material(hz_grid g, int32_t n_phases, const double* C_voigt, const uint16_t* phase) {
  HZ_GUARD_BEGIN
  if (!g) fail(HZ_EINVAL, "NULL handle");
  g->mat = make_material(g->shape.geo, n_phases, C_voigt, phase);
  g->ws = nullptr;  // tables must be re-uploaded
  return HZ_OK;
  HZ_GUARD_END
}

int hz_set_eigenstrain(hz_grid g, int32_t n_phases, const double* eps0) {
  HZ_GUARD_BEGIN
  if (!g) fail(HZ_EINVAL, "NULL handle");
  if (!g->mat) fail(HZ_ENOMATERIAL, "material not set");
  if (eps0 && n_phases != g->mat->n_phases) fail(HZ_EINVAL, "eigenstrain table must have one row per phase");
  g->mat = with_eigenstrain(*g->mat, eps0);
  g->ws = nullptr;  // tables must be re-uploaded
  return HZ_OK;
  HZ_GUARD_END
}

int64_t hz_workspace_bytes(hz_grid g, int32_t precision, int32_t n_loads) {
  HZ_GUARD_BEGIN
  if (!g || n_loads <= 0 || n_loads > 1024 || (precision != HZ_FP64 && precision != HZ_FP32_REFINE))
    fail(HZ_EINVAL, "bad workspace query");
  hz_grid_s::Off o;
  grid_layout(g, precision, n_loads, o);
  return (int64_t)o.total;
  HZ_GUARD_END
}

int hz_bind_workspace(hz_grid g, void* dev_ptr, int64_t bytes, void* hip_stream, int32_t precision,
                      int32_t n_loads) {
  HZ_GUARD_BEGIN
  if (!g || !dev_ptr || n_loads <= 0 || (precision != HZ_FP64 && precision != HZ_FP32_REFINE))
    fail(HZ_EINVAL, "bad bind arguments");
  if (n_loads > 1024) fail(HZ_EINVAL, "at most 1024 loads per handle");
  if (!g->mat) fail(HZ_ENOMATERIAL, "material not set");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) fail(HZ_EINVAL, "workspace must be 256-byte aligned");
  hz_grid_s::Off o;
  grid_layout(g, precision, n_loads, o);
  if ((int64_t)o.total > bytes) fail(HZ_EWORKSPACE, "workspace too small: need " + std::to_string(o.total) + " bytes");
  g->ws = nullptr;
  g->probs.clear();
  g->last_prec = -1;
  char* ws = static_cast<char*>(dev_ptr);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (!g->eng || g->eng->cap < n_loads) {
    g->eng = std::make_unique<Engine>();
    g->eng->init(n_loads);
  }
  g->eng->prof = &g->prof;
  g->eng->bind(ws + o.engine, st);
  g->tab = upload_shape_tables(g->shape, ws + o.shape_tab, st);
  g->mtab = upload_material_tables(*g->mat, ws + o.mat_tab, st);
  g->off = o;
  g->ws = ws;
  g->ws_bytes = bytes;
  g->stream = st;
  g->prec = precision;
  g->cap = n_loads;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_solve(hz_grid g, int32_t n_loads, const double* E, const hz_opts* o, double* sigma_mean, double* eps_out,
             double* sig_out, hz_info* info) {
  HZ_GUARD_BEGIN
  if (!g || !E || !o || n_loads <= 0) fail(HZ_EINVAL, "bad solve arguments");
  check_opts(*o);
  check_loads(E, n_loads);
  check_bound(g);
  if (n_loads > g->cap) fail(HZ_EWORKSPACE, "workspace bound for fewer loads");
  if (o->scheme == HZ_SCHEME_STRAIN && 2 * n_loads > g->cap)
    fail(HZ_EWORKSPACE, "the strain-based scheme needs a workspace bound for 2 n_loads loads");
  if (o->precision != g->prec) fail(HZ_EWORKSPACE, "workspace bound for another precision");
  return grid_solve(g, n_loads, E, *o, sigma_mean, eps_out, sig_out, info);
  HZ_GUARD_END
}

int hz_solve_static(hz_grid g, void* hip_stream, int32_t n_loads, const double* E, const hz_opts* o,
                    double* sigma_mean, double* eps_out, double* sig_out, hz_info* info) {
  HZ_GUARD_BEGIN
  if (!g || !E || !o || n_loads <= 0) fail(HZ_EINVAL, "bad solve arguments");
  check_opts(*o);
  check_loads(E, n_loads);
  if (!g->mat) fail(HZ_ENOMATERIAL, "material not set");
  const int nb = o->scheme == HZ_SCHEME_STRAIN ? 2 * n_loads : n_loads;
  if (nb > 1024) fail(HZ_EINVAL, "at most 1024 loads per handle");
  hz_grid_s::Off off;
  grid_layout(g, o->precision, nb, off);
  if (off.total > kScratchBytes)
    fail(HZ_EWORKSPACE, "hz_solve_static: the problem needs " + std::to_string(off.total) +
                            " bytes of workspace; the static workspace holds " + std::to_string(kScratchBytes));
  char* base = scratch_address();
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  BindingSwap keep(g);
  if (!g->seng || g->seng->cap < nb) {
    g->seng.reset();
    auto e = std::make_unique<Engine>();
    e->init(nb, false);
    g->seng = std::move(e);
  }
  g->eng = std::move(g->seng);
  g->eng->prof = &g->prof;
  g->eng->bind(base + off.engine, st);
  g->tab = upload_shape_tables(g->shape, base + off.shape_tab, st);
  g->mtab = upload_material_tables(*g->mat, base + off.mat_tab, st);
  g->off = off;
  g->ws = base;
  g->ws_bytes = (int64_t)kScratchBytes;
  g->stream = st;
  g->prec = o->precision;
  g->cap = nb;
  return grid_solve(g, n_loads, E, *o, sigma_mean, eps_out, sig_out, info);
  HZ_GUARD_END
}

int hz_effective_stiffness(hz_grid g, const hz_opts* o, double C_eff[36], hz_info info[6]) {
  HZ_GUARD_BEGIN
  if (!g || !o || !C_eff) fail(HZ_EINVAL, "bad arguments");
  if (o->loading != HZ_LOAD_STRAIN) fail(HZ_EINVAL, "the effective stiffness takes unit strains");
  if (g->mat && !g->mat->eig.empty()) fail(HZ_EINVAL, "the effective stiffness needs a material without eigenstrains");
  double E[36] = {0};
  for (int J = 0; J < 6; ++J) E[J * 6 + J] = J < 3 ? 1.0 : 0.5;
  double sm[36];
  const int rc = hz_solve(g, 6, E, o, sm, nullptr, nullptr, info);
  if (rc < 0) return rc;
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) C_eff[I * 6 + J] = sm[J * 6 + I];
  return rc;
  HZ_GUARD_END
}

int hz_get_displacement(hz_grid g, int32_t load, double* out) {
  HZ_GUARD_BEGIN
  if (!g || !out) fail(HZ_EINVAL, "bad arguments");
  check_bound(g);
  if (g->last_prec < 0 || load < 0 || load >= (int)g->probs.size()) fail(HZ_EINVAL, "no such load in the last solve");
  const Prob& p = g->probs[load];
  if (p.form == HZ_SCHEME_STRAIN) fail(HZ_EINVAL, "the strain-based scheme keeps strains, not the displacement");
  const size_t n = (size_t)3 * g->shape.geo.S;
  const void* src = p.prec == HZ_FP64 ? (p.parity ? p.base.u[1] : p.base.u[0]) : p.base.u64;
  hip_check(hipStreamSynchronize(g->stream), "sync");
  hip_check(hipMemcpy(out, src, n * 16, hipMemcpyDeviceToHost), "u D2H");
  return HZ_OK;
  HZ_GUARD_END
}

int hz_scheme_available(hz_grid g, int32_t scheme) {
  HZ_GUARD_BEGIN
  if (!g) fail(HZ_EINVAL, "NULL handle");
  if (scheme == HZ_SCHEME_SPECTRAL || scheme == HZ_SCHEME_AUTO || scheme == HZ_SCHEME_STRAIN) return 1;
  if (scheme == HZ_SCHEME_STENCIL) return g->shape.stencil ? 1 : 0;
  fail(HZ_EINVAL, "unknown scheme");
  HZ_GUARD_END
}

int hz_reference_medium(int32_t n_phases, const double* C_voigt, double C0_out[36]) {
  HZ_GUARD_BEGIN
  if (n_phases <= 0 || !C_voigt || !C0_out) fail(HZ_EINVAL, "bad arguments");
  auto_reference(n_phases, C_voigt, C0_out);
  return HZ_OK;
  HZ_GUARD_END
}

int hz_profile(hz_grid g, int32_t enable) {
  HZ_GUARD_BEGIN
  if (!g) fail(HZ_EINVAL, "NULL handle");
  if (enable < 0 || enable >= 2 + 2 * K_COUNT) fail(HZ_EINVAL, "profile mode out of range");
  if (enable) g->prof.reset();
  g->prof.on = enable != 0;
  g->prof.only = enable >= 2 ? enable - 2 : -1;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_profile_read(hz_grid g, int32_t max, const char** names, double* total_ms, int64_t* launches) {
  HZ_GUARD_BEGIN
  if (!g) fail(HZ_EINVAL, "NULL handle");
  static std::vector<std::string> store;
  if (store.empty())
    for (int k = 0; k < K_COUNT; ++k)
      for (int d = 0; d < 2; ++d) store.push_back(std::string(kKindNames[k]) + (d ? "_f64" : "_f32"));
  int n = 0;
  for (int k = 0; k < K_COUNT; ++k)
    for (int d = 0; d < 2; ++d) {
      if (n < max) {
        if (names) names[n] = store[k * 2 + d].c_str();
        if (total_ms) total_ms[n] = g->prof.ms[k][d];
        if (launches) launches[n] = g->prof.n[k][d];
      }
      ++n;
    }
  return n;
  HZ_GUARD_END
}

void hz_destroy_grid(hz_grid g) {
  if (!g) return;
  if (g->stream && g->ws) (void)hipStreamSynchronize(g->stream);
  delete g;
}

// ---------------------------------------------------------------------------
// server
// ---------------------------------------------------------------------------
int64_t hz_server_bytes(int32_t max_problems) {
  HZ_GUARD_BEGIN
  if (max_problems <= 0 || max_problems > 4096) fail(HZ_EINVAL, "max_problems out of range [1, 4096]");
  return (int64_t)align_up(Engine::table_bytes(max_problems));
  HZ_GUARD_END
}

int64_t hz_request_bytes(hz_grid g, int32_t precision, int32_t n_loads) {
  HZ_GUARD_BEGIN
  if (!g || n_loads <= 0 || (precision != HZ_FP64 && precision != HZ_FP32_REFINE)) fail(HZ_EINVAL, "bad query");
  if (!g->mat) fail(HZ_ENOMATERIAL, "material not set");
  return (int64_t)request_bytes(g->shape, *g->mat, precision, n_loads);
  HZ_GUARD_END
}

int hz_server_create(void* dev_ptr, int64_t bytes, void* hip_stream, int32_t max_problems, int32_t check_every,
                     hz_server* out) {
  HZ_GUARD_BEGIN
  if (!out) fail(HZ_EINVAL, "out is NULL");
  *out = nullptr;
  if (!dev_ptr || bytes <= 0) fail(HZ_EINVAL, "bad workspace");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) fail(HZ_EINVAL, "workspace must be 256-byte aligned");
  if (max_problems <= 0 || max_problems > 4096) fail(HZ_EINVAL, "max_problems out of range [1, 4096]");
  const size_t fixed = align_up(Engine::table_bytes(max_problems));
  if ((size_t)bytes <= fixed) fail(HZ_EWORKSPACE, "workspace smaller than the server tables");
  auto s = std::make_unique<hz_server_s>();
  s->ws = static_cast<char*>(dev_ptr);
  s->bytes = bytes;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->max_problems = max_problems;
  s->eng.init(max_problems);
  s->eng.prof = &s->prof;
  s->eng.bind(s->ws, s->stream);
  s->eng.check_every = std::max(1, check_every);
  s->arena_base = fixed;
  s->arena.init((size_t)bytes - fixed);
  for (int i = max_problems - 1; i >= 0; --i) s->free_slots.push_back(i);
  *out = s.release();
  return HZ_OK;
  HZ_GUARD_END
}

int hz_server_submit(hz_server s, hz_grid g, int32_t n_loads, const double* E, const hz_opts* o, int64_t* id) {
  HZ_GUARD_BEGIN
  if (!s || !g || !E || !o || !id || n_loads <= 0) fail(HZ_EINVAL, "bad submit arguments");
  if (!g->mat) fail(HZ_ENOMATERIAL, "material not set");
  check_opts(*o);
  pick_form(g->shape, o->scheme);
  if (o->fixed_iters >= 0) fail(HZ_EINVAL, "fixed_iters is not served");
  if (o->scheme == HZ_SCHEME_STRAIN) fail(HZ_EINVAL, "the strain-based scheme is not served (hz_solve only)");
  if (o->green != HZ_GREEN_TETRA) fail(HZ_EINVAL, "the comparison Green operators are not served (hz_solve only)");
  if (o->u_init || o->Ebar_init) fail(HZ_EINVAL, "initial guesses are not served (hz_solve only)");
  check_loads(E, n_loads);
  if (n_loads > s->max_problems) fail(HZ_EWORKSPACE, "more loads than the server has slots");
  auto r = std::make_unique<Req>();
  r->mat = g->mat;
  r->shape = g->shape;
  r->opts = *o;
  r->opts.trace_residual = nullptr;
  r->opts.trace_mean = nullptr;
  r->ref = make_reference(*o, *g->mat);
  r->n = n_loads;
  r->E.assign(E, E + 6 * (size_t)n_loads);
  r->pb = prob_bytes(r->shape, o->precision, o->precision == HZ_FP64);
  r->bytes = (size_t)n_loads * r->pb;
  if (request_bytes(r->shape, *r->mat, o->precision, n_loads) > s->arena.total)
    fail(HZ_EWORKSPACE, "request larger than the server workspace");
  r->id = s->next_id++;
  r->t_submit = std::chrono::steady_clock::now();
  *id = r->id;
  s->queue.push_back(r.get());
  s->reqs.emplace(r->id, std::move(r));
  return HZ_OK;
  HZ_GUARD_END
}

int hz_server_step(hz_server s, int32_t* completed) {
  HZ_GUARD_BEGIN
  if (!s) fail(HZ_EINVAL, "NULL handle");
  int done = 0;
  if (s->eng.live.empty()) s->eng.start_clock();  // device clock restarts whenever the server is idle
  admit(s);
  if (!s->eng.live.empty()) {
    const std::vector<Prob*> fin = s->eng.tick();
    const auto now = std::chrono::steady_clock::now();
    for (Prob* p : fin) {
      Req* r = static_cast<Req*>(p->owner);
      r->code = worst_code(r->code, p->code);
      if (--r->remaining == 0) {
        r->state = 2;
        r->t_done = now;
        release_request_memory(s, r);
        s->running--;
        ++done;
      }
    }
  }
  if (completed) *completed = done;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_server_query(hz_server s, int64_t id, double* sigma_mean, hz_info* info) {
  HZ_GUARD_BEGIN
  if (!s) fail(HZ_EINVAL, "NULL handle");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) fail(HZ_EINVAL, "unknown request id");
  Req* r = it->second.get();
  if (r->state != 2) return HZ_PENDING;
  const double wall = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  for (int b = 0; b < r->n; ++b) {
    const Prob& p = r->probs[b];
    if (sigma_mean)
      for (int c = 0; c < 6; ++c) sigma_mean[6 * b + c] = p.mean[c];
    if (info) fill_info(p, p.t_start, wall, info[b]);
  }
  return r->code;
  HZ_GUARD_END
}

int hz_server_release(hz_server s, int64_t id) {
  HZ_GUARD_BEGIN
  if (!s) fail(HZ_EINVAL, "NULL handle");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) fail(HZ_EINVAL, "unknown request id");
  Req* r = it->second.get();
  if (r->state == 1) fail(HZ_EINVAL, "request is running");
  if (r->state == 0) s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
  s->reqs.erase(it);
  return HZ_OK;
  HZ_GUARD_END
}

int hz_server_pending(hz_server s, int32_t* queued, int32_t* running) {
  HZ_GUARD_BEGIN
  if (!s) fail(HZ_EINVAL, "NULL handle");
  if (queued) *queued = (int32_t)s->queue.size();
  if (running) *running = s->running;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_server_set_streams(hz_server s, int32_t n_streams) {
  HZ_GUARD_BEGIN
  if (!s) fail(HZ_EINVAL, "NULL handle");
  if (n_streams < 1 || n_streams > kMaxLanes) fail(HZ_EINVAL, "n_streams out of range [1, 8]");
  s->eng.set_lanes(n_streams);
  return HZ_OK;
  HZ_GUARD_END
}

void hz_server_destroy(hz_server s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  delete s;
}

}  // extern "C"
