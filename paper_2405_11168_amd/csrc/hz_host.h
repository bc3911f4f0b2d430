// Host-side structures of the solver: grid shapes and their tiling, device
// table layouts, per-load problems with their state machines, and the
// executor that advances many problems with grouped kernel launches.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/hz.h"
#include "hz_internal.h"

namespace hz {

// ---- launch wrappers (hz_kernels.hip)
template <typename T>
hipError_t launch_zexp(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*, const void*,
                       hipStream_t);
template <typename T>
hipError_t launch_yline(const Desc*, const int*, int, const YGeo&, const Plan*, const void*, bool, hipStream_t);
template <typename T>
hipError_t launch_xpass(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template <typename T>
hipError_t launch_xfused(const Desc*, const int*, int, int, const XGeo&, const Plan*, const Plan*, const void*,
                         hipStream_t);
template <typename T>
hipError_t launch_zcon(const Desc*, const int*, int, bool, int, const ZGeo&, const Plan*, const void*, const void*,
                       const void*, const void*, hipStream_t);
template <typename T>
hipError_t launch_zstrain(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*,
                          const void*, const void*, hipStream_t);
// stencil-form displacement (FP64, in place): u(q) -> mixed domain (inverse) or back
hipError_t launch_zconv3(void* u, bool inverse, const ZGeo&, const Plan*, const void*, hipStream_t);
template <typename T>
hipError_t launch_xc2r(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template <typename T>
hipError_t launch_xr2c(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template <typename T>
hipError_t launch_stencil(const Desc*, const int*, int, int, int, const SGeo&, hipStream_t);
// continuous-frequency comparison operator (hz_green.hip, FP64): z kernels over `sub`
// columns of a z tile at a time
hipError_t launch_zexp_cont(const Desc*, const int*, int, const ZGeo&, int, float, const Plan*, const void*,
                            hipStream_t);
hipError_t launch_zcon_cont(const Desc*, const int*, int, const ZGeo&, int, float, const Plan*, const void*,
                            hipStream_t);
hipError_t launch_finalize(const Desc*, const int*, int, const FinGeo&, hipStream_t);
hipError_t launch_accumulate(const Desc*, const int*, int, long long, hipStream_t);
hipError_t launch_zero(const Desc*, const int*, int, int, long long, hipStream_t);

// ---- errors: thrown inside the library, turned into codes at the C ABI
struct HzError {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& m);
void hip_check(hipError_t e, const char* what);

// rows per block of the stencil form's 3-field x transforms, at most (compile-time tuning)
#ifndef HZ_TY3_CAP
#define HZ_TY3_CAP 32
#endif

constexpr int kTraceCap = 4097;        // iterates recorded per load (eps_k, <sigma>_k)
constexpr int kMaxIters = 1000000;     // cap on max_iters
constexpr int kMaxLanes = 8;           // streams a server may spread iterate groups over
constexpr int kLdsBytes = 65536 - 512;  // LDS budget of one work-group
// LDS budget of a z-kernel work-group (3 components x TX columns x N3 and the twiddles):
// above 64 KB where that keeps a tile's rows at 4 FP64 columns (64-byte segments) for
// N3 up to 340, instead of 3 (48-byte segments, partly wasted HBM transactions)
constexpr int kLdsBytesZ = 68 * 1024;

float recip(int d);
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }
bool factor_ok(int n);

// ---- grid shape: transform plans and tile sizes of every pass, both precisions
struct Shape {
  Geo geo{};
  Plan plans[8]{};  // N1, N2, N3, N1/2, fused x pass: inverse and forward factorisations of N1/2,
                    // stencil form's C2R / R2C x transforms: inverse and forward factorisations
  bool xfused = false;  // the x pass runs in its fused form (needs >= 2 radix passes of N1/2)
  int TXz[2]{}, TXy[2]{}, TYx[2]{}, H1p[2]{};  // [0] FP32 kernels, [1] FP64 kernels
  int PYy[2]{};                                // LDS line pitch of the y kernel
  YGeo ygeo(int d, long long nlines, long long off, int from_state = 0) const {
    return YGeo{geo.N2, TXy[d], nlines, off, from_state, PYy[d], PYy[d] == lds_pitch(geo.N2) ? 4 : 31};
  }
  int nbx[2]{}, nbq[2]{};                      // partial-sum blocks of the x and z passes
  int subc = 0;        // continuous operator: columns per LDS round of an FP64 z tile (0: N3 too large)
  float rsubc6 = 0.f;  // 1 / (6 subc)
  // stencil form (every accepted grid, see make_split_plans)
  bool stencil = false;
  int TY3[2]{};  // rows per block of the 3-field x transforms
  SGeo sg{};
  int nbs = 0;   // stencil blocks (partial sums of <sigma>)
  void init(int n1, int n2, int n3);            // throws HzError for unsupported sizes
  int nbx_max() const {
    int m = nbx[0] > nbx[1] ? nbx[0] : nbx[1];
    return m > nbs ? m : nbs;
  }
  int nbq_max() const { return nbq[0] > nbq[1] ? nbq[0] : nbq[1]; }
  bool same(const Shape& o) const { return geo.N1 == o.geo.N1 && geo.N2 == o.geo.N2 && geo.N3 == o.geo.N3; }
};

// Device copies of a shape's twiddle tables (exp(-2 pi i j / L) per axis) and plans.
struct ShapeTables {
  const char* tw64[3];
  const char* tw32[3];
  const Plan* plans;
};
size_t shape_table_bytes(const Shape& s);
ShapeTables upload_shape_tables(const Shape& s, char* dev, hipStream_t st);

// ---- material: host copy and its device tables
struct Material {
  int n_phases = 0;
  std::vector<double> C;       // [n_phases][36] engineering Voigt
  std::vector<uint16_t> phase; // [N3][N2][N1]
  int iso = 0;                 // every phase isotropic: tables hold (lambda, mu)
  std::vector<double> c64;     // [n_phases][24]
  std::vector<float> c32;
  std::vector<double> frac;    // volume fraction of each phase
  // eigenstrains (empty: none)
  std::vector<double> eig;     // [n_phases][6] eps0_p, tensor comps
  std::vector<double> tau64;   // [n_phases][8] eigenstress lambda_p:eps0_p, tensor comps (2 pad)
  std::vector<float> tau32;
  double tau_mean[6]{};        // <lambda:eps0>
};
std::shared_ptr<Material> make_material(const Geo& geo, int n_phases, const double* C, const uint16_t* phase);
// a copy of m with per-phase eigenstrains eps0[n_phases][6] (tensor comps); null clears them
std::shared_ptr<Material> with_eigenstrain(const Material& m, const double* eps0);
struct MaterialTables {
  const double* C64;
  const float* C32;
  const uint16_t* phase;
  const double* tau64;  // null without eigenstrains
  const float* tau32;
};
size_t material_table_bytes(int n_phases, long long N);
size_t material_table_bytes(const Material& m);
MaterialTables upload_material_tables(const Material& m, char* dev, hipStream_t st);

// ---- reference medium
struct Reference {
  double C0t[81];  // full tensor
  double S0[36];   // lambda0^-1 acting on tensor comps (11,22,33,23,13,12), row-major
  int iso = 0;
  double lam0 = 0, mu0 = 0;
};
bool isotropic(const double* C, double& lam, double& mu);
void voigt_to_tensor(const double* C, double* T);
void sym_eig6(const double* A, double* ev);
void mandel(const double* C, double* M);
void auto_reference(int np, const double* C, double* C0);
// validated reference medium from the options (explicit lambda0 or the automatic rule)
Reference make_reference(const hz_opts& o, const Material& m);

// ---- per-load device buffers
struct ProbBuffers {
  void* spec;
  void* u0;
  void* u1;
  void* u64;
  void* r32;
  double* part_sig;
  double* part_res;
  double* trace;  // may be null
};
size_t prob_bytes(const Shape& s, int prec, bool trace);
ProbBuffers carve_prob(const Shape& s, int prec, bool trace, char* dev);

// ---- per-kernel timing with HIP events
enum Kind {
  K_ZEXP, K_YINV, K_XPASS, K_YFWD, K_ZCON, K_FINAL, K_ACCUM, K_ZERO,
  K_ZCONV3, K_YINV3, K_XC2R, K_STEN, K_XR2C, K_YFWD3, K_ZCON3, K_ZSTRAIN, K_COUNT
};
extern const char* const kKindNames[K_COUNT];

struct Prof {
  bool on = false;
  int only = -1;  // >= 0: record only launches with this key (kind * 2 + FP64)
  bool records(int key) const { return on && (only < 0 || only == key); }
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  double ms[K_COUNT][2]{};
  long long n[K_COUNT][2]{};
  void reset();
  void drain();  // after the stream has been synchronised
  ~Prof();
};

// ---- one load case of one grid: a state machine advanced by the executor
// PS_FB64: FP64 iterations from the anchor U after the refinement stopped gaining
enum PState { PS_NEW, PS_IT64, PS_R0, PS_SWEEP, PS_CORR, PS_FB64, PS_DONE };

struct Prob {
  // set by the owner before Engine::add
  int slot = -1;  // row of the executor's descriptor and status tables
  const Shape* shape = nullptr;
  ShapeTables tab{};
  int prec = HZ_FP64;
  int form = HZ_SCHEME_SPECTRAL;  // realisation of the iteration (same iterates either way)
  int green = HZ_GREEN_TETRA;     // gradient discretisation (the comparison operators: spectral form)
  int loading = HZ_LOAD_STRAIN;
  double E[6]{};      // applied mean strain, or applied stress under HZ_LOAD_STRESS
  double Eb0[6]{};    // mean strain of iterate 0: E, or lambda0^-1:sigma^a
  double Ebar[6]{};   // mean strain of the reported iterate
  const double* u_init = nullptr;  // host: displacement of iterate 0 (3 S complex FP64), or null
  double tol = 1e-8;
  int max_iters = 2000, fixed_iters = -1, inner_max = 400;
  double rho = 1e-3;
  Desc base{};  // buffers, material, reference medium
  // state
  PState st = PS_NEW;
  bool enter = false;  // the state was just entered: upload descriptor and status, clear buffers
  bool accum = false;  // U += delta pending
  int k0 = 0;          // iterates measured when the current tick started
  bool started = false;
  // results
  int code = HZ_OK, iters = 0, rounds = 0, inner_total = 0, slow = 0, parity = 0;
  bool fb = false;  // the refinement fell back to FP64 iterations (reported as the path used)
  double err = 0, prev_err = 1e300, mean[6]{};
  double sweep_norm = 0;                      // ||<sigma>|| of the last FP64 sweep
  double t_start = 0, t_done = 0, t_1e6 = -1;  // device ms since the executor's clock start
  std::vector<double> times;                  // FP64: device ms at which iterate t was measured
  std::vector<double> trace;                  // FP64 with a trace buffer: [iters+1][7] at the end
  void* owner = nullptr;                      // request this load belongs to (server)
};

// Advances problems with one grouped launch per pass for every (shape,
// kernel precision) group, check_every iterations per tick, one status read
// per tick.  Problems of different grids, materials, loads and precisions mix
// freely; each keeps its own descriptor, status block and buffers, so its
// arithmetic does not depend on what else runs.
struct Engine {
  hipStream_t stream = nullptr;
  int cap = 0;
  int active_cap = 0;
  Desc* d_desc = nullptr;
  double* d_status = nullptr;
  int* d_active = nullptr;
  Desc* h_desc = nullptr;    // host mirrors: pinned, or pageable for an engine that must
  double* h_status = nullptr;  // not call an allocator of the HIP runtime
  int* h_active = nullptr;
  bool pinned = true;
  int check_every = 8;
  Prof* prof = nullptr;  // owned by the grid or server; never null once bound
  std::vector<Prob*> live;
  hipEvent_t epoch = nullptr;
  std::vector<hipEvent_t> evs;
  std::vector<double> ev_ms;
  // lanes > 1: the iterate groups of a tick are spread over `stream` and lanes - 1
  // more streams (non-blocking, default priority), forked from and joined into
  // `stream` with events
  int lanes = 1;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> fork_join;

  static size_t table_bytes(int cap);
  void init(int cap, bool pinned_mirrors = true);
  void bind(char* dev, hipStream_t s);
  void set_lanes(int n);
  void start_clock();
  void add(Prob* p);
  // one tick; returns the problems that finished in it
  std::vector<Prob*> tick();
  ~Engine();

 private:
  hipEvent_t event(size_t i);
  void enter_state(Prob* p);
  // stencil-form iterate u (FP64) in place: u(q) -> mixed domain (inverse) or back
  void convert_stencil_state(void* u, const Prob& p, bool inverse);
  void advance(Prob* p, const double* s, const double* t_iter);
};

// Output fields of one finished problem (eq. final_fields): P1..P3 once with
// the field writer of the x pass enabled, into eps_out/sig_out (device, [6][N]).
void output_fields(Engine& e, Prob& p, double* eps_dev, double* sig_dev);

}  // namespace hz
