// Host driver and C ABI of the tetrahedral-stencil FFT homogenization solver.
//
// The driver owns no device memory: a caller-bound workspace is carved into
// tables, per-load spectra and small status blocks.  Each iteration is a fixed
// sequence of kernel launches on the caller's stream; the stop rule runs on
// the device (k_finalize), so the host only polls status every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/hz.h"
#include "hz_internal.h"

namespace hz {

template <typename T>
hipError_t launch_zexp(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*, const void*,
                       hipStream_t);
template <typename T>
hipError_t launch_yline(const Desc*, const int*, int, const YGeo&, const Plan*, const void*, bool, hipStream_t);
template <typename T>
hipError_t launch_xpass(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template <typename T>
hipError_t launch_zcon(int, const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*,
                       const void*, const void*, hipStream_t);
hipError_t launch_finalize(const Desc*, const int*, int, const FinGeo&, hipStream_t);
hipError_t launch_accumulate(const Desc*, const int*, int, long long, hipStream_t);
hipError_t launch_zero(const Desc*, const int*, int, int, long long, hipStream_t);

}  // namespace hz

using namespace hz;

namespace {

thread_local std::string g_err;

struct HzError {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& m) { throw HzError{code, m}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(HZ_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int kTraceCap = 4097;
constexpr int kLdsBytes = 65536 - 512;

bool factor_ok(int n) {
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}

// r = (1 + 2^-20) / d rounded up to float: floor(a / d) = int(float(a) * r) for a < 2^19
float recip(int d) {
  const double x = (1.0 + std::ldexp(1.0, -20)) / (double)d;
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, 2.0f * f + 1.0f);
  return f;
}

Plan make_plan(int L) {
  Plan p{};
  p.L = L;
  p.np = 0;
  int n = L;
  auto push = [&](int r) {
    if (p.np >= kMaxPasses) fail(HZ_EINVAL, "too many radix passes");
    p.radix[p.np++] = r;
    n /= r;
  };
  while (n % 16 == 0) push(16);
  while (n % 8 == 0) push(8);
  while (n % 4 == 0) push(4);
  while (n % 2 == 0) push(2);
  while (n % 7 == 0) push(7);
  while (n % 5 == 0) push(5);
  while (n % 3 == 0) push(3);
  if (n != 1) fail(HZ_EINVAL, "transform length " + std::to_string(L) + " not supported");
  int ns = 1;
  for (int s = 0; s < p.np; ++s) {
    p.rLR[s] = recip(L / p.radix[s]);
    p.rNs[s] = recip(ns);
    ns *= p.radix[s];
  }
  return p;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// largest divisor of n that is <= cap
int divisor_le(int n, int cap) {
  for (int t = std::min(n, cap); t >= 1; --t)
    if (n % t == 0) return t;
  return 1;
}

const char* kKindNames[] = {"zexpand", "yinv", "xpass", "yfwd", "zcontract", "finalize", "accumulate", "zero"};
enum Kind { K_ZEXP, K_YINV, K_XPASS, K_YFWD, K_ZCON, K_FINAL, K_ACCUM, K_ZERO, K_COUNT };

}  // namespace

struct hz_grid_s {
  Geo geo{};
  int n_phases = 0;
  std::vector<double> C;
  std::vector<uint16_t> phase;
  bool material = false;

  // tiling
  Plan plan1{}, plan2{}, plan3{}, planM{};
  int TXz[2]{}, TXy[2]{}, TYx[2]{}, H1p[2]{};  // [0]=FP32, [1]=FP64
  long long nbx[2]{}, nbq[2]{};

  // bound workspace
  char* ws = nullptr;
  int64_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int prec = -1;
  int cap = 0;
  int iso = 0;
  int c0_iso = 0;
  double lam0 = 0, mu0 = 0;
  struct Off {
    size_t tw64[3], tw32[3], plans, C64, C32, phase, descs, active, status, status2, part_sig, part_res, trace, fields;
    std::vector<size_t> spec, u0, u1, u64, r32;
    size_t total;
  } off;
  double* h_status = nullptr;  // pinned
  std::vector<Desc> hdesc, hdesc2;
  int last_loads = 0;
  int last_prec = -1;

  // profiling
  bool prof = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double prof_ms[K_COUNT][2]{};
  long long prof_n[K_COUNT][2]{};
  std::vector<hipEvent_t> iter_ev;  // one per iteration for time-to-target
};

namespace {

template <typename T>
T* P(hz_grid g, size_t off) { return reinterpret_cast<T*>(g->ws + off); }

void compute_tiling(hz_grid g) {
  const Geo& G = g->geo;
  g->plan1 = make_plan(G.N1);
  g->plan2 = make_plan(G.N2);
  g->plan3 = make_plan(G.N3);
  g->planM = make_plan(G.N1 / 2);
  for (int d = 0; d < 2; ++d) {
    const int csz = d ? 16 : 8;
    const int tile = (d ? 16 : 32) * kThreads;  // elements per transform call (emax)
    const int rowcap = 256 / csz;               // TX giving 256-byte rows
    // z kernels: 3 comps x TX columns x N3 in LDS (+ N3 twiddles), TX | N2
    int tx = std::min(rowcap, G.N2);
    while (tx > 1 && (3 * tx * G.N3 > tile || (3 * tx * G.N3 + G.N3) * csz > kLdsBytes || G.N2 % tx)) --tx;
    if (3 * tx * G.N3 > tile || (3 * tx * G.N3 + G.N3) * csz > kLdsBytes) fail(HZ_EINVAL, "N3 too large");
    g->TXz[d] = tx;
    // y kernel: TX rows of N2 (+ N2 twiddles)
    int ty = std::min(64, tile / G.N2);
    while (ty > 1 && (ty * G.N2 + G.N2) * csz > kLdsBytes) --ty;
    if (ty < 1 || G.N2 > tile || (ty * G.N2 + G.N2) * csz > kLdsBytes) fail(HZ_EINVAL, "N2 too large");
    g->TXy[d] = ty;
    // x kernel: 6 comps x TY rows x (N1/2+1) in LDS (+ N1 twiddles), TY | N2
    const int hp = (G.N1 / 2) | 1;  // lines hold M = N1/2 values; odd pitch spreads rows over banks
    int tyx = std::min(16, G.N2);
    while (tyx > 1 && ((6 * tyx * hp + G.N1) * csz > kLdsBytes || 6 * tyx * (G.N1 / 2) > tile || G.N2 % tyx)) --tyx;
    if ((6 * tyx * hp + G.N1) * csz > kLdsBytes || 6 * tyx * (G.N1 / 2) > tile) fail(HZ_EINVAL, "N1 too large");
    g->TYx[d] = tyx;
    g->H1p[d] = hp;
    g->nbx[d] = 2LL * G.N3 * (G.N2 / tyx);
    g->nbq[d] = (long long)G.H1 * (G.N2 / tx);
  }
}

void layout(hz_grid g, int prec, int nl, hz_grid_s::Off& o) {
  const Geo& G = g->geo;
  size_t p = 0;
  auto take = [&](size_t bytes) { size_t r = p; p = align_up(p + bytes); return r; };
  const int Ns[3] = {G.N1, G.N2, G.N3};
  for (int a = 0; a < 3; ++a) o.tw64[a] = take((size_t)Ns[a] * 16);
  for (int a = 0; a < 3; ++a) o.tw32[a] = take((size_t)Ns[a] * 8);
  o.plans = take(4 * sizeof(Plan));  // N1, N2, N3, N1/2
  const int np = std::max(1, g->n_phases);
  o.C64 = take((size_t)np * 24 * 8);
  o.C32 = take((size_t)np * 24 * 4);
  o.phase = take((size_t)G.N * 2);
  o.descs = take((size_t)nl * sizeof(Desc) * 2);
  o.active = take((size_t)nl * 4);
  o.status = take((size_t)nl * kStatusLen * 8);
  o.status2 = take((size_t)nl * kStatusLen * 8);
  const long long nbx = std::max(g->nbx[0], g->nbx[1]);
  o.part_sig = take((size_t)nl * nbx * 6 * 8);
  o.part_res = take((size_t)nl * std::max(g->nbq[0], g->nbq[1]) * 8);
  o.trace = take((size_t)nl * kTraceCap * 7 * 8);
  o.fields = take((size_t)12 * G.N * 8);
  o.spec.assign(nl, 0);
  o.u0.assign(nl, 0);
  o.u1.assign(nl, 0);
  o.u64.assign(nl, 0);
  o.r32.assign(nl, 0);
  for (int b = 0; b < nl; ++b) {
    o.spec[b] = take((size_t)12 * G.S * 16);
    if (prec == HZ_FP64) {
      o.u0[b] = take((size_t)3 * G.S * 16);
      o.u1[b] = take((size_t)3 * G.S * 16);
    } else {
      o.u0[b] = take((size_t)3 * G.S * 8);
      o.u1[b] = take((size_t)3 * G.S * 8);
      o.u64[b] = take((size_t)3 * G.S * 16);
      o.r32[b] = take((size_t)3 * G.S * 8);
    }
  }
  o.total = p;
}

bool isotropic(const double* C, double& lam, double& mu);

void upload_tables(hz_grid g) {
  const Geo& G = g->geo;
  const int Ns[3] = {G.N1, G.N2, G.N3};
  for (int a = 0; a < 3; ++a) {
    const int L = Ns[a];
    std::vector<double> t64(2 * L);
    std::vector<float> t32(2 * L);
    for (int j = 0; j < L; ++j) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)L;
      t64[2 * j] = (double)cosl(ang);
      t64[2 * j + 1] = (double)sinl(ang);
      t32[2 * j] = (float)cosl(ang);
      t32[2 * j + 1] = (float)sinl(ang);
    }
    hip_check(hipMemcpy(g->ws + g->off.tw64[a], t64.data(), t64.size() * 8, hipMemcpyHostToDevice), "upload twiddles");
    hip_check(hipMemcpy(g->ws + g->off.tw32[a], t32.data(), t32.size() * 4, hipMemcpyHostToDevice), "upload twiddles");
  }
  const Plan plans[4] = {g->plan1, g->plan2, g->plan3, g->planM};
  hip_check(hipMemcpy(g->ws + g->off.plans, plans, sizeof(plans), hipMemcpyHostToDevice), "upload plans");
  // per-phase tables: (lambda, mu) when every phase is isotropic, else the Voigt upper triangle
  const int np = g->n_phases;
  std::vector<double> c64((size_t)np * 24, 0.0);
  g->iso = 1;
  for (int p = 0; p < np; ++p) {
    double lam, mu;
    if (!isotropic(g->C.data() + 36 * p, lam, mu)) g->iso = 0;
  }
  for (int p = 0; p < np; ++p) {
    const double* C = g->C.data() + 36 * p;
    if (g->iso) {
      isotropic(C, c64[2 * p], c64[2 * p + 1]);
    } else {
      int n = 0;
      for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) c64[(size_t)p * 24 + n++] = C[i * 6 + j];
    }
  }
  std::vector<float> c32(c64.size());
  for (size_t i = 0; i < c32.size(); ++i) c32[i] = (float)c64[i];
  hip_check(hipMemcpy(g->ws + g->off.C64, c64.data(), c64.size() * 8, hipMemcpyHostToDevice), "upload C");
  hip_check(hipMemcpy(g->ws + g->off.C32, c32.data(), c32.size() * 4, hipMemcpyHostToDevice), "upload C");
  hip_check(hipMemcpy(g->ws + g->off.phase, g->phase.data(), g->phase.size() * 2, hipMemcpyHostToDevice),
            "upload phase map");
}

// isotropic engineering Voigt stiffness: C11=C22=C33 = lam + 2 mu, C12=C13=C23 = lam,
// C44=C55=C66 = mu, every other entry zero (relative tolerance 1e-12)
bool isotropic(const double* C, double& lam, double& mu) {
  lam = C[1];
  mu = C[21];
  double scale = 0;
  for (int i = 0; i < 36; ++i) scale = std::max(scale, std::fabs(C[i]));
  const double tol = 1e-12 * scale;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double e = 0;
      if (i < 3 && j < 3) e = (i == j) ? lam + 2 * mu : lam;
      else if (i == j) e = mu;
      if (std::fabs(C[i * 6 + j] - e) > tol) return false;
    }
  return true;
}

void voigt_to_tensor(const double* C, double* T) {
  static const int pr[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      const int i = pr[I][0], j = pr[I][1], k = pr[J][0], l = pr[J][1];
      const double v = C[I * 6 + J];
      T[((i * 3 + j) * 3 + k) * 3 + l] = v;
      T[((j * 3 + i) * 3 + k) * 3 + l] = v;
      T[((i * 3 + j) * 3 + l) * 3 + k] = v;
      T[((j * 3 + i) * 3 + l) * 3 + k] = v;
    }
}

// symmetric eigenvalues of a 6x6 by Jacobi rotations (host only, tiny)
void sym_eig6(const double* A_in, double* ev) {
  double A[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) A[i][j] = A_in[i * 6 + j];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) off += A[i][j] * A[i][j];
    if (off < 1e-30) break;
    for (int p = 0; p < 6; ++p)
      for (int q = p + 1; q < 6; ++q) {
        if (std::fabs(A[p][q]) < 1e-300) continue;
        const double th = 0.5 * (A[q][q] - A[p][p]) / A[p][q];
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 6; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 6; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
      }
  }
  for (int i = 0; i < 6; ++i) ev[i] = A[i][i];
}

// Mandel form of an engineering-shear Voigt stiffness
void mandel(const double* C, double* M) {
  const double s[6] = {1, 1, 1, std::sqrt(2.0), std::sqrt(2.0), std::sqrt(2.0)};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) M[i * 6 + j] = C[i * 6 + j] * s[i] * s[j];
}

void auto_reference(int np, const double* C, double* C0) {
  double lo = 1e300, hi = -1e300;
  for (int p = 0; p < np; ++p) {
    double M[36], ev[6];
    mandel(C + 36 * p, M);
    sym_eig6(M, ev);
    for (double e : ev) {
      lo = std::min(lo, e);
      hi = std::max(hi, e);
    }
  }
  const double m = 0.5 * (std::max(lo, 0.0) + hi);  // Mandel modulus: 3K0 = 2 mu0 = m (nu0 = 0)
  std::fill(C0, C0 + 36, 0.0);
  for (int i = 0; i < 3; ++i) C0[i * 6 + i] = m;
  for (int i = 3; i < 6; ++i) C0[i * 6 + i] = 0.5 * m;
}

// ---------------------------------------------------------------------------
// launch bookkeeping with optional per-kernel event timing
// ---------------------------------------------------------------------------
struct Launcher {
  hz_grid g;
  int kind = 0, dbl = 0;
  hipEvent_t a = nullptr, b = nullptr;
  hipEvent_t take() {
    if (g->ev_used == g->ev_pool.size()) {
      hipEvent_t e;
      hip_check(hipEventCreate(&e), "hipEventCreate");
      g->ev_pool.push_back(e);
    }
    return g->ev_pool[g->ev_used++];
  }
  void begin(int k, int d) {
    kind = k;
    dbl = d;
    if (g->prof) {
      a = take();
      b = take();
      hip_check(hipEventRecord(a, g->stream), "hipEventRecord");
    }
  }
  void end(hipError_t e, const char* what) {
    hip_check(e, what);
    if (g->prof) {
      hip_check(hipEventRecord(b, g->stream), "hipEventRecord");
      g->pending.push_back({kind * 2 + dbl, {a, b}});
    }
  }
};

void drain_profile(hz_grid g) {
  if (!g->prof) return;
  for (auto& p : g->pending) {
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, p.second.first, p.second.second), "hipEventElapsedTime");
    g->prof_ms[p.first / 2][p.first % 2] += ms;
    g->prof_n[p.first / 2][p.first % 2] += 1;
  }
  g->pending.clear();
  g->ev_used = 0;
}

// after several iterations the event pool would grow without bound; drain periodically
void maybe_drain(hz_grid g) {
  if (g->prof && g->pending.size() > 4096) {
    hip_check(hipStreamSynchronize(g->stream), "sync");
    drain_profile(g);
  }
}

struct Ctx {
  hz_grid g;
  Desc* dd;       // device descriptors
  int* act;       // device active list
  int nact;
};

// P1 (expand + inverse z) and P2 (inverse y) in precision T; src 0 = u[parity], 1 = u64
template <typename T>
void pipeline_front(Ctx& c, int parity, int src) {
  hz_grid g = c.g;
  const Geo& G = g->geo;
  const int d = sizeof(T) == 8;
  const size_t* tw = d ? g->off.tw64 : g->off.tw32;
  Launcher L{g};
  ZGeo zg{G.N1, G.N2, G.N3, G.H1, g->TXz[d], G.N2 / g->TXz[d], recip(g->TXz[d]), recip(3 * g->TXz[d]),
          recip(G.N2 / g->TXz[d]), G.S, parity, src};
  L.begin(K_ZEXP, d);
  L.end(launch_zexp<T>(c.dd, c.act, c.nact, zg, P<Plan>(g, g->off.plans) + 2, g->ws + tw[2], g->ws + g->off.tw64[0],
                       g->ws + g->off.tw64[1], g->stream),
        "z expand");
  YGeo yg{G.N2, g->TXy[d], (long long)12 * G.H1 * G.N3};
  L.begin(K_YINV, d);
  L.end(launch_yline<T>(c.dd, c.act, c.nact, yg, P<Plan>(g, g->off.plans) + 1, g->ws + tw[1], true, g->stream), "y inverse");
}

template <typename T>
void pipeline_x(Ctx& c, int fields) {
  hz_grid g = c.g;
  const Geo& G = g->geo;
  const int d = sizeof(T) == 8;
  const size_t* tw = d ? g->off.tw64 : g->off.tw32;
  Launcher L{g};
  // with fields, T1 writes and T2 then adds its half of the averages: two launches
  for (int h = fields ? 0 : -1; h < (fields ? 2 : 0); ++h) {
    const int M = G.N1 / 2;
    XGeo xg{G.N1, G.N2, G.N3, G.H1, g->H1p[d], g->TYx[d], M, recip(g->TYx[d]), recip(M / 2 + 1), recip(M),
            G.S, 1.0 / (double)G.N, fields, h};
    L.begin(K_XPASS, d);
    L.end(launch_xpass<T>(c.dd, c.act, c.nact, xg, P<Plan>(g, g->off.plans) + 3, g->ws + tw[0], g->stream), "x pass");
  }
}

// P4 (forward y) and P5 (forward z + contraction + update); mode as k_zcon
template <typename T>
void pipeline_back(Ctx& c, int parity, int mode) {
  hz_grid g = c.g;
  const Geo& G = g->geo;
  const int d = sizeof(T) == 8;
  const size_t* tw = d ? g->off.tw64 : g->off.tw32;
  Launcher L{g};
  YGeo yg{G.N2, g->TXy[d], (long long)12 * G.H1 * G.N3};
  L.begin(K_YFWD, d);
  L.end(launch_yline<T>(c.dd, c.act, c.nact, yg, P<Plan>(g, g->off.plans) + 1, g->ws + tw[1], false, g->stream), "y forward");
  ZGeo zg{G.N1, G.N2, G.N3, G.H1, g->TXz[d], G.N2 / g->TXz[d], recip(g->TXz[d]), recip(3 * g->TXz[d]),
          recip(G.N2 / g->TXz[d]), G.S, parity, 0};
  L.begin(K_ZCON, d);
  L.end(launch_zcon<T>(mode, c.dd, c.act, c.nact, zg, P<Plan>(g, g->off.plans) + 2, g->ws + tw[2], g->ws + g->off.tw64[0],
                       g->ws + g->off.tw64[1], g->ws + g->off.tw64[2], g->stream),
        "z contract");
}

void finalize(Ctx& c, int parity, int mode, int dbl, int inner_max = 0) {
  hz_grid g = c.g;
  FinGeo fg{(int)g->nbx[dbl], (int)g->nbq[dbl], 1.0 / (double)g->geo.N, parity, mode, inner_max};
  Launcher L{g};
  L.begin(K_FINAL, dbl);
  L.end(launch_finalize(c.dd, c.act, c.nact, fg, g->stream), "finalize");
}

void check_material(hz_grid g) {
  if (!g->material) fail(HZ_ENOMATERIAL, "material not set");
  if (!g->ws) fail(HZ_EWORKSPACE, "workspace not bound");
}

Desc base_desc(hz_grid g, int b, const double* E, const double* C0t, double tol, int max_iters, int fixed,
               bool inner) {
  Desc d{};
  const auto& o = g->off;
  d.spec = g->ws + o.spec[b];
  d.u[0] = g->ws + o.u0[b];
  d.u[1] = g->ws + o.u1[b];
  d.u64 = o.u64[b] ? g->ws + o.u64[b] : nullptr;
  d.r32 = o.r32[b] ? g->ws + o.r32[b] : nullptr;
  d.phase = P<uint16_t>(g, o.phase);
  d.C64 = P<double>(g, o.C64);
  d.C32 = P<float>(g, o.C32);
  const int dbl = (g->prec == HZ_FP64 || !inner) ? 1 : 0;
  d.part_sig = P<double>(g, o.part_sig) + (size_t)b * std::max(g->nbx[0], g->nbx[1]) * 6;
  d.part_res = P<double>(g, o.part_res) + (size_t)b * std::max(g->nbq[0], g->nbq[1]);
  d.status = P<double>(g, inner ? o.status2 : o.status) + (size_t)b * kStatusLen;
  d.eps_out = P<double>(g, o.fields);
  d.sig_out = P<double>(g, o.fields) + 6 * g->geo.N;
  d.trace = inner ? nullptr : P<double>(g, o.trace) + (size_t)b * kTraceCap * 7;
  d.trace_len = inner ? 0 : kTraceCap;
  for (int c = 0; c < 6; ++c) d.Ebar[c] = inner ? 0.0 : E[c];
  std::memcpy(d.C0, C0t, sizeof(d.C0));
  d.iso = g->iso;
  d.c0_iso = g->c0_iso;
  d.lam0 = g->lam0;
  d.mu0 = g->mu0;
  d.tol = tol;
  d.max_iters = max_iters;
  d.fixed_iters = fixed;
  (void)dbl;
  return d;
}

void read_status(hz_grid g, size_t off, int n) {
  hip_check(hipMemcpyAsync(g->h_status, g->ws + off, (size_t)n * kStatusLen * 8, hipMemcpyDeviceToHost, g->stream),
            "status D2H");
  hip_check(hipStreamSynchronize(g->stream), "sync");
}

void zero_status(hz_grid g, size_t off, int n) {
  std::vector<double> z((size_t)n * kStatusLen, 0.0);
  hip_check(hipMemcpyAsync(g->ws + off, z.data(), z.size() * 8, hipMemcpyHostToDevice, g->stream), "status H2D");
  hip_check(hipStreamSynchronize(g->stream), "sync");
}

hipEvent_t iter_event(hz_grid g, size_t k) {
  while (g->iter_ev.size() <= k) {
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    g->iter_ev.push_back(e);
  }
  return g->iter_ev[k];
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  hip_check(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
  return ms;
}

void output_fields(hz_grid g, Ctx& c, int b, double* eps_out, double* sig_out, int src, int parity) {
  // one load at a time through P1..P3 with the field writer enabled
  std::vector<int> one{b};
  hip_check(hipMemcpyAsync(c.act, one.data(), 4, hipMemcpyHostToDevice, g->stream), "active H2D");
  Ctx c1{g, c.dd, c.act, 1};
  if (src == 1) {
    pipeline_front<double>(c1, 0, 1);
  } else {
    pipeline_front<double>(c1, parity, 0);
  }
  pipeline_x<double>(c1, 1);
  const size_t n6 = (size_t)6 * g->geo.N;
  hip_check(hipStreamSynchronize(g->stream), "sync");
  if (eps_out)
    hip_check(hipMemcpy(eps_out + (size_t)b * n6, g->ws + g->off.fields, n6 * 8, hipMemcpyDeviceToHost), "eps D2H");
  if (sig_out)
    hip_check(hipMemcpy(sig_out + (size_t)b * n6, g->ws + g->off.fields + n6 * 8, n6 * 8, hipMemcpyDeviceToHost),
              "sigma D2H");
}

// ---------------------------------------------------------------------------
// FP64 basic scheme on all loads at once
// ---------------------------------------------------------------------------
int solve_fp64(hz_grid g, int nl, const double* E, const hz_opts& o, const double* C0t, double* sigma_mean,
               double* eps_out, double* sig_out, hz_info* info) {
  const Geo& G = g->geo;
  Desc* dd = P<Desc>(g, g->off.descs);
  int* act = P<int>(g, g->off.active);
  g->hdesc.resize(nl);
  for (int b = 0; b < nl; ++b) g->hdesc[b] = base_desc(g, b, E + 6 * b, C0t, o.tol, o.max_iters, o.fixed_iters, false);
  hip_check(hipMemcpyAsync(dd, g->hdesc.data(), nl * sizeof(Desc), hipMemcpyHostToDevice, g->stream), "desc H2D");
  std::vector<int> ha(nl);
  for (int b = 0; b < nl; ++b) ha[b] = b;
  hip_check(hipMemcpyAsync(act, ha.data(), nl * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
  zero_status(g, g->off.status, nl);
  Ctx c{g, dd, act, nl};
  {
    Launcher L{g};
    L.begin(K_ZERO, 1);
    L.end(launch_zero(dd, act, nl, 0, 3 * G.S, g->stream), "zero");
  }
  hipEvent_t ev0 = iter_event(g, 0);
  hip_check(hipEventRecord(ev0, g->stream), "event");
  const int check = std::max(1, o.check_every);
  const int cap = o.fixed_iters >= 0 ? o.fixed_iters : o.max_iters;
  std::vector<int> done(nl, 0);
  int it = 0;
  for (;;) {
    const int parity = it & 1;
    pipeline_front<double>(c, parity, 0);
    pipeline_x<double>(c, 0);
    pipeline_back<double>(c, parity, 0);
    finalize(c, parity, 0, 1);
    hip_check(hipEventRecord(iter_event(g, it + 1), g->stream), "event");
    ++it;
    maybe_drain(g);
    if (it % check == 0 || it > cap) {
      read_status(g, g->off.status, nl);
      std::vector<int> na;
      for (int b = 0; b < nl; ++b)
        if (g->h_status[b * kStatusLen + ST_DONE] == 0.0) na.push_back(b);
      if (na.empty()) break;
      if (it > cap + 1) fail(HZ_EINVAL, "stop rule did not fire");
      if ((int)na.size() != c.nact) {
        hip_check(hipMemcpyAsync(act, na.data(), na.size() * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
        c.nact = (int)na.size();
      }
    }
  }
  hip_check(hipStreamSynchronize(g->stream), "sync");
  drain_profile(g);
  // results
  std::vector<double> trace;
  int worst = HZ_OK;
  for (int b = 0; b < nl; ++b) {
    const double* s = g->h_status + b * kStatusLen;
    const int k = (int)s[ST_ITERS];
    const int st = (int)s[ST_DONE];
    const int code = st == 1 ? HZ_OK : (st == 2 ? HZ_NOT_CONVERGED : HZ_EDIVERGED);
    if (code < 0 || (worst >= 0 && code > worst)) worst = code < 0 ? code : std::max(worst, code);
    if (sigma_mean)
      for (int cc = 0; cc < 6; ++cc) sigma_mean[6 * b + cc] = s[ST_MEAN + cc];
    const int ntr = std::min(k + 1, kTraceCap);
    trace.resize((size_t)ntr * 7);
    hip_check(hipMemcpy(trace.data(), P<double>(g, g->off.trace) + (size_t)b * kTraceCap * 7, trace.size() * 8,
                        hipMemcpyDeviceToHost),
              "trace D2H");
    if (o.trace_residual || o.trace_mean) {
      const int stride = (o.fixed_iters >= 0 ? o.fixed_iters : o.max_iters) + 1;
      for (int t = 0; t < ntr && t < stride; ++t) {
        if (o.trace_residual) o.trace_residual[(size_t)b * stride + t] = trace[t * 7];
        if (o.trace_mean)
          for (int cc = 0; cc < 6; ++cc) o.trace_mean[((size_t)b * stride + t) * 6 + cc] = trace[t * 7 + 1 + cc];
      }
    }
    if (info) {
      hz_info& in = info[b];
      in.status = code;
      in.iters = k;
      in.outer_rounds = 0;
      in.precision_used = HZ_FP64;
      in.residual = s[ST_ERR];
      in.seconds = 1e-3 * elapsed(ev0, iter_event(g, k + 1));
      in.seconds_to_1e6 = -1;
      for (int t = 0; t < ntr; ++t)
        if (trace[t * 7] < 1e-6) {
          in.seconds_to_1e6 = 1e-3 * elapsed(ev0, iter_event(g, t + 1));
          break;
        }
    }
  }
  if (eps_out || sig_out) {
    // re-enable the problems for the output pass (fresh status blocks)
    for (int b = 0; b < nl; ++b) g->hdesc[b].status = P<double>(g, g->off.status2) + (size_t)b * kStatusLen;
    hip_check(hipMemcpyAsync(dd, g->hdesc.data(), nl * sizeof(Desc), hipMemcpyHostToDevice, g->stream), "desc H2D");
    zero_status(g, g->off.status2, nl);
    for (int b = 0; b < nl; ++b) {
      const int parity = (int)g->h_status[b * kStatusLen + ST_PARITY];
      output_fields(g, c, b, eps_out, sig_out, 0, parity);
    }
  }
  return worst;
}

// ---------------------------------------------------------------------------
// FP32 fields + FP64 anchor (iterative refinement).  Outer round:
//   FP64 sweep of the full pipeline on U -> r64, eps64 (stop if < tol)
//   FP32 basic-scheme iterations on the correction delta with Ebar = 0 and r64
//   added to the equilibrium residual, from delta = 0, until the inner residual
//   falls to rho * eps64 or stalls;  then U += delta.
// In exact arithmetic the inner iterates are those of the plain scheme on U + delta.
// ---------------------------------------------------------------------------
int solve_refine(hz_grid g, int nl, const double* E, const hz_opts& o, const double* C0t, double* sigma_mean,
                 double* eps_out, double* sig_out, hz_info* info) {
  const Geo& G = g->geo;
  Desc* dd = P<Desc>(g, g->off.descs);        // sweep descriptors (FP64 spec, anchor U)
  Desc* dd2 = dd + nl;                          // inner descriptors (FP32 spec, delta)
  int* act = P<int>(g, g->off.active);
  g->hdesc.resize(nl);
  g->hdesc2.resize(nl);
  for (int b = 0; b < nl; ++b) {
    g->hdesc[b] = base_desc(g, b, E + 6 * b, C0t, o.tol, 1 << 30, -1, false);
    g->hdesc2[b] = base_desc(g, b, E + 6 * b, C0t, o.tol, 1 << 30, -1, true);
  }
  hip_check(hipMemcpyAsync(dd, g->hdesc.data(), nl * sizeof(Desc), hipMemcpyHostToDevice, g->stream), "desc H2D");
  hip_check(hipMemcpyAsync(dd2, g->hdesc2.data(), nl * sizeof(Desc), hipMemcpyHostToDevice, g->stream), "desc H2D");
  std::vector<int> active(nl);
  for (int b = 0; b < nl; ++b) active[b] = b;
  hip_check(hipMemcpyAsync(act, active.data(), nl * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
  zero_status(g, g->off.status, nl);
  {
    Launcher L{g};
    L.begin(K_ZERO, 1);
    L.end(launch_zero(dd, act, nl, 2, 3 * G.S, g->stream), "zero");
  }
  hipEvent_t ev0 = iter_event(g, 0);
  hip_check(hipEventRecord(ev0, g->stream), "event");
  std::vector<int> rounds(nl, 0), inner_total(nl, 0), code(nl, HZ_OK), finished(nl, 0);
  std::vector<double> err(nl, 0), prev_err(nl, 1e300), mean((size_t)nl * 6, 0), t_1e6(nl, -1), t_done(nl, 0);
  std::vector<int> slow(nl, 0);
  size_t evk = 1;
  const int check = std::max(1, o.check_every);
  const int inner_max = o.inner_max > 0 ? o.inner_max : 400;
  const double rho = o.inner_rho > 0 ? o.inner_rho : 1e-3;
  // ---- round 0: the plain basic scheme in FP32 on the full problem (Ebar applied,
  // FP64 reductions) from u = 0 down to a moderate residual; U = its iterate
  {
    std::vector<Desc> d0 = g->hdesc2;
    for (int b = 0; b < nl; ++b)
      for (int cc = 0; cc < 6; ++cc) d0[b].Ebar[cc] = E[6 * b + cc];
    hip_check(hipMemcpyAsync(dd2, d0.data(), nl * sizeof(Desc), hipMemcpyHostToDevice, g->stream), "desc H2D");
    std::vector<double> init((size_t)nl * kStatusLen, 0.0);
    for (int b = 0; b < nl; ++b) {
      // stop well above the FP32 rounding floor of the full problem (~1e-6 relative);
      // correction rounds take the residual the rest of the way
      init[(size_t)b * kStatusLen + ST_REF] = std::max(0.5 * o.tol, 3e-5);
      init[(size_t)b * kStatusLen + ST_BEST] = 1e300;
    }
    hip_check(hipMemcpyAsync(g->ws + g->off.status2, init.data(), init.size() * 8, hipMemcpyHostToDevice, g->stream),
              "status H2D");
    Ctx ci{g, dd2, act, nl};
    {
      Launcher L{g};
      L.begin(K_ZERO, 0);
      L.end(launch_zero(dd2, act, nl, 0, 3 * G.S / 2, g->stream), "zero");
    }
    std::vector<int> r0 = active;
    int it = 0;
    for (;;) {
      const int parity = it & 1;
      pipeline_front<float>(ci, parity, 0);
      pipeline_x<float>(ci, 0);
      pipeline_back<float>(ci, parity, 0);
      finalize(ci, parity, 3, 0, inner_max);
      ++it;
      maybe_drain(g);
      if (it % check == 0 || it >= inner_max) {
        read_status(g, g->off.status2, nl);
        std::vector<int> na;
        for (int b : r0)
          if (g->h_status[b * kStatusLen + ST_DONE] == 0.0) na.push_back(b);
        if (na.empty()) break;
        if (it > inner_max + 1) fail(HZ_EINVAL, "round-0 stop rule did not fire");
        if (na.size() != r0.size()) {
          r0 = na;
          hip_check(hipMemcpyAsync(act, na.data(), na.size() * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
          ci.nact = (int)na.size();
        }
      }
    }
    std::vector<int> good;
    for (int b = 0; b < nl; ++b) {
      inner_total[b] += (int)g->h_status[b * kStatusLen + ST_ITERS];
      if (g->h_status[b * kStatusLen + ST_DONE] != 3.0) good.push_back(b);  // a diverged round 0 keeps U = 0
    }
    if (!good.empty()) {
      hip_check(hipMemcpyAsync(act, good.data(), good.size() * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
      Launcher L{g};
      L.begin(K_ACCUM, 1);
      L.end(launch_accumulate(dd2, act, (int)good.size(), 3 * G.S, g->stream), "accumulate");
    }
    hip_check(hipMemcpyAsync(dd2, g->hdesc2.data(), nl * sizeof(Desc), hipMemcpyHostToDevice, g->stream), "desc H2D");
  }
  for (int round = 0;; ++round) {
    // ---- FP64 sweep on the active loads
    Ctx c{g, dd, act, (int)active.size()};
    hip_check(hipMemcpyAsync(act, active.data(), active.size() * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
    pipeline_front<double>(c, 0, 1);
    pipeline_x<double>(c, 0);
    pipeline_back<double>(c, 0, 1);
    finalize(c, 0, 1, 1);
    hipEvent_t evs = iter_event(g, evk++);
    hip_check(hipEventRecord(evs, g->stream), "event");
    read_status(g, g->off.status, nl);
    const float t_ms = elapsed(ev0, evs);
    std::vector<int> next;
    std::vector<double> inner_init((size_t)nl * kStatusLen, 0.0);
    for (int b : active) {
      const double* s = g->h_status + b * kStatusLen;
      err[b] = s[ST_ERR];
      for (int cc = 0; cc < 6; ++cc) mean[6 * b + cc] = s[ST_MEAN + cc];
      rounds[b] = round + 1;
      if (t_1e6[b] < 0 && err[b] < 1e-6) t_1e6[b] = 1e-3 * t_ms;
      bool stop = false;
      if (!(err[b] == err[b]) || std::isinf(err[b])) { code[b] = HZ_EDIVERGED; stop = true; }
      else if (err[b] < o.tol) { code[b] = HZ_OK; stop = true; }
      else if (inner_total[b] >= o.max_iters) { code[b] = HZ_NOT_CONVERGED; stop = true; }
      else {
        slow[b] = err[b] > 0.5 * prev_err[b] ? slow[b] + 1 : 0;
        if (slow[b] >= 3) { code[b] = HZ_STAGNATED; stop = true; }
      }
      if (stop) {
        finished[b] = 1;
        t_done[b] = 1e-3 * t_ms;
        continue;
      }
      prev_err[b] = err[b];
      next.push_back(b);
      double* si = inner_init.data() + b * kStatusLen;
      si[ST_NORM] = s[ST_NORM];
      si[ST_FIRST_ERR] = err[b];
      si[ST_BEST] = err[b];
      double tgt = rho * err[b];
      if (tgt < o.tol) tgt = 0.5 * o.tol;  // aim to finish in this round
      si[ST_REF] = std::max(0.3 * o.tol, tgt);
    }
    active = next;
    if (active.empty()) break;
    // ---- FP32 inner iterations on delta
    hip_check(hipMemcpyAsync(g->ws + g->off.status2, inner_init.data(), inner_init.size() * 8, hipMemcpyHostToDevice,
                             g->stream),
              "status H2D");
    hip_check(hipMemcpyAsync(act, active.data(), active.size() * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
    Ctx ci{g, dd2, act, (int)active.size()};
    {
      Launcher L{g};
      L.begin(K_ZERO, 0);
      L.end(launch_zero(dd2, act, ci.nact, 0, 3 * G.S / 2, g->stream), "zero");
    }
    std::vector<int> inner_act = active;
    int it = 0;
    for (;;) {
      const int parity = it & 1;
      pipeline_front<float>(ci, parity, 0);
      pipeline_x<float>(ci, 0);
      pipeline_back<float>(ci, parity, 2);
      finalize(ci, parity, 2, 0, inner_max);
      ++it;
      maybe_drain(g);
      if (it % check == 0 || it >= inner_max) {
        read_status(g, g->off.status2, nl);
        std::vector<int> na;
        for (int b : inner_act)
          if (g->h_status[b * kStatusLen + ST_DONE] == 0.0) na.push_back(b);
        if (na.empty()) break;
        if (it > inner_max + 1) fail(HZ_EINVAL, "inner stop rule did not fire");
        if (na.size() != inner_act.size()) {
          inner_act = na;
          hip_check(hipMemcpyAsync(act, na.data(), na.size() * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
          ci.nact = (int)na.size();
        }
      }
    }
    for (int b : active) inner_total[b] += (int)g->h_status[b * kStatusLen + ST_ITERS];
    // ---- U += delta
    hip_check(hipMemcpyAsync(act, active.data(), active.size() * 4, hipMemcpyHostToDevice, g->stream), "active H2D");
    {
      Launcher L{g};
      L.begin(K_ACCUM, 1);
      L.end(launch_accumulate(dd2, act, (int)active.size(), 3 * G.S, g->stream), "accumulate");
    }
  }
  hip_check(hipStreamSynchronize(g->stream), "sync");
  drain_profile(g);
  int worst = HZ_OK;
  for (int b = 0; b < nl; ++b) {
    if (code[b] < 0) worst = std::min(worst, code[b]);
    else if (worst >= 0) worst = std::max(worst, code[b]);
    if (sigma_mean)
      for (int cc = 0; cc < 6; ++cc) sigma_mean[6 * b + cc] = mean[6 * b + cc];
    if (info) {
      hz_info& in = info[b];
      in.status = code[b];
      in.iters = inner_total[b];
      in.outer_rounds = rounds[b];
      in.precision_used = HZ_FP32_REFINE;
      in.residual = err[b];
      in.seconds = t_done[b];
      in.seconds_to_1e6 = t_1e6[b];
    }
  }
  if (eps_out || sig_out) {
    for (int b = 0; b < nl; ++b) g->hdesc[b].status = P<double>(g, g->off.status2) + (size_t)b * kStatusLen;
    hip_check(hipMemcpyAsync(dd, g->hdesc.data(), nl * sizeof(Desc), hipMemcpyHostToDevice, g->stream), "desc H2D");
    zero_status(g, g->off.status2, nl);
    Ctx c{g, dd, act, nl};
    for (int b = 0; b < nl; ++b) output_fields(g, c, b, eps_out, sig_out, 1, 0);
  }
  return worst;
}

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
  auto* g = new hz_grid_s();
  g->geo.N1 = n1;
  g->geo.N2 = n2;
  g->geo.N3 = n3;
  g->geo.H1 = n1 / 2 + 1;
  g->geo.S = (long long)g->geo.H1 * n3 * n2;
  g->geo.N = (long long)n1 * n2 * n3;
  try {
    compute_tiling(g);
  } catch (...) {
    delete g;
    throw;
  }
  *out = g;
  return HZ_OK;
  HZ_GUARD_END
}

int hz_set_material(hz_grid g, int32_t n_phases, const double* C_voigt, const uint16_t* phase) {
  HZ_GUARD_BEGIN
  if (!g || !C_voigt || !phase || n_phases <= 0 || n_phases > 65536) fail(HZ_EINVAL, "bad material arguments");
  for (int p = 0; p < n_phases; ++p) {
    const double* C = C_voigt + 36 * p;
    for (int i = 0; i < 36; ++i)
      if (!std::isfinite(C[i])) fail(HZ_ENOTSPD, "stiffness has a non-finite entry");
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < i; ++j)
        if (std::fabs(C[i * 6 + j] - C[j * 6 + i]) > 1e-12 * (std::fabs(C[i * 6 + j]) + std::fabs(C[j * 6 + i]) + 1e-300))
          fail(HZ_ENOTSPD, "stiffness of phase " + std::to_string(p) + " is not symmetric");
    double M[36], ev[6];
    mandel(C, M);
    sym_eig6(M, ev);
    double hi = 0;
    for (double e : ev) hi = std::max(hi, std::fabs(e));
    for (double e : ev)
      if (e < -1e-12 * hi) fail(HZ_ENOTSPD, "stiffness of phase " + std::to_string(p) + " is not positive semi-definite");
  }
  const long long N = g->geo.N;
  for (long long i = 0; i < N; ++i)
    if (phase[i] >= n_phases) fail(HZ_EINVAL, "phase id out of range at voxel " + std::to_string(i));
  g->n_phases = n_phases;
  g->C.assign(C_voigt, C_voigt + 36 * (size_t)n_phases);
  g->phase.assign(phase, phase + N);
  g->material = true;
  g->ws = nullptr;  // tables must be re-uploaded
  return HZ_OK;
  HZ_GUARD_END
}

int64_t hz_workspace_bytes(hz_grid g, int32_t precision, int32_t n_loads) {
  HZ_GUARD_BEGIN
  if (!g || n_loads <= 0 || (precision != HZ_FP64 && precision != HZ_FP32_REFINE))
    fail(HZ_EINVAL, "bad workspace query");
  hz_grid_s::Off o;
  layout(g, precision, n_loads, o);
  return (int64_t)o.total;
  HZ_GUARD_END
}

int hz_bind_workspace(hz_grid g, void* dev_ptr, int64_t bytes, void* hip_stream, int32_t precision,
                      int32_t n_loads) {
  HZ_GUARD_BEGIN
  if (!g || !dev_ptr || n_loads <= 0 || (precision != HZ_FP64 && precision != HZ_FP32_REFINE))
    fail(HZ_EINVAL, "bad bind arguments");
  if (!g->material) fail(HZ_ENOMATERIAL, "material not set");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) fail(HZ_EINVAL, "workspace must be 256-byte aligned");
  hz_grid_s::Off o;
  layout(g, precision, n_loads, o);
  if ((int64_t)o.total > bytes) fail(HZ_EWORKSPACE, "workspace too small: need " + std::to_string(o.total) + " bytes");
  g->off = o;
  g->ws = static_cast<char*>(dev_ptr);
  g->ws_bytes = bytes;
  g->stream = static_cast<hipStream_t>(hip_stream);
  g->prec = precision;
  g->cap = n_loads;
  if (!g->h_status) hip_check(hipHostMalloc((void**)&g->h_status, (size_t)1024 * kStatusLen * 8), "hipHostMalloc");
  if (n_loads > 1024) fail(HZ_EINVAL, "at most 1024 loads per handle");
  upload_tables(g);
  return HZ_OK;
  HZ_GUARD_END
}

int hz_solve(hz_grid g, int32_t n_loads, const double* E, const hz_opts* o, double* sigma_mean, double* eps_out,
             double* sig_out, hz_info* info) {
  HZ_GUARD_BEGIN
  if (!g || !E || !o || n_loads <= 0) fail(HZ_EINVAL, "bad solve arguments");
  check_material(g);
  if (n_loads > g->cap) fail(HZ_EWORKSPACE, "workspace bound for fewer loads");
  if (o->precision != g->prec) fail(HZ_EWORKSPACE, "workspace bound for another precision");
  if (!(o->tol > 0) && o->fixed_iters < 0) fail(HZ_EINVAL, "tol must be > 0");
  if (o->max_iters < 0 || o->max_iters > kTraceCap - 1) fail(HZ_EINVAL, "max_iters out of range [0, 4096]");
  if (o->fixed_iters > kTraceCap - 1) fail(HZ_EINVAL, "fixed_iters out of range");
  for (int i = 0; i < 6 * n_loads; ++i)
    if (!std::isfinite(E[i])) fail(HZ_EINVAL, "non-finite applied strain");
  double C0[36], C0t[81];
  if (o->ref_mode == 1) std::memcpy(C0, o->ref_C, sizeof(C0));
  else auto_reference(g->n_phases, g->C.data(), C0);
  {
    double M[36], ev[6];
    mandel(C0, M);
    sym_eig6(M, ev);
    for (double e : ev)
      if (!(e > 0)) fail(HZ_ENOTSPD, "reference medium is not positive definite");
  }
  voigt_to_tensor(C0, C0t);
  g->c0_iso = isotropic(C0, g->lam0, g->mu0) ? 1 : 0;
  g->last_loads = n_loads;
  g->last_prec = o->precision;
  if (o->precision == HZ_FP64) return solve_fp64(g, n_loads, E, *o, C0t, sigma_mean, eps_out, sig_out, info);
  return solve_refine(g, n_loads, E, *o, C0t, sigma_mean, eps_out, sig_out, info);
  HZ_GUARD_END
}

int hz_effective_stiffness(hz_grid g, const hz_opts* o, double C_eff[36], hz_info info[6]) {
  HZ_GUARD_BEGIN
  if (!g || !o || !C_eff) fail(HZ_EINVAL, "bad arguments");
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
  if (!g || !out || load < 0 || load >= g->last_loads) fail(HZ_EINVAL, "bad arguments");
  check_material(g);
  const size_t n = (size_t)3 * g->geo.S;
  hip_check(hipStreamSynchronize(g->stream), "sync");
  if (g->last_prec == HZ_FP64) {
    double st[kStatusLen];
    hip_check(hipMemcpy(st, g->ws + g->off.status + (size_t)load * kStatusLen * 8, sizeof(st), hipMemcpyDeviceToHost),
              "status D2H");
    const int p = (int)st[ST_PARITY];
    hip_check(hipMemcpy(out, g->ws + (p ? g->off.u1[load] : g->off.u0[load]), n * 16, hipMemcpyDeviceToHost), "u D2H");
  } else {
    hip_check(hipMemcpy(out, g->ws + g->off.u64[load], n * 16, hipMemcpyDeviceToHost), "u D2H");
  }
  return HZ_OK;
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
  if (enable) {
    std::memset(g->prof_ms, 0, sizeof(g->prof_ms));
    std::memset(g->prof_n, 0, sizeof(g->prof_n));
  }
  g->prof = enable != 0;
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
        if (total_ms) total_ms[n] = g->prof_ms[k][d];
        if (launches) launches[n] = g->prof_n[k][d];
      }
      ++n;
    }
  return n;
  HZ_GUARD_END
}

void hz_destroy_grid(hz_grid g) {
  if (!g) return;
  for (auto e : g->ev_pool) (void)hipEventDestroy(e);
  for (auto e : g->iter_ev) (void)hipEventDestroy(e);
  if (g->h_status) (void)hipHostFree(g->h_status);
  delete g;
}

}  // extern "C"
