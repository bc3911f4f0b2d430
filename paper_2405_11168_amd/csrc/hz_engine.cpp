// Executor of the solver: grid shapes and tiling, device table layouts, and
// the tick loop that advances many per-load problems with grouped launches.
//
// One iteration of Algorithm 1 (Sec. 2.6) over a group of problems of one
// shape is five launches (P1 z expand, P2 inverse y, P3 fused x pass, P4
// forward y, P5 forward z + Green update) and the stop-rule kernel.  Every
// problem carries its own descriptor (buffers, material, reference medium,
// what the contraction and the stop rule do this iteration) and status block,
// so problems in different phases of their own solve share launches:
//   PS_IT64   plain FP64 iteration (eqs. basic_scheme_dep_2, tolerance)
//   PS_R0     FP32 iterations of the full problem from u = 0 (first estimate)
//   PS_SWEEP  one FP64 pass over the FP64 anchor U: measures eps, stores r
//   PS_CORR   FP32 iterations on a correction delta with r added, Ebar = 0, no eigenstress
// In exact arithmetic the FP32 iterates of a correction round are the plain
// scheme's iterates on U + delta, so the anchored scheme converges to the same
// fixed point; the stop decision is always the FP64 sweep's residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "hz_host.h"

// rows per x-pass block at most (a compile-time tuning default)
#ifndef HZ_TYX_CAP
#define HZ_TYX_CAP 16
#endif

namespace hz {

const char* const kKindNames[K_COUNT] = {"zexpand", "yinv", "xpass", "yfwd", "zcontract", "finalize", "accumulate",
                                         "zero", "zconvert3", "yinv3", "xc2r", "stencil", "xr2c", "yfwd3",
                                         "zcontract3", "zstrain"};

[[noreturn]] void fail(int code, const std::string& m) { throw HzError{code, m}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(HZ_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

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

namespace {

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

Plan plan_of(const std::vector<int>& v, int L) {
  Plan p{};
  p.L = L;
  p.np = (int)v.size();
  int ns = 1;
  for (int s = 0; s < p.np; ++s) {
    p.radix[s] = v[s];
    p.rLR[s] = recip(L / v[s]);
    p.rNs[s] = recip(ns);
    ns *= v[s];
  }
  return p;
}

// Factorisation of M = N1/2 for the fused x pass: first radix in {16, 8, 4, 2}
// (the load/split and merge/store stages), last radix in {5, 4, 3, 2} (the pass
// the constitutive law sits between: 6 components of it stay in registers), at
// least two passes and at most kThreads butterflies per line in the last one.
// Returns false where the unfused pass is used.
bool make_xplans(int M, Plan& inv, Plan& fwd) {
  const Plan p = make_plan(M);
  std::vector<int> v(p.radix, p.radix + p.np);
  auto pow2 = [](int r) { return r == 16 || r == 8 || r == 4 || r == 2; };
  if (v.empty()) return false;  // M = 1
  if (v.back() == 7) {
    // move a factor 2 from the first radix to the end
    if (!pow2(v[0])) return false;
    if (v[0] == 2) v.erase(v.begin());
    else v[0] /= 2;
    v.push_back(2);
  }
  if (v.back() == 16) {
    v.back() = 4;
    v.push_back(4);
  } else if (v.back() == 8) {
    v.back() = 2;
    v.push_back(4);
  } else if (v.size() == 1 && v[0] == 4) {
    v = {2, 2};
  }
  const int last = v.back();
  if (v.size() < 2 || !pow2(v[0]) || !(last == 5 || last == 4 || last == 3 || last == 2) || M / last > kThreads)
    return false;
  inv = plan_of(v, M);
  std::reverse(v.begin(), v.end());
  fwd = plan_of(v, M);
  return true;
}

// Factorisation of M = N1/2 for the stencil form's separate x transforms: the C2R
// split sits in the first pass and the R2C merge in the last one, and those passes
// hold both halves of a pair in registers, so they take the smallest power-of-two
// radix, or the smallest odd one where M has no factor 2 (the inverse plan starts
// with it, the forward plan is its reverse).  A prime M (and M = 1, a radix-1 pass)
// is one pass that splits and merges alone.
bool make_split_plans(int M, Plan& inv, Plan& fwd) {
  if (M == 1) {
    inv = fwd = plan_of({1}, 1);
    return true;
  }
  const Plan p = make_plan(M);
  std::vector<int> v(p.radix, p.radix + p.np);
  auto pow2 = [](int r) { return r == 16 || r == 8 || r == 4 || r == 2; };
  if (v.empty()) return false;
  if (v.size() == 1) {  // two passes at least where M has a factor 2
    if (v[0] == 16) v = {4, 4};
    else if (v[0] == 8) v = {2, 4};
    else if (v[0] == 4) v = {2, 2};
  }
  int best = -1;
  for (int i = 0; i < (int)v.size(); ++i)
    if (pow2(v[i]) && (best < 0 || v[i] < v[best])) best = i;
  if (best < 0)
    for (int i = 0; i < (int)v.size(); ++i)
      if (best < 0 || v[i] < v[best]) best = i;
  const int r = v[best];
  v.erase(v.begin() + best);
  v.insert(v.begin(), r);
  inv = plan_of(v, M);
  std::reverse(v.begin(), v.end());
  fwd = plan_of(v, M);
  return true;
}

}  // namespace

void Shape::init(int n1, int n2, int n3) {
  geo.N1 = n1;
  geo.N2 = n2;
  geo.N3 = n3;
  geo.H1 = n1 / 2 + 1;
  geo.S = (long long)geo.H1 * n3 * n2;
  geo.N = (long long)n1 * n2 * n3;
  const Geo& G = geo;
  plans[0] = make_plan(G.N1);
  plans[1] = make_plan(G.N2);
  plans[2] = make_plan(G.N3);
  plans[3] = make_plan(G.N1 / 2);
  xfused = make_xplans(G.N1 / 2, plans[4], plans[5]);
  const bool split = make_split_plans(G.N1 / 2, plans[6], plans[7]);
  // spectra are addressed with 32-bit offsets inside one load's 12 fields
  if (12 * G.S >= (1LL << 31)) fail(HZ_EINVAL, "grid too large");
  for (int d = 0; d < 2; ++d) {
    const int csz = d ? 16 : 8;
    const int tile = (d ? 16 : 32) * kThreads;  // elements per transform call
    const int rowcap = 256 / csz;               // TX giving 256-byte rows
    // z kernels: 3 comps x TX columns x N3 in LDS (+ N3 twiddles), TX | N2
    int tx = std::min(rowcap, G.N2);
    while (tx > 1 && (3 * tx * G.N3 > tile || (3 * tx * G.N3 + G.N3) * csz > kLdsBytesZ || G.N2 % tx)) --tx;
    if (3 * tx * G.N3 > tile || (3 * tx * G.N3 + G.N3) * csz > kLdsBytesZ) fail(HZ_EINVAL, "N3 too large");
    TXz[d] = tx;
    if (d) {
      // continuous operator: 6 lines per column, the largest divisor of tx that fits
      subc = 0;
      for (int s = tx; s >= 1; --s)
        if (tx % s == 0 && 6 * s * G.N3 <= tile && (6 * s * G.N3 + G.N3) * csz <= kLdsBytes) {
          subc = s;
          break;
        }
      rsubc6 = subc ? recip(6 * subc) : 0.f;
    }
    // y kernel: TX rows of N2 (+ N2 twiddles), the lines padded after every 16 elements
    // wherever one padded line fits (the longest lines go unpadded)
    int py = lds_pitch(G.N2);
    if ((py + G.N2) * csz > kLdsBytes) py = G.N2;
    int ty = std::min(64, tile / G.N2);
    while (ty > 1 && (ty * py + G.N2) * csz > kLdsBytes) --ty;
    if (ty < 1 || G.N2 > tile || (ty * py + G.N2) * csz > kLdsBytes) fail(HZ_EINVAL, "N2 too large");
    TXy[d] = ty;
    PYy[d] = py;
    // x kernel: 6 comps x TY rows x (N1/2+1) in LDS (+ N1 twiddles), TY | N2
    const int hp = (G.N1 / 2) | 1;  // lines hold M = N1/2 values; odd pitch spreads rows over banks
    // (the whole-block transforms of the unfused pass, used for output fields, and the
    // middle passes of the fused one hold at most `tile` elements)
    auto x_fits = [&](int t) { return (6 * t * hp + G.N1) * csz <= kLdsBytes && 6 * t * (G.N1 / 2) <= tile; };
    int tyx = std::min(HZ_TYX_CAP, G.N2);
    while (tyx > 1 && (!x_fits(tyx) || G.N2 % tyx)) --tyx;
    if (!x_fits(tyx)) fail(HZ_EINVAL, "N1 too large");
    TYx[d] = tyx;
    H1p[d] = hp;
    nbx[d] = 2 * G.N3 * (G.N2 / tyx);
    nbq[d] = G.H1 * (G.N2 / tx);
    // 3-field x transforms of the stencil form
    int ty3 = std::min(HZ_TY3_CAP, G.N2);
    // row tiles small enough that at least 3 work-groups share a CU's 160 KB (larger tiles
    // left 2 at N1 = 192; tiles sized for 4 measured slower at N1 = 128 and 256)
    const int x3_lds = 53 * 1024;
    auto x3_fits = [&](int t) { return (3 * t * hp + G.N1) * csz <= x3_lds && 3 * t * (G.N1 / 2) <= tile; };
    while (ty3 > 1 && (!x3_fits(ty3) || G.N2 % ty3)) --ty3;
    TY3[d] = x3_fits(ty3) ? ty3 : 0;
  }
  stencil = split && TY3[0] > 0 && TY3[1] > 0;
  sg.N1 = G.N1;
  sg.N2 = G.N2;
  sg.N3 = G.N3;
  // z segments of kStZ planes where that still leaves about six blocks per CU for one
  // load (fewer halo planes and per-block set-ups), else half of it
  const long long tiles_xy = (long long)((G.N1 + kStX - 1) / kStX) * ((G.N2 + kStY - 1) / kStY);
  sg.TZ = std::min(tiles_xy * ((G.N3 + kStZ - 1) / kStZ) >= 1536 ? kStZ : kStZ / 2, G.N3);
  sg.tx = (G.N1 + kStX - 1) / kStX;
  sg.ty = (G.N2 + kStY - 1) / kStY;
  sg.tz = (G.N3 + sg.TZ - 1) / sg.TZ;
  nbs = sg.tx * sg.ty * sg.tz;
}

// ---------------------------------------------------------------------------
// device table layouts
// ---------------------------------------------------------------------------
size_t shape_table_bytes(const Shape& s) {
  const int Ns[3] = {s.geo.N1, s.geo.N2, s.geo.N3};
  size_t b = 0;
  for (int a = 0; a < 3; ++a) b += align_up((size_t)Ns[a] * 16) + align_up((size_t)Ns[a] * 8);
  return b + align_up(sizeof(s.plans));
}

ShapeTables upload_shape_tables(const Shape& s, char* dev, hipStream_t st) {
  ShapeTables t{};
  const int Ns[3] = {s.geo.N1, s.geo.N2, s.geo.N3};
  size_t p = 0;
  std::vector<double> t64;
  std::vector<float> t32;
  for (int a = 0; a < 3; ++a) {
    const int L = Ns[a];
    t64.assign(2 * L, 0.0);
    t32.assign(2 * L, 0.0f);
    for (int j = 0; j < L; ++j) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)L;
      t64[2 * j] = (double)cosl(ang);
      t64[2 * j + 1] = (double)sinl(ang);
      t32[2 * j] = (float)cosl(ang);
      t32[2 * j + 1] = (float)sinl(ang);
    }
    t.tw64[a] = dev + p;
    hip_check(hipMemcpyAsync(dev + p, t64.data(), t64.size() * 8, hipMemcpyHostToDevice, st), "upload twiddles");
    p += align_up((size_t)L * 16);
    t.tw32[a] = dev + p;
    hip_check(hipMemcpyAsync(dev + p, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, st), "upload twiddles");
    p += align_up((size_t)L * 8);
    hip_check(hipStreamSynchronize(st), "sync");  // the staging vectors are reused
  }
  t.plans = reinterpret_cast<const Plan*>(dev + p);
  hip_check(hipMemcpyAsync(dev + p, s.plans, sizeof(s.plans), hipMemcpyHostToDevice, st), "upload plans");
  hip_check(hipStreamSynchronize(st), "sync");
  return t;
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

namespace {
// inverse of a 6x6 matrix by Gauss-Jordan elimination with partial pivoting
bool invert6(const double* A, double* X) {
  double a[6][12];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 12; ++j) a[i][j] = j < 6 ? A[i * 6 + j] : (j - 6 == i ? 1.0 : 0.0);
  for (int c = 0; c < 6; ++c) {
    int p = c;
    for (int r = c + 1; r < 6; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
    if (!(std::fabs(a[p][c]) > 0)) return false;
    if (p != c)
      for (int j = 0; j < 12; ++j) std::swap(a[p][j], a[c][j]);
    const double inv = 1.0 / a[c][c];
    for (int j = 0; j < 12; ++j) a[c][j] *= inv;
    for (int r = 0; r < 6; ++r)
      if (r != c) {
        const double f = a[r][c];
        for (int j = 0; j < 12; ++j) a[r][j] -= f * a[c][j];
      }
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) X[i * 6 + j] = a[i][j + 6];
  return true;
}

// sigma (tensor comps) of an engineering Voigt stiffness C acting on a strain e (tensor comps)
void voigt_apply(const double* C, const double* e, double* s) {
  const double g[6] = {e[0], e[1], e[2], 2 * e[3], 2 * e[4], 2 * e[5]};
  for (int i = 0; i < 6; ++i) {
    double a = 0;
    for (int j = 0; j < 6; ++j) a += C[i * 6 + j] * g[j];
    s[i] = a;
  }
}
}  // namespace

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

Reference make_reference(const hz_opts& o, const Material& m) {
  double C0[36];
  if (o.ref_mode == 1) std::memcpy(C0, o.ref_C, sizeof(C0));
  else auto_reference(m.n_phases, m.C.data(), C0);
  for (double v : C0)
    if (!std::isfinite(v)) fail(HZ_ENOTSPD, "reference medium has a non-finite entry");
  double M[36], ev[6];
  mandel(C0, M);
  sym_eig6(M, ev);
  for (double e : ev)
    if (!(e > 0)) fail(HZ_ENOTSPD, "reference medium is not positive definite");
  Reference r;
  voigt_to_tensor(C0, r.C0t);
  // lambda0^-1 on tensor comps: eps = D^-1 M^-1 D sigma with D = diag(1,1,1,v2,v2,v2)
  double Mi[36];
  if (!invert6(M, Mi)) fail(HZ_ENOTSPD, "reference medium is singular");
  const double sq[6] = {1, 1, 1, std::sqrt(2.0), std::sqrt(2.0), std::sqrt(2.0)};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) r.S0[i * 6 + j] = Mi[i * 6 + j] * sq[j] / sq[i];
  r.iso = isotropic(C0, r.lam0, r.mu0) ? 1 : 0;
  return r;
}

std::shared_ptr<Material> make_material(const Geo& geo, int n_phases, const double* C_voigt, const uint16_t* phase) {
  if (!C_voigt || !phase || n_phases <= 0 || n_phases > 65536) fail(HZ_EINVAL, "bad material arguments");
  for (int p = 0; p < n_phases; ++p) {
    const double* C = C_voigt + 36 * p;
    for (int i = 0; i < 36; ++i)
      if (!std::isfinite(C[i])) fail(HZ_ENOTSPD, "stiffness has a non-finite entry");
    // symmetry up to rounding relative to the largest entry (a rotated stiffness
    // carries noise of that size in its small entries)
    double cmax = 0;
    for (int i = 0; i < 36; ++i) cmax = std::max(cmax, std::fabs(C[i]));
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < i; ++j)
        if (std::fabs(C[i * 6 + j] - C[j * 6 + i]) > 1e-12 * cmax)
          fail(HZ_ENOTSPD, "stiffness of phase " + std::to_string(p) + " is not symmetric");
    double M[36], ev[6];
    mandel(C, M);
    sym_eig6(M, ev);
    double hi = 0;
    for (double e : ev) hi = std::max(hi, std::fabs(e));
    for (double e : ev)
      if (e < -1e-12 * hi) fail(HZ_ENOTSPD, "stiffness of phase " + std::to_string(p) + " is not positive semi-definite");
  }
  const long long N = geo.N;
  for (long long i = 0; i < N; ++i)
    if (phase[i] >= n_phases) fail(HZ_EINVAL, "phase id out of range at voxel " + std::to_string(i));
  auto m = std::make_shared<Material>();
  m->n_phases = n_phases;
  m->C.assign(C_voigt, C_voigt + 36 * (size_t)n_phases);
  m->phase.assign(phase, phase + N);
  // per-phase tables: (lambda, mu) when every phase is isotropic, else the Voigt upper triangle
  m->iso = 1;
  for (int p = 0; p < n_phases; ++p) {
    double lam, mu;
    if (!isotropic(m->C.data() + 36 * p, lam, mu)) m->iso = 0;
  }
  m->c64.assign((size_t)n_phases * 24, 0.0);
  for (int p = 0; p < n_phases; ++p) {
    const double* C = m->C.data() + 36 * p;
    if (m->iso) {
      isotropic(C, m->c64[2 * p], m->c64[2 * p + 1]);
    } else {
      int n = 0;
      for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) m->c64[(size_t)p * 24 + n++] = C[i * 6 + j];
    }
  }
  m->c32.resize(m->c64.size());
  for (size_t i = 0; i < m->c32.size(); ++i) m->c32[i] = (float)m->c64[i];
  std::vector<long long> cnt(n_phases, 0);
  for (long long i = 0; i < N; ++i) cnt[phase[i]]++;
  m->frac.resize(n_phases);
  for (int p = 0; p < n_phases; ++p) m->frac[p] = (double)cnt[p] / (double)N;
  return m;
}

std::shared_ptr<Material> with_eigenstrain(const Material& src, const double* eps0) {
  auto m = std::make_shared<Material>(src);
  m->eig.clear();
  m->tau64.clear();
  m->tau32.clear();
  std::fill(m->tau_mean, m->tau_mean + 6, 0.0);
  if (!eps0) return m;
  const int np = m->n_phases;
  for (int i = 0; i < 6 * np; ++i)
    if (!std::isfinite(eps0[i])) fail(HZ_EINVAL, "non-finite eigenstrain");
  m->eig.assign(eps0, eps0 + 6 * (size_t)np);
  m->tau64.assign((size_t)np * 8, 0.0);
  for (int p = 0; p < np; ++p) {
    double t[6];
    voigt_apply(m->C.data() + 36 * (size_t)p, eps0 + 6 * (size_t)p, t);
    for (int c = 0; c < 6; ++c) {
      m->tau64[(size_t)p * 8 + c] = t[c];
      m->tau_mean[c] += m->frac[p] * t[c];
    }
  }
  m->tau32.resize(m->tau64.size());
  for (size_t i = 0; i < m->tau32.size(); ++i) m->tau32[i] = (float)m->tau64[i];
  return m;
}

size_t material_table_bytes(int np, long long N) {
  return align_up((size_t)np * 24 * 8) + align_up((size_t)np * 24 * 4) + align_up((size_t)N * 2) +
         align_up((size_t)np * 8 * 8) + align_up((size_t)np * 8 * 4);
}

size_t material_table_bytes(const Material& m) { return material_table_bytes(m.n_phases, (long long)m.phase.size()); }

MaterialTables upload_material_tables(const Material& m, char* dev, hipStream_t st) {
  MaterialTables t{};
  size_t p = 0;
  t.C64 = reinterpret_cast<const double*>(dev + p);
  hip_check(hipMemcpyAsync(dev + p, m.c64.data(), m.c64.size() * 8, hipMemcpyHostToDevice, st), "upload C");
  p += align_up(m.c64.size() * 8);
  t.C32 = reinterpret_cast<const float*>(dev + p);
  hip_check(hipMemcpyAsync(dev + p, m.c32.data(), m.c32.size() * 4, hipMemcpyHostToDevice, st), "upload C");
  p += align_up(m.c32.size() * 4);
  t.phase = reinterpret_cast<const uint16_t*>(dev + p);
  hip_check(hipMemcpyAsync(dev + p, m.phase.data(), m.phase.size() * 2, hipMemcpyHostToDevice, st),
            "upload phase map");
  p += align_up(m.phase.size() * 2);
  if (!m.tau64.empty()) {
    t.tau64 = reinterpret_cast<const double*>(dev + p);
    hip_check(hipMemcpyAsync(dev + p, m.tau64.data(), m.tau64.size() * 8, hipMemcpyHostToDevice, st),
              "upload eigenstress");
    p += align_up((size_t)m.n_phases * 8 * 8);
    t.tau32 = reinterpret_cast<const float*>(dev + p);
    hip_check(hipMemcpyAsync(dev + p, m.tau32.data(), m.tau32.size() * 4, hipMemcpyHostToDevice, st),
              "upload eigenstress");
  }
  hip_check(hipStreamSynchronize(st), "sync");
  return t;
}

size_t prob_bytes(const Shape& s, int prec, bool trace) {
  const size_t S = (size_t)s.geo.S;
  const size_t ub = prec == HZ_FP64 ? 16 : 8;
  // FP64: two displacement buffers.  FP32+refine: the two FP32 buffers share one block
  // of FP64 size (the second FP64 buffer of a fallback to FP64 iterations), then U, r
  size_t b = align_up(12 * S * 16) + (prec == HZ_FP64 ? 2 * align_up(3 * S * ub) : align_up(3 * S * 16));
  if (prec != HZ_FP64) b += align_up(3 * S * 16) + align_up(3 * S * 8);
  b += align_up((size_t)s.nbx_max() * 6 * 8) + align_up((size_t)s.nbq_max() * 8);
  if (trace) b += align_up((size_t)kTraceCap * 7 * 8);
  return b;
}

ProbBuffers carve_prob(const Shape& s, int prec, bool trace, char* dev) {
  const size_t S = (size_t)s.geo.S;
  const size_t ub = prec == HZ_FP64 ? 16 : 8;
  ProbBuffers b{};
  size_t p = 0;
  auto take = [&](size_t bytes) {
    char* r = dev + p;
    p += align_up(bytes);
    return r;
  };
  b.spec = take(12 * S * 16);
  if (prec == HZ_FP64) {
    b.u0 = take(3 * S * ub);
    b.u1 = take(3 * S * ub);
  } else {
    // 3 S complex doubles, or two FP32 buffers; u1 starts 3 S complex floats in (S is
    // even, so a multiple of 16 bytes)
    char* u = take(3 * S * 16);
    b.u0 = u;
    b.u1 = u + 3 * S * 8;
  }
  if (prec != HZ_FP64) {
    b.u64 = take(3 * S * 16);
    b.r32 = take(3 * S * 8);
  }
  b.part_sig = reinterpret_cast<double*>(take((size_t)s.nbx_max() * 6 * 8));
  b.part_res = reinterpret_cast<double*>(take((size_t)s.nbq_max() * 8));
  b.trace = trace ? reinterpret_cast<double*>(take((size_t)kTraceCap * 7 * 8)) : nullptr;
  return b;
}

// ---------------------------------------------------------------------------
// per-kernel event timing
// ---------------------------------------------------------------------------
void Prof::reset() {
  std::memset(ms, 0, sizeof(ms));
  std::memset(n, 0, sizeof(n));
  pending.clear();
  used = 0;
}

void Prof::drain() {
  for (auto& p : pending) {
    float t = 0;
    hip_check(hipEventElapsedTime(&t, p.second.first, p.second.second), "hipEventElapsedTime");
    ms[p.first / 2][p.first % 2] += t;
    n[p.first / 2][p.first % 2] += 1;
  }
  pending.clear();
  used = 0;
}

Prof::~Prof() {
  for (auto e : pool) (void)hipEventDestroy(e);
}

namespace {

struct Launch {
  Engine& e;
  int key;
  hipEvent_t a = nullptr;
  hipEvent_t take() {
    Prof& p = *e.prof;
    if (p.used == p.pool.size()) {
      hipEvent_t ev;
      hip_check(hipEventCreate(&ev), "hipEventCreate");
      p.pool.push_back(ev);
    }
    return p.pool[p.used++];
  }
  Launch(Engine& eng, int kind, int dbl) : e(eng), key(kind * 2 + dbl) {
    if (e.prof->records(key)) {
      a = take();
      hip_check(hipEventRecord(a, e.stream), "hipEventRecord");
    }
  }
  void done(hipError_t err, const char* what) {
    hip_check(err, what);
    if (e.prof->records(key)) {
      hipEvent_t b = take();
      hip_check(hipEventRecord(b, e.stream), "hipEventRecord");
      e.prof->pending.push_back({key, {a, b}});
    }
  }
};

ZGeo zgeo(const Shape& sh, int d) {
  const Geo& G = sh.geo;
  const int TX = sh.TXz[d];
  return ZGeo{G.N1, G.N2, G.N3, G.H1, TX, G.N2 / TX, recip(TX), recip(3 * TX), recip(G.N2 / TX), G.S};
}

// P1 (expand + inverse z) and P2 (inverse y); the continuous-frequency operator has
// z kernels of its own (FP64), the rotated one shares the tetrahedral kernels
template <typename T>
void pass_front(Engine& e, const Shape& sh, const ShapeTables& tb, const int* act, int n, int green) {
  const int d = sizeof(T) == 8;
  const Geo& G = sh.geo;
  const char* const* tw = d ? tb.tw64 : tb.tw32;
  const ZGeo zg = zgeo(sh, d);
  {
    Launch L(e, K_ZEXP, d);
    if (green == GREEN_CONTINUOUS)
      L.done(launch_zexp_cont(e.d_desc, act, n, zg, sh.subc, sh.rsubc6, sh.plans + 2, tb.tw64[2], e.stream),
             "z expand");
    else
      L.done(launch_zexp<T>(e.d_desc, act, n, zg, sh.plans + 2, tw[2], tb.tw64[0], tb.tw64[1], e.stream),
             "z expand");
  }
  const YGeo yg = sh.ygeo(d, (long long)12 * G.H1 * G.N3, 0);
  Launch L(e, K_YINV, d);
  L.done(launch_yline<T>(e.d_desc, act, n, yg, sh.plans + 1, tw[1], true, e.stream), "y inverse");
}

// P1 of the strain-based form (apply the previous update to the strains, inverse z)
// and P2
template <typename T>
void pass_front_strain(Engine& e, const Shape& sh, const ShapeTables& tb, const int* act, int n) {
  const int d = sizeof(T) == 8;
  const Geo& G = sh.geo;
  const char* const* tw = d ? tb.tw64 : tb.tw32;
  const ZGeo zg = zgeo(sh, d);
  {
    Launch L(e, K_ZSTRAIN, d);
    L.done(launch_zstrain<T>(e.d_desc, act, n, zg, sh.plans + 2, tw[2], tb.tw64[0], tb.tw64[1], tb.tw64[2],
                             e.stream),
           "z strain");
  }
  const YGeo yg = sh.ygeo(d, (long long)12 * G.H1 * G.N3, 0);
  Launch L(e, K_YINV, d);
  L.done(launch_yline<T>(e.d_desc, act, n, yg, sh.plans + 1, tw[1], true, e.stream), "y inverse");
}

// P3: x pass; with fields, T1 writes and T2 then adds its half of the averages.  The
// active list holds the problems ordered by material kind (KIND_ISO, KIND_EIG bits),
// cnt[k] of kind k, each kind launched with its own instantiation.
template <typename T>
void pass_x(Engine& e, const Shape& sh, const ShapeTables& tb, const int* act, int n, const int* cnt, int fields) {
  const int d = sizeof(T) == 8;
  const Geo& G = sh.geo;
  const char* const* tw = d ? tb.tw64 : tb.tw32;
  for (int h = fields ? 0 : -1; h < (fields ? 2 : 0); ++h) {
    const int M = G.N1 / 2;
    XGeo xg{G.N1, G.N2, G.N3, G.H1, sh.H1p[d], sh.TYx[d], M, recip(sh.TYx[d]), recip(M / 2 + 1), recip(M),
            G.S, 1.0 / (double)G.N, fields, h, 1.0f, 1.0f};
    Launch L(e, K_XPASS, d);
    if (sh.xfused && !fields) {
      const Plan& pi = sh.plans[4];
      xg.rNI = recip(M / pi.radix[0] / 2 + 1);
      xg.rLRm = recip(M / pi.radix[pi.np - 1]);
      for (int k = 0, off = 0; k < 4; off += cnt[k++])
        if (cnt[k] > 0)
          L.done(launch_xfused<T>(e.d_desc, act + off, cnt[k], k, xg, sh.plans + 4, sh.plans + 5, tw[0], e.stream),
                 "x pass");
    } else {
      L.done(launch_xpass<T>(e.d_desc, act, n, xg, sh.plans + 3, tw[0], e.stream), "x pass");
    }
  }
}

// P4 (forward y), P5 (forward z + contraction + update) and the stop rule
template <typename T>
void pass_back(Engine& e, const Shape& sh, const ShapeTables& tb, const int* act, int n, int c0, int green) {
  const int d = sizeof(T) == 8;
  const Geo& G = sh.geo;
  const char* const* tw = d ? tb.tw64 : tb.tw32;
  {
    const YGeo yg = sh.ygeo(d, (long long)12 * G.H1 * G.N3, 0);
    Launch L(e, K_YFWD, d);
    L.done(launch_yline<T>(e.d_desc, act, n, yg, sh.plans + 1, tw[1], false, e.stream), "y forward");
  }
  {
    const ZGeo zg = zgeo(sh, d);
    Launch L(e, K_ZCON, d);
    if (green == GREEN_CONTINUOUS)
      L.done(launch_zcon_cont(e.d_desc, act, n, zg, sh.subc, sh.rsubc6, sh.plans + 2, tb.tw64[2], e.stream),
             "z contract");
    else
      L.done(launch_zcon<T>(e.d_desc, act, n, false, c0, zg, sh.plans + 2, tw[2], tb.tw64[0], tb.tw64[1],
                            tb.tw64[2], e.stream),
             "z contract");
  }
  const FinGeo fg{sh.nbx[d], sh.nbq[d], 1.0 / (double)G.N};
  Launch L(e, K_FINAL, d);
  L.done(launch_finalize(e.d_desc, act, n, fg, e.stream), "finalize");
}

template <typename T>
void iteration(Engine& e, const Shape& sh, const ShapeTables& tb, const int* act, int n, const int* cnt, int c0,
               int green) {
  pass_front<T>(e, sh, tb, act, n, green);
  pass_x<T>(e, sh, tb, act, n, cnt, 0);
  pass_back<T>(e, sh, tb, act, n, c0, green);
}

// the strain-based form (Algorithm 2): the strains are the iterate, the contraction
// stores w = Omega r (cmode 3) and the next P1 applies it
template <typename T>
void iteration_strain(Engine& e, const Shape& sh, const ShapeTables& tb, const int* act, int n, const int* cnt,
                      int c0) {
  pass_front_strain<T>(e, sh, tb, act, n);
  pass_x<T>(e, sh, tb, act, n, cnt, 0);
  pass_back<T>(e, sh, tb, act, n, c0, GREEN_TETRA);
}

// the same iteration in the stencil form: 3-field transforms around the real-space
// strain / constitutive / corner-force kernel.  The displacement state is held in the
// mixed domain (inverse z transform of u(q)): the iteration starts with the inverse y
// transform of the state and the contraction updates the state in that domain.
template <typename T>
void iteration_stencil(Engine& e, const Shape& sh, const ShapeTables& tb, const int* act, int n, const int* cnt,
                       const int* maxph,
                       int c0) {
  const int d = sizeof(T) == 8;
  const Geo& G = sh.geo;
  const char* const* tw = d ? tb.tw64 : tb.tw32;
  const ZGeo zg = zgeo(sh, d);
  {
    const YGeo yg = sh.ygeo(d, (long long)3 * G.H1 * G.N3, 0, 1);
    Launch L(e, K_YINV3, d);
    L.done(launch_yline<T>(e.d_desc, act, n, yg, sh.plans + 1, tw[1], true, e.stream), "y inverse");
  }
  const int M = G.N1 / 2;
  XGeo xg{G.N1, G.N2, G.N3, G.H1, sh.H1p[d], sh.TY3[d], M, recip(sh.TY3[d]), recip(M / 2 + 1), recip(M),
          G.S, 1.0 / (double)G.N, 0, 0, 1.0f, 1.0f};
  {
    const Plan& pi = sh.plans[6];
    xg.rNI = recip(M / pi.radix[0] / 2 + 1);
    Launch L(e, K_XC2R, d);
    L.done(launch_xc2r<T>(e.d_desc, act, n, xg, sh.plans + 6, pi.radix[0], tw[0], e.stream), "x c2r");
  }
  {
    Launch L(e, K_STEN, d);
    for (int k = 0, off = 0; k < 4; off += cnt[k++])
      if (cnt[k] > 0) L.done(launch_stencil<T>(e.d_desc, act + off, cnt[k], k, maxph[k], sh.sg, e.stream), "stencil");
  }
  {
    const Plan& pf = sh.plans[7];
    xg.rNI = recip(M / pf.radix[pf.np - 1] / 2 + 1);
    Launch L(e, K_XR2C, d);
    L.done(launch_xr2c<T>(e.d_desc, act, n, xg, sh.plans + 7, pf.radix[pf.np - 1], tw[0], e.stream), "x r2c");
  }
  {
    const YGeo yg = sh.ygeo(d, (long long)3 * G.H1 * G.N3, 9 * G.S);
    Launch L(e, K_YFWD3, d);
    L.done(launch_yline<T>(e.d_desc, act, n, yg, sh.plans + 1, tw[1], false, e.stream), "y forward");
  }
  {
    Launch L(e, K_ZCON3, d);
    L.done(launch_zcon<T>(e.d_desc, act, n, true, c0, zg, sh.plans + 2, tw[2], tb.tw64[0], tb.tw64[1], tb.tw64[2],
                          e.stream),
           "z contract");
  }
  const FinGeo fg{sh.nbs, sh.nbq[d], 1.0 / (double)G.N};
  Launch L(e, K_FINAL, d);
  L.done(launch_finalize(e.d_desc, act, n, fg, e.stream), "finalize");
}

bool kernel_fp64(PState s) { return s == PS_IT64 || s == PS_SWEEP || s == PS_FB64; }

// material kind in the problem's current state (a correction round has no eigenstress)
int kind_of(const Prob* p) {
  return (p->base.iso ? KIND_ISO : 0) | (p->base.tau64 && p->st != PS_CORR ? KIND_EIG : 0);
}

}  // namespace

// ---------------------------------------------------------------------------
// executor
// ---------------------------------------------------------------------------
size_t Engine::table_bytes(int cap) {
  return align_up((size_t)cap * sizeof(Desc)) + align_up((size_t)cap * kStatusLen * 8) +
         align_up((size_t)(4 * cap + 16) * 4);
}

void Engine::init(int c, bool pinned_mirrors) {
  if (cap) fail(HZ_EINVAL, "executor initialised twice");
  cap = c;
  active_cap = 4 * c + 16;
  pinned = pinned_mirrors;
  if (pinned) {
    hip_check(hipHostMalloc((void**)&h_desc, (size_t)cap * sizeof(Desc)), "hipHostMalloc");
    hip_check(hipHostMalloc((void**)&h_status, (size_t)cap * kStatusLen * 8), "hipHostMalloc");
    hip_check(hipHostMalloc((void**)&h_active, (size_t)active_cap * 4), "hipHostMalloc");
  } else {
    // ordinary host memory: the copies from and to it are staged by the runtime
    h_desc = new Desc[cap];
    h_status = new double[(size_t)cap * kStatusLen];
    h_active = new int[active_cap];
  }
  std::memset(h_status, 0, (size_t)cap * kStatusLen * 8);
}

void Engine::bind(char* dev, hipStream_t s) {
  stream = s;
  d_desc = reinterpret_cast<Desc*>(dev);
  size_t p = align_up((size_t)cap * sizeof(Desc));
  d_status = reinterpret_cast<double*>(dev + p);
  p += align_up((size_t)cap * kStatusLen * 8);
  d_active = reinterpret_cast<int*>(dev + p);
}

hipEvent_t Engine::event(size_t i) {
  while (evs.size() <= i) {
    hipEvent_t ev;
    hip_check(hipEventCreate(&ev), "hipEventCreate");
    evs.push_back(ev);
  }
  return evs[i];
}

void Engine::set_lanes(int n) {
  if (n < 1 || n > kMaxLanes) fail(HZ_EINVAL, "stream count out of range [1, 8]");
  while ((int)side.size() < n - 1) {
    hipStream_t st;
    hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    side.push_back(st);
  }
  while (fork_join.size() < side.size() + 1) {
    hipEvent_t ev;
    hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreateWithFlags");
    fork_join.push_back(ev);
  }
  lanes = n;
}

void Engine::start_clock() {
  if (!epoch) hip_check(hipEventCreate(&epoch), "hipEventCreate");
  hip_check(hipEventRecord(epoch, stream), "hipEventRecord");
}

Engine::~Engine() {
  for (auto st : side) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto ev : fork_join) (void)hipEventDestroy(ev);
  for (auto ev : evs) (void)hipEventDestroy(ev);
  if (epoch) (void)hipEventDestroy(epoch);
  if (pinned) {
    if (h_desc) (void)hipHostFree(h_desc);
    if (h_status) (void)hipHostFree(h_status);
    if (h_active) (void)hipHostFree(h_active);
  } else {
    delete[] h_desc;
    delete[] h_status;
    delete[] h_active;
  }
}

void Engine::add(Prob* p) {
  if (p->slot < 0 || p->slot >= cap) fail(HZ_EINVAL, "problem slot out of range");
  p->st = p->prec == HZ_FP64 ? PS_IT64 : PS_R0;
  p->enter = true;
  p->accum = false;
  p->started = false;
  live.push_back(p);
}

void Engine::convert_stencil_state(void* u, const Prob& p, bool inverse) {
  Launch L(*this, K_ZCONV3, 1);
  L.done(launch_zconv3(u, inverse, zgeo(*p.shape, 1), p.shape->plans + 2, p.tab.tw64[2], stream), "z convert");
}

void Engine::enter_state(Prob* p) {
  Desc d = p->base;
  d.status = d_status + (size_t)p->slot * kStatusLen;
  double* s = h_status + (size_t)p->slot * kStatusLen;
  std::fill(s, s + kStatusLen, 0.0);
  s[ST_K1E6] = -1.0;
  d.trace = nullptr;
  d.trace_len = 0;
  d.tol = p->tol;
  d.max_iters = p->max_iters;
  d.fixed_iters = p->fixed_iters;
  d.inner_max = p->inner_max;
  for (int c = 0; c < 6; ++c) s[ST_EBAR + c] = p->Eb0[c];
  switch (p->st) {
    case PS_IT64:
      d.cmode = p->form == HZ_SCHEME_STRAIN ? 3 : 0;
      d.fmode = 0;
      d.src = 0;
      d.trace = p->base.trace;
      d.trace_len = p->base.trace ? kTraceCap : 0;
      p->times.clear();
      break;
    case PS_R0:
      // stop well above the FP32 rounding floor of the full problem (~1e-6 relative);
      // correction rounds take the residual the rest of the way
      d.cmode = 0;
      d.fmode = 3;
      d.src = 0;
      s[ST_REF] = std::max(0.5 * p->tol, 3e-5);
      s[ST_BEST] = 1e300;
      break;
    case PS_SWEEP:
      d.cmode = 1;
      d.fmode = 1;
      d.src = 1;
      break;
    case PS_FB64:
      // plain FP64 iterations of the full problem from U, ping-ponging between U and the
      // block of the two FP32 buffers; the rest of the iteration budget
      d.cmode = 0;
      d.fmode = 0;
      d.src = 0;
      d.u[0] = p->base.u64;
      d.u[1] = p->base.u[0];
      d.fixed_iters = -1;
      d.max_iters = std::max(0, p->max_iters - p->inner_total);
      break;
    case PS_CORR: {
      d.cmode = 2;
      d.fmode = 2;
      d.src = 0;
      // the correction solves the linear part alone: no mean strain, no eigenstress
      for (int c = 0; c < 6; ++c) s[ST_EBAR + c] = 0.0;
      d.tau64 = nullptr;
      d.tau32 = nullptr;
      // residual of U + delta is measured against the sweep's ||<sigma>||; the round
      // stops at rho times the sweep's residual (half of tol when that is below tol)
      s[ST_NORM] = p->sweep_norm;
      s[ST_FIRST_ERR] = p->err;
      s[ST_BEST] = p->err;
      double tgt = p->rho * p->err;
      if (tgt < p->tol) tgt = 0.5 * p->tol;
      s[ST_REF] = std::max(0.3 * p->tol, tgt);
      break;
    }
    default:
      fail(HZ_EINVAL, "problem entered an invalid state");
  }
  h_desc[p->slot] = d;
  p->k0 = 0;
}

std::vector<Prob*> Engine::tick() {
  std::vector<Prob*> fin;
  if (live.empty()) return fin;
  struct Seg {
    int cat;  // 0 accumulate, 1 zero u0 FP64, 2 zero u0 FP32, 3 zero U, 4 iterate FP64, 5 iterate FP32
    const Prob* proto;
    std::vector<Prob*> ps;
    int off = 0, K = 0, ev0 = 0;
    int cnt[4]{};  // problems of each material kind, in kind order
    int maxph[4]{};  // most phases among the problems of each kind (stiffness tables in LDS)
  };
  std::vector<Seg> segs;
  auto put = [&](int cat, Prob* p) {
    for (auto& s : segs)
      if (s.cat == cat && s.proto->tab.plans == p->tab.plans &&
          (cat < 4 || (s.proto->form == p->form && s.proto->green == p->green))) {
        s.ps.push_back(p);
        return;
      }
    segs.push_back(Seg{cat, p, {p}});
  };
  bool dirty = false;
  int hi = 0;
  for (Prob* p : live) {
    hi = std::max(hi, p->slot + 1);
    if (p->accum) put(0, p);
    if (p->enter) {
      enter_state(p);
      dirty = true;
      if (p->st == PS_IT64) {
        if (p->u_init) {  // resume: iterate 0 is the given displacement
          hip_check(hipMemcpyAsync(p->base.u[0], p->u_init, (size_t)3 * p->shape->geo.S * 16, hipMemcpyHostToDevice,
                                   stream),
                    "initial displacement H2D");
          if (p->form == HZ_SCHEME_STENCIL) convert_stencil_state(p->base.u[0], *p, true);
        } else {
          put(1, p);
        }
      }
      if (p->st == PS_R0) {
        put(2, p);
        put(3, p);
      }
      if (p->st == PS_CORR) put(2, p);
    }
    put(kernel_fp64(p->st) ? 4 : 5, p);
  }
  std::stable_sort(segs.begin(), segs.end(), [](const Seg& a, const Seg& b) { return a.cat < b.cat; });
  // iterate groups list their problems by material kind (the kernels that apply the
  // constitutive law have an instantiation for each)
  for (auto& s : segs)
    if (s.cat >= 4) {
      std::stable_sort(s.ps.begin(), s.ps.end(), [](const Prob* a, const Prob* b) { return kind_of(a) < kind_of(b); });
      for (const Prob* p : s.ps) {
        s.cnt[kind_of(p)]++;
        s.maxph[kind_of(p)] = std::max(s.maxph[kind_of(p)], p->base.n_phases);
      }
    }
  int cur = 0;
  for (auto& s : segs) {
    s.off = cur;
    for (Prob* p : s.ps) h_active[cur++] = p->slot;
    if (cur > active_cap) fail(HZ_EINVAL, "active list overflow");
  }
  hip_check(hipMemcpyAsync(d_active, h_active, (size_t)cur * 4, hipMemcpyHostToDevice, stream), "active H2D");
  // U += delta reads the finished round's parity from the status block: before the upload
  for (auto& s : segs)
    if (s.cat == 0) {
      Launch L(*this, K_ACCUM, 1);
      L.done(launch_accumulate(d_desc, d_active + s.off, (int)s.ps.size(), 3 * s.proto->shape->geo.S, stream),
             "accumulate");
      for (Prob* p : s.ps) p->accum = false;
    }
  if (dirty) {
    hip_check(hipMemcpyAsync(d_desc, h_desc, (size_t)hi * sizeof(Desc), hipMemcpyHostToDevice, stream), "desc H2D");
    hip_check(hipMemcpyAsync(d_status, h_status, (size_t)hi * kStatusLen * 8, hipMemcpyHostToDevice, stream),
              "status H2D");
  }
  for (auto& s : segs) {
    if (s.cat < 1 || s.cat > 3) continue;
    const long long S = s.proto->shape->geo.S;
    // counts in 16-byte units: FP64 u is 3S complex doubles, FP32 u 3S complex floats
    const long long n16 = s.cat == 2 ? 3 * S / 2 : 3 * S;
    const int what = s.cat == 3 ? 2 : 0;
    Launch L(*this, K_ZERO, s.cat != 2);
    L.done(launch_zero(d_desc, d_active + s.off, (int)s.ps.size(), what, n16, stream), "zero");
  }
  for (Prob* p : live) p->enter = false;
  size_t nev = 0;
  hip_check(hipEventRecord(event(nev++), stream), "hipEventRecord");  // tick start
  std::vector<Seg*> its;
  for (auto& s : segs) {
    if (s.cat < 4) continue;
    int need = 1;
    for (Prob* p : s.ps) {
      int r = 1;
      if (p->st == PS_IT64) r = (p->fixed_iters >= 0 ? p->fixed_iters : p->max_iters) - p->k0 + 1;
      else if (p->st == PS_R0 || p->st == PS_CORR) r = p->inner_max - p->k0;
      else if (p->st == PS_FB64) r = std::max(0, p->max_iters - p->inner_total) - p->k0 + 1;
      need = std::max(need, r);
    }
    s.K = std::max(1, std::min(check_every, need));
    s.ev0 = (int)nev;
    nev += s.K;
    its.push_back(&s);
  }
  if (nev > 0) event(nev - 1);  // every event of the tick exists before any is recorded
  // lanes: with one, the groups run in turn on `stream`; with more, each group goes to
  // the lane with the least estimated work so far (voxels x problems x iterations,
  // FP64 counted twice) and the lanes take one iteration of each of their groups in
  // turn.  Groups hold disjoint problems, so the order changes no result.
  const int L = std::min<int>(lanes, (int)its.size());
  std::vector<int> lane_of(its.size(), 0);
  if (L > 1) {
    std::vector<double> cost(its.size()), load(L, 0.0);
    std::vector<int> order(its.size());
    for (size_t j = 0; j < its.size(); ++j) {
      cost[j] = (double)its[j]->proto->shape->geo.N * its[j]->ps.size() * its[j]->K * (its[j]->cat == 4 ? 2 : 1);
      order[j] = (int)j;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int j : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      lane_of[j] = l;
      load[l] += cost[j];
    }
    hip_check(hipEventRecord(fork_join[0], stream), "hipEventRecord");
    for (int l = 1; l < L; ++l) hip_check(hipStreamWaitEvent(side[l - 1], fork_join[0], 0), "hipStreamWaitEvent");
  }
  const hipStream_t main_stream = stream;
  auto run_iteration = [&](Seg& s, int i) {
    const int* act = d_active + s.off;
    const int n = (int)s.ps.size();
    const int form = s.proto->form;
    int c0 = 0;
    for (const Prob* q : s.ps) c0 |= q->base.c0_iso ? 1 : 2;
    const Shape& sh = *s.proto->shape;
    const ShapeTables& tb = s.proto->tab;
    if (s.cat == 4) {
      if (form == HZ_SCHEME_STENCIL) iteration_stencil<double>(*this, sh, tb, act, n, s.cnt, s.maxph, c0);
      else if (form == HZ_SCHEME_STRAIN) iteration_strain<double>(*this, sh, tb, act, n, s.cnt, c0);
      else iteration<double>(*this, sh, tb, act, n, s.cnt, c0, s.proto->green);
    } else {
      if (form == HZ_SCHEME_STENCIL) iteration_stencil<float>(*this, sh, tb, act, n, s.cnt, s.maxph, c0);
      else iteration<float>(*this, sh, tb, act, n, s.cnt, c0, s.proto->green);
    }
    hip_check(hipEventRecord(evs[s.ev0 + i], stream), "hipEventRecord");
  };
  if (L <= 1) {
    for (Seg* s : its)
      for (int i = 0; i < s->K; ++i) run_iteration(*s, i);
  } else {
    struct Restore {  // `stream` names the server's stream again however the loop ends
      Engine& e;
      hipStream_t s;
      ~Restore() { e.stream = s; }
    } restore{*this, main_stream};
    int kmax = 0;
    for (Seg* s : its) kmax = std::max(kmax, s->K);
    for (int i = 0; i < kmax; ++i)
      for (size_t j = 0; j < its.size(); ++j) {
        if (i >= its[j]->K) continue;
        stream = lane_of[j] == 0 ? main_stream : side[lane_of[j] - 1];  // the launches below go there
        run_iteration(*its[j], i);
      }
    stream = main_stream;
    for (int l = 1; l < L; ++l) {
      hip_check(hipEventRecord(fork_join[l], side[l - 1]), "hipEventRecord");
      hip_check(hipStreamWaitEvent(stream, fork_join[l], 0), "hipStreamWaitEvent");
    }
  }
  hip_check(hipMemcpyAsync(h_status, d_status, (size_t)hi * kStatusLen * 8, hipMemcpyDeviceToHost, stream),
            "status D2H");
  hip_check(hipStreamSynchronize(stream), "sync");
  if (prof->on) prof->drain();
  ev_ms.assign(nev, 0.0);
  for (size_t i = 0; i < nev; ++i) {
    float t = 0;
    hip_check(hipEventElapsedTime(&t, epoch, evs[i]), "hipEventElapsedTime");
    ev_ms[i] = t;
  }
  for (auto& s : segs) {
    if (s.cat < 4) continue;
    for (Prob* p : s.ps) {
      if (!p->started) {
        p->started = true;
        p->t_start = ev_ms[0];
      }
      const double* st = h_status + (size_t)p->slot * kStatusLen;
      const int k1 = (int)st[ST_K];
      if (k1 - p->k0 > s.K || k1 < p->k0) fail(HZ_EINVAL, "iteration count out of step");
      advance(p, st, ev_ms.data() + s.ev0);
      if (p->st == PS_DONE) fin.push_back(p);
    }
  }
  // a problem that fell back to FP64 iterations reports its iterate through U like every
  // refined problem: copy it there when it sits in the second buffer
  for (Prob* p : fin)
    if (p->fb && p->parity == 1)
      hip_check(hipMemcpyAsync(p->base.u64, p->base.u[0], (size_t)3 * p->shape->geo.S * 16, hipMemcpyDeviceToDevice,
                               stream),
                "fallback iterate to U");
  // a finished stencil-form problem reports u(q): its iterate leaves the mixed domain
  for (Prob* p : fin)
    if (p->form == HZ_SCHEME_STENCIL)
      convert_stencil_state(p->prec == HZ_FP64 ? p->base.u[p->parity & 1] : p->base.u64, *p, false);
  bool copied = false;
  if (prof->on && !fin.empty()) copied = true;  // the synchronisation below lets the conversions' events drain
  // FP64 traces of the problems that finished
  for (Prob* p : fin)
    if (p->base.trace && p->prec == HZ_FP64) {
      const int ntr = std::min(p->iters + 1, kTraceCap);
      p->trace.assign((size_t)ntr * 7, 0.0);
      hip_check(hipMemcpyAsync(p->trace.data(), p->base.trace, p->trace.size() * 8, hipMemcpyDeviceToHost, stream),
                "trace D2H");
      copied = true;
    }
  if (copied) hip_check(hipStreamSynchronize(stream), "sync");
  if (prof->on) prof->drain();
  live.erase(std::remove_if(live.begin(), live.end(), [](Prob* p) { return p->st == PS_DONE; }), live.end());
  return fin;
}

void Engine::advance(Prob* p, const double* s, const double* t_iter) {
  const int k1 = (int)s[ST_K];
  const int flag = (int)s[ST_DONE];
  switch (p->st) {
    case PS_IT64: {
      for (int t = p->k0; t < k1; ++t) p->times.push_back(t_iter[t - p->k0]);
      p->k0 = k1;
      // the device records the first iterate below 1e-6; map it to its event
      const int k6 = (int)s[ST_K1E6];
      if (p->t_1e6 < 0 && k6 >= 0 && k6 < (int)p->times.size()) p->t_1e6 = p->times[k6];
      if (!flag) {
        const int cap_it = p->fixed_iters >= 0 ? p->fixed_iters : p->max_iters;
        if (k1 > cap_it + 1) fail(HZ_EINVAL, "stop rule did not fire");
        return;
      }
      p->code = flag == 1 ? HZ_OK : (flag == 2 ? HZ_NOT_CONVERGED : HZ_EDIVERGED);
      p->iters = (int)s[ST_ITERS];
      p->parity = (int)s[ST_PARITY];
      p->err = s[ST_ERR];
      for (int c = 0; c < 6; ++c) p->mean[c] = s[ST_MEAN + c];
      for (int c = 0; c < 6; ++c) p->Ebar[c] = s[ST_EBAR + c];
      p->t_done = p->iters < (int)p->times.size() ? p->times[p->iters] : p->times.back();
      p->st = PS_DONE;
      return;
    }
    case PS_R0:
    case PS_CORR: {
      p->k0 = k1;
      if (!flag) {
        if (k1 > p->inner_max) fail(HZ_EINVAL, "FP32 stop rule did not fire");
        return;
      }
      p->inner_total += (int)s[ST_ITERS];
      if (p->st == PS_CORR && flag == 3) {
        // a correction that blew up leaves U as the last sweep measured it; the rest of
        // the budget runs as plain FP64 iterations from U
        p->st = PS_FB64;
        p->fb = true;
        p->enter = true;
        return;
      }
      if (p->fixed_iters >= 0 && flag == 3) {  // a fixed count that blew up has nothing to measure
        p->code = HZ_EDIVERGED;
        p->iters = p->inner_total;
        p->st = PS_DONE;
        return;
      }
      // a diverged first estimate keeps U = 0
      p->accum = flag != 3;
      p->st = PS_SWEEP;
      p->enter = true;
      return;
    }
    case PS_SWEEP: {
      if (!flag) fail(HZ_EINVAL, "sweep did not complete");
      const double t = t_iter[0];
      p->rounds += 1;
      p->err = s[ST_ERR];
      for (int c = 0; c < 6; ++c) p->mean[c] = s[ST_MEAN + c];
      p->t_done = t;
      if (p->t_1e6 < 0 && p->err < 1e-6) p->t_1e6 = t;
      bool stop = false;
      if (!(p->err == p->err) || std::isinf(p->err)) {
        p->code = HZ_EDIVERGED;
        stop = true;
      } else if (p->fixed_iters >= 0) {  // a fixed FP32 count: the sweep only measures it
        p->code = HZ_OK;
        stop = true;
      } else if (p->err < p->tol) {
        p->code = HZ_OK;
        stop = true;
      } else if (p->inner_total >= p->max_iters) {
        p->code = HZ_NOT_CONVERGED;
        stop = true;
      } else {
        // the refinement stopped gaining (three sweeps in a row under 10%): the rest of
        // the budget runs as plain FP64 iterations from U
        p->slow = p->err > 0.9 * p->prev_err ? p->slow + 1 : 0;
        if (p->slow >= 3) {
          p->st = PS_FB64;
          p->fb = true;
          p->enter = true;
          return;
        }
      }
      if (stop) {
        p->iters = p->inner_total;
        p->st = PS_DONE;
        return;
      }
      p->prev_err = p->err;
      p->sweep_norm = s[ST_NORM];
      p->st = PS_CORR;
      p->enter = true;
      return;
    }
    case PS_FB64: {
      const int kk0 = p->k0;
      p->k0 = k1;
      const int k6 = (int)s[ST_K1E6];
      if (p->t_1e6 < 0 && k6 >= kk0 && k6 < k1) p->t_1e6 = t_iter[k6 - kk0];
      if (!flag) {
        if (k1 > std::max(0, p->max_iters - p->inner_total) + 1) fail(HZ_EINVAL, "stop rule did not fire");
        return;
      }
      p->code = flag == 1 ? HZ_OK : (flag == 2 ? HZ_NOT_CONVERGED : HZ_EDIVERGED);
      p->iters = p->inner_total + (int)s[ST_ITERS];
      p->parity = (int)s[ST_PARITY];
      p->err = s[ST_ERR];
      for (int c = 0; c < 6; ++c) p->mean[c] = s[ST_MEAN + c];
      for (int c = 0; c < 6; ++c) p->Ebar[c] = s[ST_EBAR + c];
      p->t_done = t_iter[std::max(0, k1 - 1 - kk0)];
      p->st = PS_DONE;
      return;
    }
    default:
      fail(HZ_EINVAL, "problem in an invalid state");
  }
}

void output_fields(Engine& e, Prob& p, double* eps_dev, double* sig_dev) {
  Desc d = p.base;
  d.status = e.d_status + (size_t)p.slot * kStatusLen;
  d.eps_out = eps_dev;
  d.sig_out = sig_dev;
  d.trace = nullptr;
  d.trace_len = 0;
  d.cmode = 0;
  d.fmode = 0;
  d.src = p.prec == HZ_FP64 ? 0 : 1;  // the reported iterate: u_k, or the FP64 anchor U
  double* s = e.h_status + (size_t)p.slot * kStatusLen;
  std::fill(s, s + kStatusLen, 0.0);
  s[ST_K] = p.prec == HZ_FP64 ? p.parity : 0;  // selects the slot the expansion reads
  for (int c = 0; c < 6; ++c) s[ST_EBAR + c] = p.Ebar[c];
  e.h_desc[p.slot] = d;
  e.h_active[0] = p.slot;
  hip_check(hipMemcpyAsync(e.d_desc + p.slot, e.h_desc + p.slot, sizeof(Desc), hipMemcpyHostToDevice, e.stream),
            "desc H2D");
  hip_check(hipMemcpyAsync(e.d_status + (size_t)p.slot * kStatusLen, s, kStatusLen * 8, hipMemcpyHostToDevice,
                           e.stream),
            "status H2D");
  hip_check(hipMemcpyAsync(e.d_active, e.h_active, 4, hipMemcpyHostToDevice, e.stream), "active H2D");
  if (p.form == HZ_SCHEME_STRAIN) pass_front_strain<double>(e, *p.shape, p.tab, e.d_active, 1);
  else pass_front<double>(e, *p.shape, p.tab, e.d_active, 1, p.green);
  int cnt[4]{};
  cnt[(p.base.iso ? KIND_ISO : 0) | (p.base.tau64 ? KIND_EIG : 0)] = 1;
  pass_x<double>(e, *p.shape, p.tab, e.d_active, 1, cnt, 1);
  hip_check(hipStreamSynchronize(e.stream), "sync");
  if (e.prof->on) e.prof->drain();
}

}  // namespace hz
