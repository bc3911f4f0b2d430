// Device helpers shared by the kernels of both realisations of the iteration:
// reductions, Fourier symbols, the constitutive law, and the stages of the fused
// x transforms (C2R split / first pass, last pass / R2C merge).
#pragma once
#include "hz_fft.h"

namespace hz {

// ----------------------------------------------------------------------------
// helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block reduction of NV doubles per thread; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /* LDS, NV*4 */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = wave_sum(v[c]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) red[c * 4 + wid] = v[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = (red[c * 4 + 0] + red[c * 4 + 1]) + (red[c * 4 + 2] + red[c * 4 + 3]);
  }
}

// A problem's status block as the iteration kernels read it: through the scalar cache
// (constant address space), since none of them writes it; the stop-rule kernel, which
// does, reads it through ordinary vector loads.
#define HZ_CONST __attribute__((address_space(4)))
__device__ __forceinline__ const HZ_CONST double* status_ro(const Desc& d) {
  return (const HZ_CONST double*)d.status;
}
__device__ __forceinline__ bool problem_done(const Desc& d) { return status_ro(d)[ST_DONE] != 0.0; }
// ping-pong slot holding the current iterate
__device__ __forceinline__ int cur_slot(const Desc& d) { return ((int)status_ro(d)[ST_K]) & 1; }
// the displacement buffer of slot s (a select, so the pointer stays in scalar registers)
__device__ __forceinline__ void* u_slot(const Desc& d, int s) { return s ? d.u[1] : d.u[0]; }

// Copy a table of n complex values from global memory to LDS: every thread issues all
// of its loads before its first store, so the table costs one memory latency.
template <typename T>
__device__ __forceinline__ void stage_table(cpx<T>* dst, const cpx<T>* __restrict__ src, int n) {
  constexpr int U = 8;
#pragma unroll 1
  for (int i0 = threadIdx.x; i0 < n; i0 += U * kThreads) {
    cpx<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kThreads;
      if (i < n) v[u] = gld(glb(src) + i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kThreads;
      if (i < n) dst[i] = v[u];
    }
  }
}

// D~ (tetrahedron T1) and D~2 (T2) at q from per-axis tables t_a = exp(-i q_a)
__device__ __forceinline__ void symbols(cpx<double> t1, cpx<double> t2, cpx<double> t3,
                                        cpx<double>* d1, cpx<double>* d2) {
  const cpx<double> one = {1.0, 0.0};
  const cpx<double> a = t2 * t3, b = t1 * t3, c = t1 * t2, abc = c * t3;
  d1[0] = scale(one + a - b - c, 0.5);
  d1[1] = scale(one - a + b - c, 0.5);
  d1[2] = scale(one - a - b + c, 0.5);
  const cpx<double> m = {-abc.x, -abc.y};
  d2[0] = scale(m - t1 + t2 + t3, 0.5);
  d2[1] = scale(m + t1 - t2 + t3, 0.5);
  d2[2] = scale(m + t1 + t2 - t3, 0.5);
}

template <typename T>
__device__ __forceinline__ cpx<T> ld(const void* p, long long i) {
  return reinterpret_cast<const cpx<T>*>(p)[i];
}
template <typename T>
__device__ __forceinline__ void st(void* p, long long i, cpx<T> v) {
  reinterpret_cast<cpx<T>*>(p)[i] = v;
}
template <typename T>
__device__ __forceinline__ cpx<double> to64(cpx<T> a) { return {(double)a.x, (double)a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> fr64(cpx<double> a) { return {(T)a.x, (T)a.y}; }


// Blocks are dispatched to the 8 XCDs round-robin (block b -> XCD b % 8).  Map
// them so that each XCD walks a contiguous range of tiles: neighbouring tiles
// that share cache lines then meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// coefficients of D~ = a1 + t3 b1 and D~2 = a2 + t3 b2 at (h1, h2)
__device__ __forceinline__ void affine_symbols(cpx<double> t1, cpx<double> t2, cpx<double>* a1, cpx<double>* b1,
                                               cpx<double>* a2, cpx<double>* b2) {
  const cpx<double> one = {1.0, 0.0};
  const cpx<double> t12 = t1 * t2;
  const cpx<double> P = scale(one - t12, 0.5), Q = scale(t2 - t1, 0.5);
  const cpx<double> S = scale(one + t12, 0.5), R = scale(t1 + t2, 0.5);
  const cpx<double> mQ = {-Q.x, -Q.y}, mR = {-R.x, -R.y}, mS = {-S.x, -S.y};
  a1[0] = P; a1[1] = P; a1[2] = S;
  b1[0] = Q; b1[1] = mQ; b1[2] = mR;
  a2[0] = Q; a2[1] = mQ; a2[2] = R;
  b2[0] = P; b2[1] = P; b2[2] = mS;
}

// The rotated comparison operator (eq. Dq_rotated) is the mean of the two tetrahedral
// gradients, with the same half-voxel phase: D~rot = (D~ + D~2)/2 for both strain
// fields.  Applied to symbol or affine coefficients of T1 (a) and T2 (b) in place.
__device__ __forceinline__ void rotated_mean(cpx<double>* a, cpx<double>* b) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a[c] = scale(a[c] + b[c], 0.5);
    b[c] = a[c];
  }
}

// A wave-uniform value moved into scalar registers.
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// What the constitutive law of one problem needs besides the stiffness: the mean
// strain of the current iterate (status block, in kernel precision) and the
// per-phase eigenstress table.
template <typename T>
struct Mean {
  T Eb[6];
  const HZ_GLB T* tau;  // [n_phases][8] lambda_p:eps0_p, or null
};
template <typename T>
__device__ __forceinline__ Mean<T> mean_state(const Desc& d) {
  Mean<T> m;
#pragma unroll
  for (int c = 0; c < 6; ++c) m.Eb[c] = (T)status_ro(d)[ST_EBAR + c];
  const T* t;
  if constexpr (sizeof(T) == 8) t = reinterpret_cast<const T*>(d.tau64);
  else t = reinterpret_cast<const T*>(d.tau32);
  m.tau = glb(t);
  return m;
}
// sigma -= lambda_p:eps0_p (eq. linear_elasticity with an eigenstrain); EIG: the
// problem has eigenstrains (its table pointer is not null)
template <bool EIG, typename T>
__device__ __forceinline__ void eigenstress(const Mean<T>& M, int ph, T (&s)[6]) {
  if constexpr (EIG) {
    const HZ_GLB cpx<T>* t = reinterpret_cast<const HZ_GLB cpx<T>*>(M.tau + ph * 8);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const cpx<T> v = gld(t + i);
      s[2 * i] -= v.x;
      s[2 * i + 1] -= v.y;
    }
  }
}

// sigma = C:(Ebar + deps) - lambda:eps0 in tensor comps (11,22,33,23,13,12); C as an
// engineering Voigt matrix stored as its upper triangle (21 of 24 slots) row by row
template <bool EIG, typename T>
__device__ __forceinline__ void constitutive(const HZ_GLB T* __restrict__ Cp, const Mean<T>& M, int ph,
                                             const T (&de)[6], T (&s)[6]) {
  T g[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) g[c] = M.Eb[c] + de[c];
  g[3] *= (T)2; g[4] *= (T)2; g[5] *= (T)2;  // engineering shears
  T Cu[24];
#pragma unroll
  for (int i = 0; i < 24; i += 2) {
    const cpx<T> v = gld(reinterpret_cast<const HZ_GLB cpx<T>*>(Cp) + i / 2);
    Cu[i] = v.x;
    Cu[i + 1] = v.y;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T acc = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int a = i < j ? i : j, b = i < j ? j : i;
      acc += Cu[a * 6 - a * (a - 1) / 2 + (b - a)] * g[j];
    }
    s[i] = acc;
  }
  eigenstress<EIG>(M, ph, s);
}

// the same law for the two tetrahedra of one voxel (one phase): the stiffness entries
// are loaded once for both and each is used as it arrives (C_ab enters sigma_a and, off
// the diagonal, sigma_b), so only a few of them are live at a time
// ld(i) returns the i-th complex pair of the phase's 24-slot row (from HBM or from a
// copy of the table in LDS)
template <bool EIG, typename T, class LD>
__device__ __forceinline__ void constitutive_pair_ld(LD ld, const Mean<T>& M, int ph, const T (&de0)[6],
                                                     const T (&de1)[6], T (&s0)[6], T (&s1)[6]) {
  T g0[6], g1[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    g0[c] = M.Eb[c] + de0[c];
    g1[c] = M.Eb[c] + de1[c];
    s0[c] = 0;
    s1[c] = 0;
  }
#pragma unroll
  for (int c = 3; c < 6; ++c) {  // engineering shears
    g0[c] *= (T)2;
    g1[c] *= (T)2;
  }
  // packed entry k of the upper triangle is (a, b): row a = 0 holds k = 0..5, a = 1
  // k = 6..10, a = 2 k = 11..14, a = 3 k = 15..17, a = 4 k = 18..19, a = 5 k = 20
#pragma unroll
  for (int k2 = 0; k2 < 21; k2 += 2) {
    const cpx<T> v = ld(k2 / 2);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = k2 + h;
      if (k > 20) break;
      const int a = k < 6 ? 0 : k < 11 ? 1 : k < 15 ? 2 : k < 18 ? 3 : k < 20 ? 4 : 5;
      const int b = a + k - (a * 6 - a * (a - 1) / 2);
      const T c = h ? v.y : v.x;
      s0[a] += c * g0[b];
      s1[a] += c * g1[b];
      if (a != b) {
        s0[b] += c * g0[a];
        s1[b] += c * g1[a];
      }
    }
  }
  eigenstress<EIG>(M, ph, s0);
  eigenstress<EIG>(M, ph, s1);
}
template <bool EIG, typename T>
__device__ __forceinline__ void constitutive_pair(const HZ_GLB T* __restrict__ Cp, const Mean<T>& M, int ph,
                                                  const T (&de0)[6], const T (&de1)[6], T (&s0)[6], T (&s1)[6]) {
  const HZ_GLB cpx<T>* row = reinterpret_cast<const HZ_GLB cpx<T>*>(Cp);
  constitutive_pair_ld<EIG, T>([&](int i) { return gld(row + i); }, M, ph, de0, de1, s0, s1);
}

// isotropic phase: sigma = lambda tr(eps) I + 2 mu eps - lambda:eps0
template <bool EIG, typename T>
__device__ __forceinline__ void constitutive_iso(T lam, T mu, const Mean<T>& M, int ph, const T (&de)[6],
                                                 T (&s)[6]) {
  T e[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = M.Eb[c] + de[c];
  const T lt = lam * (e[0] + e[1] + e[2]), m2 = (T)2 * mu;
  s[0] = lt + m2 * e[0];
  s[1] = lt + m2 * e[1];
  s[2] = lt + m2 * e[2];
  s[3] = m2 * e[3];
  s[4] = m2 * e[4];
  s[5] = m2 * e[5];
  eigenstress<EIG>(M, ph, s);
}

// ----------------------------------------------------------------------------
// P3, fused form (every iteration wherever M = N1/2 factors as below; the
// output pass, which writes real-space fields, uses the unfused k_xpass).
// The length-M transforms use radices r0 .. r_{s-1} (inverse) and the reverse
// order (forward), with r0 in {16, 8, 4, 2} and r_{s-1} in {5, 4, 3, 2}:
//  * butterfly j of the first inverse pass reads Z at j + m LR (LR = M/r0); the
//    C2R split partners M - (j + m LR) are the inputs of butterfly LR - j, so one
//    thread takes both butterflies and every half-spectrum value is loaded once;
//  * the last inverse pass writes positions j + m LRm, which are exactly the
//    inputs of butterfly j of the first forward pass (same radix): the
//    constitutive law runs in registers between the two, on all 6 components;
//  * the last forward pass writes Z at j + m LR, and the R2C merge pairs it with
//    butterfly LR - j again, so the merge feeds the stores.
// For s = 2 each element goes through LDS twice (write + read) per direction.
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cpx<T> c2r_split(cpx<T> a, cpx<T> b, cpx<T> twk) {
  // Z[k] = X[k] + conj(X[M-k]) + i w^k (X[k] - conj(X[M-k])),  w^k = conj(exp(-2 pi i k / N1))
  return (a + conjg(b)) + mul_i(conjg(twk) * (a - conjg(b)));
}

template <typename T>
__device__ __forceinline__ cpx<T> r2c_merge(cpx<T> a, cpx<T> b, cpx<T> twk, T hs) {
  // X[k] = (Z[k] + conj(Z[M-k]) - i w^-k (Z[k] - conj(Z[M-k]))) / 2, times 1/N (eq. FT)
  return scale((a + conjg(b)) - mul_i(twk * (a - conjg(b))), hs);
}

// load + split + first inverse radix pass; writes line positions j*R + m.
// Butterfly j takes h1 = j + m LR and its split partners h1 = LR - j + m LR (the
// Nyquist value h1 = M for j = 0); both sets are loaded before any arithmetic, and for
// small radices a thread issues the loads of U butterflies at once, so several HBM
// round trips overlap.
template <typename T, int R, int NC = 6>
__device__ __forceinline__ void xf_load(const XGeo& xg, const HZ_GLB cpx<T>* __restrict__ src, cpx<T>* buf,
                                        const cpx<T>* twl) {
  constexpr int U = R <= 4 ? 2 : 1;
  const int M = xg.M, LR = M / R, TY = xg.TY, nI = LR / 2 + 1;
  const int n = NC * nI * TY;
  const int hs = xg.N3 * xg.N2;  // stride between h1 planes
#pragma unroll 1
  for (int w0 = threadIdx.x; w0 < n; w0 += U * kThreads) {
    cpx<T> x[U][R], y[U][R];
    int jj[U], rr[U], cc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int w = w0 + u * kThreads;
      jj[u] = -1;
      if (w < n) {
        const int q = fdiv(w, xg.rTY), r = w - q * TY;
        const int c = fdiv(q, xg.rNI), it = q - c * nI;
        const HZ_GLB cpx<T>* s = src + c * xg.S + r;
        jj[u] = it;
        rr[u] = r;
        cc[u] = c;
#pragma unroll
        for (int m = 0; m < R; ++m) x[u][m] = gld(s + (it + m * LR) * hs);
        // partners: h1 = LR - it + m LR <= M (for it = 0, y[R-1] is the Nyquist value)
#pragma unroll
        for (int m = 0; m < R; ++m) y[u][m] = gld(s + (LR - it + m * LR) * hs);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = jj[u];
      if (j < 0) continue;
      const int j2 = LR - j;
      cpx<T>* line = buf + (cc[u] * TY + rr[u]) * xg.H1p;
      if (j == 0) {
        // positions m LR; partner of m >= 1 is R - m, partner of 0 is the Nyquist value X[M]
        cpx<T> z[R];
        z[0] = c2r_split(x[u][0], y[u][R - 1], twl[0]);
#pragma unroll
        for (int m = 1; m < R; ++m) z[m] = c2r_split(x[u][m], x[u][R - m], twl[m * LR]);
        Dft<T, R, true>::run(z);
#pragma unroll
        for (int m = 0; m < R; ++m) line[m] = z[m];
      } else if (j2 == j) {
        // butterfly LR/2 is its own partner: m <-> R-1-m
        cpx<T>* xv = x[u];
#pragma unroll
        for (int m = 0; m < R / 2; ++m) {
          const cpx<T> a = xv[m], b = xv[R - 1 - m];
          xv[m] = c2r_split(a, b, twl[j + m * LR]);
          xv[R - 1 - m] = c2r_split(b, a, twl[j + (R - 1 - m) * LR]);
        }
        if (R & 1) xv[R / 2] = c2r_split(xv[R / 2], xv[R / 2], twl[j + (R / 2) * LR]);
        Dft<T, R, true>::run(x[u]);
#pragma unroll
        for (int m = 0; m < R; ++m) line[j * R + m] = x[u][m];
      } else {
#pragma unroll
        for (int m = 0; m < R; ++m) {
          const cpx<T> a = x[u][m], b = y[u][R - 1 - m];
          x[u][m] = c2r_split(a, b, twl[j + m * LR]);
          y[u][R - 1 - m] = c2r_split(b, a, twl[j2 + (R - 1 - m) * LR]);
        }
        Dft<T, R, true>::run(x[u]);
        Dft<T, R, true>::run(y[u]);
#pragma unroll
        for (int m = 0; m < R; ++m) {
          line[j * R + m] = x[u][m];
          line[j2 * R + m] = y[u][m];
        }
      }
    }
  }
}

// last inverse pass -> constitutive law on the voxel pairs -> first forward pass.
// Rounds of whole lines, so a round never reads what an earlier round wrote.
template <typename T, bool ISO, bool EIG, int R>
__device__ __forceinline__ void xf_middle(const Desc& d, const XGeo& xg, cpx<T>* buf, const cpx<T>* twl,
                                          const HZ_GLB uint16_t* __restrict__ ph, double (&acc)[6]) {
  const int M = xg.M, LR = M / R, TY = xg.TY, H1p = xg.H1p;
  const int n = TY * LR;
  const int per = (kThreads / LR) * LR;
  const HZ_GLB T* C = glb(sizeof(T) == 8 ? reinterpret_cast<const T*>(d.C64) : reinterpret_cast<const T*>(d.C32));
  const Mean<T> Mn = mean_state<T>(d);
#pragma unroll 1
  for (int w0 = 0; w0 < n; w0 += per) {
    const int w = w0 + (int)threadIdx.x;
    const bool act = (int)threadIdx.x < per && w < n;
    cpx<T> z[6][R];
    int r = 0, j = 0;
    if (act) {
      r = fdiv(w, xg.rLRm);
      j = w - r * LR;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const cpx<T>* line = buf + (c * TY + r) * H1p + j;
#pragma unroll
        for (int m = 0; m < R; ++m) z[c][m] = line[m * LR];
      }
      // twiddles of the last inverse pass: exp(+2 pi i m j / M) = conj(tw[2 m j])
#pragma unroll
      for (int m = 1; m < R; ++m) {
        const cpx<T> t = conjg(twl[2 * m * j]);
#pragma unroll
        for (int c = 0; c < 6; ++c) z[c][m] = z[c][m] * t;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) Dft<T, R, true>::run(z[c]);
      // z[c][m] = eps(2n) + i eps(2n+1), n = j + m LR
      const HZ_GLB uint32_t* ph2 = reinterpret_cast<const HZ_GLB uint32_t*>(ph + (long long)r * xg.N1);
#pragma unroll
      for (int m = 0; m < R; ++m) {
        __builtin_amdgcn_sched_barrier(0);  // keeps the stiffness loads of one position at a time
        const int nn = j + m * LR;
        const uint32_t pp = ph2[nn];
        const int pa = (int)(pp & 0xffffu), pb = (int)(pp >> 16);
        T ea[6], eb[6], sa[6], sb[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          ea[c] = z[c][m].x;
          eb[c] = z[c][m].y;
        }
        if (ISO) {
          const cpx<T> la = gld(reinterpret_cast<const HZ_GLB cpx<T>*>(C) + pa), lb = gld(reinterpret_cast<const HZ_GLB cpx<T>*>(C) + pb);
          constitutive_iso<EIG, T>(la.x, la.y, Mn, pa, ea, sa);
          constitutive_iso<EIG, T>(lb.x, lb.y, Mn, pb, eb, sb);
        } else {
          constitutive<EIG, T>(C + pa * 24, Mn, pa, ea, sa);
          __builtin_amdgcn_sched_barrier(0);  // one stiffness row set live at a time
          constitutive<EIG, T>(C + pb * 24, Mn, pb, eb, sb);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          acc[c] += 0.5 * ((double)sa[c] + (double)sb[c]);
          z[c][m] = cpx<T>{sa[c], sb[c]};
        }
      }
      // first forward pass (no twiddles): outputs at j*R + m
#pragma unroll
      for (int c = 0; c < 6; ++c) Dft<T, R, false>::run(z[c]);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        cpx<T>* line = buf + (c * TY + r) * H1p + j * R;
#pragma unroll
        for (int m = 0; m < R; ++m) line[m] = z[c][m];
      }
    }
    __syncthreads();
  }
}

// last forward pass + R2C merge + stores (with the 1/N of eq. FT)
template <typename T, int R, int NC = 6>
__device__ __forceinline__ void xf_store(const XGeo& xg, HZ_GLB cpx<T>* __restrict__ dst, const cpx<T>* buf,
                                         const cpx<T>* twl) {
  const int M = xg.M, LR = M / R, TY = xg.TY, nI = LR / 2 + 1;
  const int n = NC * nI * TY;
  const int hs = xg.N3 * xg.N2;
  const T hN = (T)(0.5 * xg.invN), sN = (T)xg.invN;
#pragma unroll 1
  for (int w = threadIdx.x; w < n; w += kThreads) {
    const int q = fdiv(w, xg.rTY), r = w - q * TY;
    const int c = fdiv(q, xg.rNI), it = q - c * nI;
    const cpx<T>* line = buf + (c * TY + r) * xg.H1p;
    HZ_GLB cpx<T>* o = dst + c * xg.S + r;
    const int j = it, j2 = LR - it;
    cpx<T> x[R];
#pragma unroll
    for (int m = 0; m < R; ++m) x[m] = line[j + m * LR];
    if (it != 0) {
#pragma unroll
      for (int m = 1; m < R; ++m) x[m] = x[m] * twl[2 * m * j];
    }
    Dft<T, R, false>::run(x);
    if (it == 0) {
      gst(o, cpx<T>{(x[0].x + x[0].y) * sN, (T)0});
      gst(o + M * hs, cpx<T>{(x[0].x - x[0].y) * sN, (T)0});
#pragma unroll
      for (int m = 1; m < R; ++m) gst(o + m * LR * hs, r2c_merge(x[m], x[R - m], twl[m * LR], hN));
    } else if (j2 == j) {
#pragma unroll
      for (int m = 0; m < R; ++m) gst(o + (j + m * LR) * hs, r2c_merge(x[m], x[R - 1 - m], twl[j + m * LR], hN));
    } else {
      cpx<T> y[R];
#pragma unroll
      for (int m = 0; m < R; ++m) y[m] = line[j2 + m * LR];
#pragma unroll
      for (int m = 1; m < R; ++m) y[m] = y[m] * twl[2 * m * j2];
      Dft<T, R, false>::run(y);
#pragma unroll
      for (int m = 0; m < R; ++m) {
        gst(o + (j + m * LR) * hs, r2c_merge(x[m], y[R - 1 - m], twl[j + m * LR], hN));
        gst(o + (j2 + m * LR) * hs, r2c_merge(y[m], x[R - 1 - m], twl[j2 + m * LR], hN));
      }
    }
  }
}

}  // namespace hz
