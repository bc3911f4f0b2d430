// HIP kernels (gfx950) of one iteration of the tetrahedral-stencil basic scheme.
//
// Spectra are stored [comp][h1][h3][h2] (h1 in [0, N1/2], h2 fastest).  Iteration
// (Algorithm 1, Sec. 2.6):
//   k_zexp      u(q) (3 comps) -> inverse z transform of the 3 displacement comps,
//               then the 12 strain comps eps^T1 = D~ (x)_s u, eps^T2 = D~2 (x)_s u
//               formed in the mixed (h1, h2, l3) domain
//   k_yline     inverse y (12 comps)
//   k_xpass     per (l3, l2-tile): C2R along x, sigma = C(phase):(Ebar + eps), R2C along x,
//               FP64 partial sums of <sigma>
//   k_yline     forward y
//   k_zcon      r = sigma^T1.conj(D~) + sigma^T2.conj(D~2) formed in the mixed domain,
//               forward z transform of its 3 comps, Omega(q) in FP64, u update,
//               FP64 partial sums of w |r/2|^2
//   k_finalize  fixed-order sums, eps_k = L2/||<sigma>||, device-side stop rule
//
// Phase convention.  With integer-indexed displacement corners the state is
// u~(q) = exp(i q.(1/2,1/2,1/2)) u(q).  Then D~(q) = D(q) exp(-i q.(1/2,1/2,1/2))
// is the corner sum  sum_{o in T1} v(o) exp(i q.o)  over o in {0,-1}^3 with
// 8 v1 v2 v3 = +1, D~2 = -conj(D) exp(-i q.(1/2,...)) the same sum over the
// other four corners (eqs. Dq, DA1-DA2), both periodic in h, and the update
// u~ <- u~ - Omega r~ is the paper's update multiplied by the same phase
// (Omega is real).  Outputs in real space do not see the phase at all.
//
// Why the z transforms run on 3 fields.  With t_a = exp(-i q_a) every component
// of D~ and D~2 is affine in t3:  D~ = alpha + t3 beta, with alpha, beta functions
// of (h1, h2) only:
//   D~  = 1/2 (P, P, S)  + t3 1/2 (Q, -Q, -R)      P = 1 - t1 t2, Q = t2 - t1,
//   D~2 = 1/2 (Q, -Q, R) + t3 1/2 (P, P, -S)       S = 1 + t1 t2, R = t1 + t2.
// Multiplying by t3 is a shift by one voxel along l3 after the inverse z
// transform, and multiplying by conj(t3) a shift by -1 before the forward one.
// So the 12 strain spectra are 2-tap combinations of the z-transformed 3
// displacement components, and the residual's 3 components are 2-tap
// combinations of the 12 stresses taken before the forward z transform.
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

__device__ __forceinline__ bool problem_done(const Desc& d) { return d.status[ST_DONE] != 0.0; }
// ping-pong slot holding the current iterate
__device__ __forceinline__ int cur_slot(const Desc& d) { return ((int)d.status[ST_K]) & 1; }

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

// ----------------------------------------------------------------------------
// P1: inverse z transform of u (3 comps) and the 12 strain spectra
// (eqs. desp_T1_dep_Q, desp_T2_dep_Q) as 2-tap combinations along l3.
// Tile: TX adjacent h2 columns of one h1 plane.  LDS: 3*TX lines x N3, then twiddles.
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zexp(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                   ZGeo zg, const Plan* __restrict__ plan3, const cpx<T>* __restrict__ tw3T,
                                                   const cpx<double>* __restrict__ tw1,
                                                   const cpx<double>* __restrict__ tw2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int TX = zg.TX, N2 = zg.N2, N3 = zg.N3;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int h1 = tile / zg.tiles;
  const int h2_0 = (tile % zg.tiles) * TX;
  const int lines = 3 * TX;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = buf + lines * N3;
  for (int i = threadIdx.x; i < N3; i += kThreads) twl[i] = tw3T[i];
  const long long plane = (long long)h1 * N3 * N2 + h2_0;
  const LdsAcc<T> lds{buf, 1, lines};
  const void* usrc = d.src == 1 ? d.u64 : d.u[cur_slot(d)];
  const GblAcc<T> src{glb(reinterpret_cast<cpx<T>*>(const_cast<void*>(usrc))) + plane, (int)zg.S, TX, 1, N2};
  fft_lines<T, emax<T>(), true>(*plan3, lines, zg.rLines, false, twl, 1, lds, src, lds);
  __syncthreads();
  HZ_GLB cpx<T>* out = glb(reinterpret_cast<cpx<T>*>(d.spec)) + plane;
  const cpx<double> t1 = tw1[h1];
  for (int e = threadIdx.x; e < TX * N3; e += kThreads) {
    const int l3 = fdiv(e, zg.rTX), col = e - l3 * TX;
    const int lm = l3 == 0 ? N3 - 1 : l3 - 1;
    cpx<double> a1[3], b1[3], a2[3], b2[3];
    affine_symbols(t1, tw2[h2_0 + col], a1, b1, a2, b2);
    cpx<double> U[3], Um[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      U[c] = to64(lds.get(c * TX + col, l3));
      Um[c] = to64(lds.get(c * TX + col, lm));
    }
    const long long o = (long long)l3 * N2 + col;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const cpx<double>* A = t == 0 ? a1 : a2;
      const cpx<double>* B = t == 0 ? b1 : b2;
      // G[i][j] = (D_i u_j) in the mixed domain = A_i U_j + B_i U_j(l3-1)
      cpx<double> G[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) G[i][j] = A[i] * U[j] + B[i] * Um[j];
      cpx<double> e6[6];
      e6[0] = G[0][0];
      e6[1] = G[1][1];
      e6[2] = G[2][2];
      e6[3] = scale(G[1][2] + G[2][1], 0.5);
      e6[4] = scale(G[0][2] + G[2][0], 0.5);
      e6[5] = scale(G[0][1] + G[1][0], 0.5);
#pragma unroll
      for (int c = 0; c < 6; ++c) gst(out + (t * 6 + c) * zg.S + o, fr64<T>(e6[c]));
    }
  }
}

// ----------------------------------------------------------------------------
// y pass: TX contiguous rows of length N2; first radix pass straight from HBM,
// last radix pass straight to HBM, twiddles in LDS.
// ----------------------------------------------------------------------------
template <typename T, bool INV>
__global__ __launch_bounds__(kThreads) void k_yline(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                    YGeo yg, const Plan* __restrict__ plan2, const cpx<T>* __restrict__ tw2T) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int N2 = yg.N2;
  const long long t0 = (long long)blockIdx.x * yg.TX;
  const int lines = (int)((yg.nlines - t0) < yg.TX ? (yg.nlines - t0) : yg.TX);
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = buf + yg.TX * N2;
  for (int i = threadIdx.x; i < N2; i += kThreads) twl[i] = tw2T[i];
  const LdsAcc<T> lds{buf, N2, 1};
  const GblAcc<T> g{glb(reinterpret_cast<cpx<T>*>(d.spec)) + yg.off + t0 * N2, N2, 1, 0, 1};
  fft_lines<T, emax<T>(), INV>(*plan2, lines, 0.f, true, twl, 1, lds, g, g);
}

// ----------------------------------------------------------------------------
// P3: fused x pass.  One block owns TY consecutive rows l2 at one l3 and handles
// T1 then T2: load 6 half-spectrum rows (h1 = 0..N1/2) per row, C2R of length N1
// as a complex transform of length M = N1/2, constitutive law per voxel,
// R2C back (with the 1/N of eq. FT), store.  FP64 partials of <sigma>.
// ----------------------------------------------------------------------------
// sigma = C:(Ebar + deps) in tensor comps (11,22,33,23,13,12); C as an engineering
// Voigt matrix stored as its upper triangle (21 of 24 slots) row by row
template <typename T>
__device__ __forceinline__ void constitutive(const HZ_GLB T* __restrict__ Cp, const double* Eb, const T (&de)[6],
                                             T (&s)[6]) {
  T g[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) g[c] = (T)Eb[c] + de[c];
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
}

// isotropic phase: sigma = lambda tr(eps) I + 2 mu eps
template <typename T>
__device__ __forceinline__ void constitutive_iso(T lam, T mu, const double* Eb, const T (&de)[6], T (&s)[6]) {
  T e[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = (T)Eb[c] + de[c];
  const T lt = lam * (e[0] + e[1] + e[2]), m2 = (T)2 * mu;
  s[0] = lt + m2 * e[0];
  s[1] = lt + m2 * e[1];
  s[2] = lt + m2 * e[2];
  s[3] = m2 * e[3];
  s[4] = m2 * e[4];
  s[5] = m2 * e[5];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_xpass(const Desc* __restrict__ descs,
                                                    const int* __restrict__ active, XGeo xg,
                                                    const Plan* __restrict__ planM, const cpx<T>* __restrict__ twN1) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[6 * 4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int tiles2 = xg.N2 / xg.TY;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  // one block per (row tile, tetrahedron): half 0 = T1 comps 0..5, half 1 = T2 comps 6..11
  const int half = xg.half >= 0 ? xg.half : (tile & 1);
  const int rt = xg.half >= 0 ? tile : (tile >> 1);
  const int l3 = rt / tiles2;
  const int l2_0 = (rt % tiles2) * xg.TY;
  const int TY = xg.TY, H1p = xg.H1p, M = xg.M;
  const long long N3N2 = (long long)xg.N3 * xg.N2;
  const long long rowoff = (long long)l3 * xg.N2 + l2_0;
  const HZ_GLB T* C = glb(sizeof(T) == 8 ? reinterpret_cast<const T*>(d.C64) : reinterpret_cast<const T*>(d.C32));
  const HZ_GLB uint16_t* ph = glb(d.phase) + ((long long)l3 * xg.N2 + l2_0) * xg.N1;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);  // 6*TY lines of M (pitch H1p)
  cpx<T>* twl = buf + 6 * TY * H1p;
  for (int i = threadIdx.x; i < xg.N1; i += kThreads) twl[i] = twN1[i];
  const int kh = M / 2 + 1;             // (k, M-k) pairs per line, k = 0..M/2
  const int npair = 6 * kh * TY;
  const LdsAcc<T> lds{buf, H1p, 1};
  const HZ_GLB cpx<T>* src = glb(reinterpret_cast<const cpx<T>*>(d.spec)) + (long long)half * 6 * xg.S + rowoff;
  HZ_GLB cpx<T>* dst = glb(reinterpret_cast<cpx<T>*>(d.spec)) + (long long)half * 6 * xg.S + rowoff;

  // 1) load half-spectrum pairs X[k], X[M-k] of each row and apply the C2R split
  //    Z[k] = X[k] + conj(X[M-k]) + i w^k (X[k] - conj(X[M-k])),  w = exp(2 pi i / N1)
  constexpr int NPT = 4;
#pragma unroll 1
  for (int p0 = 0; p0 < npair; p0 += NPT * kThreads) {
    cpx<T> xa[NPT], xb[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int p = min(p0 + (int)threadIdx.x + i * kThreads, npair - 1);
      const int q = fdiv(p, xg.rTY), r = p - q * TY;
      const int c = fdiv(q, xg.rKH), kk = q - c * kh;
      const HZ_GLB cpx<T>* s = src + c * xg.S + r;
      xa[i] = gld(s + kk * N3N2);
      xb[i] = gld(s + (M - kk) * N3N2);
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int p = p0 + threadIdx.x + i * kThreads;
      if (p < npair) {
        const int q = fdiv(p, xg.rTY), r = p - q * TY;
        const int c = fdiv(q, xg.rKH), kk = q - c * kh;
        cpx<T>* Z = buf + (c * TY + r) * H1p;
        const cpx<T> a = xa[i], b = xb[i];
        if (kk == 0) {
          Z[0] = (a + conjg(b)) + mul_i(a - conjg(b));
        } else {
          const int k2 = M - kk;
          Z[kk] = (a + conjg(b)) + mul_i(conjg(twN1[kk]) * (a - conjg(b)));
          if (k2 != kk) Z[k2] = (b + conjg(a)) + mul_i(conjg(twN1[k2]) * (b - conjg(a)));
        }
      }
    }
  }
  __syncthreads();
  // 2) complex inverse transforms of length M: z[n] = x[2n] + i x[2n+1]
  fft_lines<T, emax<T>(), true>(*planM, 6 * TY, 0.f, true, twl, 2, lds, lds, lds);
  __syncthreads();
  // 3) constitutive law on voxel pairs (2n, 2n+1): real / imaginary parts
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int it = threadIdx.x; it < TY * M; it += kThreads) {
    const int r = fdiv(it, xg.rM), n = it - r * M;
    T ea[6], eb[6], sa[6], sb[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const cpx<T> z = buf[(c * TY + r) * H1p + n];
      ea[c] = z.x;
      eb[c] = z.y;
    }
    const int pa = ph[r * xg.N1 + 2 * n], pb = ph[r * xg.N1 + 2 * n + 1];
    if (d.iso) {
      const cpx<T> la = gld(reinterpret_cast<const HZ_GLB cpx<T>*>(C) + pa), lb = gld(reinterpret_cast<const HZ_GLB cpx<T>*>(C) + pb);
      constitutive_iso<T>(la.x, la.y, d.Ebar, ea, sa);
      constitutive_iso<T>(lb.x, lb.y, d.Ebar, eb, sb);
    } else {
      constitutive<T>(C + pa * 24, d.Ebar, ea, sa);
      constitutive<T>(C + pb * 24, d.Ebar, eb, sb);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      acc[c] += 0.5 * ((double)sa[c] + (double)sb[c]);
      buf[(c * TY + r) * H1p + n] = cpx<T>{sa[c], sb[c]};
    }
    if (xg.fields) {
      const long long vox = ((long long)l3 * xg.N2 + l2_0 + r) * xg.N1 + 2 * n;
      const long long Nn = (long long)xg.N1 * xg.N2 * xg.N3;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double e0 = 0.5 * ((double)d.Ebar[c] + (double)ea[c]);
        const double e1 = 0.5 * ((double)d.Ebar[c] + (double)eb[c]);
        const double s0 = 0.5 * (double)sa[c], s1 = 0.5 * (double)sb[c];
        if (half == 0) {
          d.eps_out[c * Nn + vox] = e0; d.eps_out[c * Nn + vox + 1] = e1;
          d.sig_out[c * Nn + vox] = s0; d.sig_out[c * Nn + vox + 1] = s1;
        } else {
          d.eps_out[c * Nn + vox] += e0; d.eps_out[c * Nn + vox + 1] += e1;
          d.sig_out[c * Nn + vox] += s0; d.sig_out[c * Nn + vox + 1] += s1;
        }
      }
    }
  }
  __syncthreads();
  // 4) forward transforms of length M
  fft_lines<T, emax<T>(), false>(*planM, 6 * TY, 0.f, true, twl, 2, lds, lds, lds);
  __syncthreads();
  // 5) R2C merge straight to HBM (with the 1/N of eq. FT):
  //    X[k] = (A - i w^-k B)/2, A = Z[k] + conj(Z[M-k]), B = Z[k] - conj(Z[M-k]);
  //    X[0] = Re Z0 + Im Z0, X[M] = Re Z0 - Im Z0
  const T hs = (T)(0.5 * xg.invN), sN = (T)xg.invN;
  for (int p = threadIdx.x; p < npair; p += kThreads) {
    const int q = fdiv(p, xg.rTY), r = p - q * TY;
    const int c = fdiv(q, xg.rKH), kk = q - c * kh;
    const cpx<T>* Z = buf + (c * TY + r) * H1p;
    HZ_GLB cpx<T>* o = dst + c * xg.S + r;
    if (kk == 0) {
      const cpx<T> z = Z[0];
      gst(o, cpx<T>{(z.x + z.y) * sN, (T)0});
      gst(o + M * N3N2, cpx<T>{(z.x - z.y) * sN, (T)0});
    } else {
      const int k2 = M - kk;
      const cpx<T> a = Z[kk], b = Z[k2];
      gst(o + kk * N3N2, scale((a + conjg(b)) - mul_i(twN1[kk] * (a - conjg(b))), hs));
      if (k2 != kk) gst(o + k2 * N3N2, scale((b + conjg(a)) - mul_i(twN1[k2] * (b - conjg(a))), hs));
    }
  }
  block_sum<6>(acc, red);
  if (threadIdx.x == 0) {
    double* pp = d.part_sig + (long long)(xg.half >= 0 ? 2 * tile + half : tile) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) pp[c] = acc[c];
  }
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

// load + split + first inverse radix pass; writes line positions j*R + m
template <typename T, int R, int NC = 6>
__device__ __forceinline__ void xf_load(const XGeo& xg, const HZ_GLB cpx<T>* __restrict__ src, cpx<T>* buf,
                                        const cpx<T>* twl) {
  const int M = xg.M, LR = M / R, TY = xg.TY, nI = LR / 2 + 1;
  const int n = NC * nI * TY;
  const int hs = xg.N3 * xg.N2;  // stride between h1 planes
#pragma unroll 1
  for (int w = threadIdx.x; w < n; w += kThreads) {
    const int q = fdiv(w, xg.rTY), r = w - q * TY;
    const int c = fdiv(q, xg.rNI), it = q - c * nI;
    const HZ_GLB cpx<T>* s = src + c * xg.S + r;
    cpx<T>* line = buf + (c * TY + r) * xg.H1p;
    const int j = it, j2 = LR - it;
    cpx<T> x[R];
#pragma unroll
    for (int m = 0; m < R; ++m) x[m] = gld(s + (j + m * LR) * hs);
    if (it == 0) {
      // positions m LR; partner of m >= 1 is R - m, partner of 0 is the Nyquist value X[M]
      const cpx<T> xM = gld(s + M * hs);
      cpx<T> z[R];
      z[0] = c2r_split(x[0], xM, twl[0]);
#pragma unroll
      for (int m = 1; m < R; ++m) z[m] = c2r_split(x[m], x[R - m], twl[m * LR]);
      Dft<T, R, true>::run(z);
#pragma unroll
      for (int m = 0; m < R; ++m) line[m] = z[m];
    } else if (j2 == j) {
      // butterfly LR/2 is its own partner: m <-> R-1-m
#pragma unroll
      for (int m = 0; m < R / 2; ++m) {
        const cpx<T> a = x[m], b = x[R - 1 - m];
        x[m] = c2r_split(a, b, twl[j + m * LR]);
        x[R - 1 - m] = c2r_split(b, a, twl[j + (R - 1 - m) * LR]);
      }
      if (R & 1) x[R / 2] = c2r_split(x[R / 2], x[R / 2], twl[j + (R / 2) * LR]);
      Dft<T, R, true>::run(x);
#pragma unroll
      for (int m = 0; m < R; ++m) line[j * R + m] = x[m];
    } else {
      cpx<T> y[R];
#pragma unroll
      for (int m = 0; m < R; ++m) y[m] = gld(s + (j2 + m * LR) * hs);
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const cpx<T> a = x[m], b = y[R - 1 - m];
        x[m] = c2r_split(a, b, twl[j + m * LR]);
        y[R - 1 - m] = c2r_split(b, a, twl[j2 + (R - 1 - m) * LR]);
      }
      Dft<T, R, true>::run(x);
      Dft<T, R, true>::run(y);
#pragma unroll
      for (int m = 0; m < R; ++m) {
        line[j * R + m] = x[m];
        line[j2 * R + m] = y[m];
      }
    }
  }
}

// last inverse pass -> constitutive law on the voxel pairs -> first forward pass.
// Rounds of whole lines, so a round never reads what an earlier round wrote.
template <typename T, bool ISO, int R>
__device__ __forceinline__ void xf_middle(const Desc& d, const XGeo& xg, cpx<T>* buf, const cpx<T>* twl,
                                          const HZ_GLB uint16_t* __restrict__ ph, double (&acc)[6]) {
  const int M = xg.M, LR = M / R, TY = xg.TY, H1p = xg.H1p;
  const int n = TY * LR;
  const int per = (kThreads / LR) * LR;
  const HZ_GLB T* C = glb(sizeof(T) == 8 ? reinterpret_cast<const T*>(d.C64) : reinterpret_cast<const T*>(d.C32));
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
          constitutive_iso<T>(la.x, la.y, d.Ebar, ea, sa);
          constitutive_iso<T>(lb.x, lb.y, d.Ebar, eb, sb);
        } else {
          constitutive<T>(C + pa * 24, d.Ebar, ea, sa);
          __builtin_amdgcn_sched_barrier(0);  // one stiffness row set live at a time
          constitutive<T>(C + pb * 24, d.Ebar, eb, sb);
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

// ISO: every phase of the material is isotropic (separate instantiations keep the
// register budget of each at two waves per SIMD in FP64)
template <typename T, bool ISO>
__global__ __launch_bounds__(kThreads) void k_xfused(const Desc* __restrict__ descs,
                                                     const int* __restrict__ active, XGeo xg,
                                                     const Plan* __restrict__ planXi,
                                                     const Plan* __restrict__ planXf,
                                                     const cpx<T>* __restrict__ twN1) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[6 * 4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d) || (d.iso != 0) != ISO) return;
  const int tiles2 = xg.N2 / xg.TY;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int half = xg.half >= 0 ? xg.half : (tile & 1);
  const int rt = xg.half >= 0 ? tile : (tile >> 1);
  const int l3 = rt / tiles2;
  const int l2_0 = (rt % tiles2) * xg.TY;
  const int TY = xg.TY, M = xg.M;
  const long long row0 = (long long)l3 * xg.N2 + l2_0;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = buf + 6 * TY * xg.H1p;
  for (int i = threadIdx.x; i < xg.N1; i += kThreads) twl[i] = twN1[i];
  __syncthreads();
  const int off = (int)(half * 6 * xg.S + row0);
  const HZ_GLB cpx<T>* src = glb(reinterpret_cast<const cpx<T>*>(d.spec)) + off;
  HZ_GLB cpx<T>* dst = glb(reinterpret_cast<cpx<T>*>(d.spec)) + off;
  const Plan& pi = *planXi;
  const Plan& pf = *planXf;
  const int np = pi.np;
  switch (pi.radix[0]) {
    case 16: xf_load<T, 16>(xg, src, buf, twl); break;
    case 8: xf_load<T, 8>(xg, src, buf, twl); break;
    case 4: xf_load<T, 4>(xg, src, buf, twl); break;
    default: xf_load<T, 2>(xg, src, buf, twl); break;
  }
  __syncthreads();
  const LdsAcc<T> lds{buf, xg.H1p, 1};
  int Ns = pi.radix[0];
#pragma unroll 1
  for (int p = 1; p < np - 1; ++p) {
    pass_any<T, emax<T>(), true>(pi.radix[p], M, Ns, 6 * TY, true, twl, 2, lds, lds, true, pi.rLR[p], pi.rNs[p], 0.f);
    __syncthreads();
    Ns *= pi.radix[p];
  }
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const HZ_GLB uint16_t* ph = glb(d.phase) + row0 * xg.N1;
  switch (pi.radix[np - 1]) {
    case 4: xf_middle<T, ISO, 4>(d, xg, buf, twl, ph, acc); break;
    case 2: xf_middle<T, ISO, 2>(d, xg, buf, twl, ph, acc); break;
    case 5: xf_middle<T, ISO, 5>(d, xg, buf, twl, ph, acc); break;
    default: xf_middle<T, ISO, 3>(d, xg, buf, twl, ph, acc); break;
  }
  Ns = pf.radix[0];
#pragma unroll 1
  for (int p = 1; p < np - 1; ++p) {
    pass_any<T, emax<T>(), false>(pf.radix[p], M, Ns, 6 * TY, true, twl, 2, lds, lds, true, pf.rLR[p], pf.rNs[p], 0.f);
    __syncthreads();
    Ns *= pf.radix[p];
  }
  switch (pf.radix[np - 1]) {
    case 16: xf_store<T, 16>(xg, dst, buf, twl); break;
    case 8: xf_store<T, 8>(xg, dst, buf, twl); break;
    case 4: xf_store<T, 4>(xg, dst, buf, twl); break;
    default: xf_store<T, 2>(xg, dst, buf, twl); break;
  }
  block_sum<6>(acc, red);
  if (threadIdx.x == 0) {
    double* pp = d.part_sig + (long long)(xg.half >= 0 ? 2 * tile + half : tile) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) pp[c] = acc[c];
  }
}

// ----------------------------------------------------------------------------
// Stencil form of one iteration.  The symbols of eq. Dq are the 4-corner finite
// differences of eqs. DA1-DA2: with the library's integer corner indexing, voxel
// r has corners r + o, o in {0,-1}^3, each with weight w(o) = o + (1/2,1/2,1/2);
// tetrahedron T1 takes the corners with even o1+o2+o3, T2 the odd ones, and
//   D^Tk_i[u](r) = sum_{o in Tk} w_i(o) u(r + o),
//   g_i(c) = sum_k sum_{o in Tk} sum_j sigma^Tk_ij(c - o) w_j(o),
// whose transform (1/N) is the residual r(q) of the Fourier form.  So only the
// 3 displacement and 3 force components go through the transforms.
// ----------------------------------------------------------------------------

// inverse z transform of u (3 comps): u(q) -> slot 0, layout [c][h1][l3][h2]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zexp3(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                    ZGeo zg, const Plan* __restrict__ plan3,
                                                    const cpx<T>* __restrict__ tw3T) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int TX = zg.TX, N2 = zg.N2, N3 = zg.N3;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int h1 = tile / zg.tiles;
  const int h2_0 = (tile % zg.tiles) * TX;
  const int lines = 3 * TX;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = buf + lines * N3;
  for (int i = threadIdx.x; i < N3; i += kThreads) twl[i] = tw3T[i];
  __syncthreads();
  const long long plane = (long long)h1 * N3 * N2 + h2_0;
  const LdsAcc<T> lds{buf, 1, lines};
  const void* usrc = d.src == 1 ? d.u64 : d.u[cur_slot(d)];
  const GblAcc<T> src{glb(reinterpret_cast<cpx<T>*>(const_cast<void*>(usrc))) + plane, (int)zg.S, TX, 1, N2};
  const GblAcc<T> dst{glb(reinterpret_cast<cpx<T>*>(d.spec)) + plane, (int)zg.S, TX, 1, N2};
  fft_lines<T, emax<T>(), true>(*plan3, lines, zg.rLines, false, twl, 1, lds, src, dst);
}

// C2R along x of u (slot 0 -> slot 3 real rows).  Uses the fused pass's
// factorisation: split + first inverse pass, middle passes, last pass to HBM.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_xc2r(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                   XGeo xg, const Plan* __restrict__ planXi,
                                                   const cpx<T>* __restrict__ twN1) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int tiles2 = xg.N2 / xg.TY;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int l3 = tile / tiles2;
  const int l2_0 = (tile % tiles2) * xg.TY;
  const int TY = xg.TY, M = xg.M;
  const int row0 = l3 * xg.N2 + l2_0;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = buf + 3 * TY * xg.H1p;
  for (int i = threadIdx.x; i < xg.N1; i += kThreads) twl[i] = twN1[i];
  __syncthreads();
  HZ_GLB cpx<T>* spec = glb(reinterpret_cast<cpx<T>*>(d.spec));
  const Plan& pi = *planXi;
  const int np = pi.np;
  switch (pi.radix[0]) {
    case 16: xf_load<T, 16, 3>(xg, spec + row0, buf, twl); break;
    case 8: xf_load<T, 8, 3>(xg, spec + row0, buf, twl); break;
    case 4: xf_load<T, 4, 3>(xg, spec + row0, buf, twl); break;
    default: xf_load<T, 2, 3>(xg, spec + row0, buf, twl); break;
  }
  __syncthreads();
  const LdsAcc<T> lds{buf, xg.H1p, 1};
  int Ns = pi.radix[0];
#pragma unroll 1
  for (int p = 1; p < np - 1; ++p) {
    pass_any<T, emax<T>(), true>(pi.radix[p], M, Ns, 3 * TY, true, twl, 2, lds, lds, true, pi.rLR[p], pi.rNs[p], 0.f);
    __syncthreads();
    Ns *= pi.radix[p];
  }
  // real row (l3, l2) of comp c as M complex values z[n] = x[2n] + i x[2n+1]
  const int half_n = (xg.N1 / 2) * xg.N2 * xg.N3;
  const GblAcc<T> out{spec + 3 * xg.S + (long long)row0 * M, half_n, TY, M, 1};
  pass_any<T, emax<T>(), true>(pi.radix[np - 1], M, Ns, 3 * TY, true, twl, 2, lds, out, false, pi.rLR[np - 1],
                               pi.rNs[np - 1], 0.f);
}

// R2C along x of the corner force g (slot 6 real rows -> slot 9), with 1/N
template <typename T>
__global__ __launch_bounds__(kThreads) void k_xr2c(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                   XGeo xg, const Plan* __restrict__ planXf,
                                                   const cpx<T>* __restrict__ twN1) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int tiles2 = xg.N2 / xg.TY;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int l3 = tile / tiles2;
  const int l2_0 = (tile % tiles2) * xg.TY;
  const int TY = xg.TY, M = xg.M;
  const int row0 = l3 * xg.N2 + l2_0;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = buf + 3 * TY * xg.H1p;
  for (int i = threadIdx.x; i < xg.N1; i += kThreads) twl[i] = twN1[i];
  __syncthreads();
  HZ_GLB cpx<T>* spec = glb(reinterpret_cast<cpx<T>*>(d.spec));
  const Plan& pf = *planXf;
  const int np = pf.np;
  const LdsAcc<T> lds{buf, xg.H1p, 1};
  const int half_n = (xg.N1 / 2) * xg.N2 * xg.N3;
  const GblAcc<T> in{spec + 6 * xg.S + (long long)row0 * M, half_n, TY, M, 1};
  pass_any<T, emax<T>(), false>(pf.radix[0], M, 1, 3 * TY, true, twl, 2, in, lds, false, pf.rLR[0], pf.rNs[0], 0.f);
  __syncthreads();
  int Ns = pf.radix[0];
#pragma unroll 1
  for (int p = 1; p < np - 1; ++p) {
    pass_any<T, emax<T>(), false>(pf.radix[p], M, Ns, 3 * TY, true, twl, 2, lds, lds, true, pf.rLR[p], pf.rNs[p], 0.f);
    __syncthreads();
    Ns *= pf.radix[p];
  }
  switch (pf.radix[np - 1]) {
    case 16: xf_store<T, 16, 3>(xg, spec + 9 * xg.S + row0, buf, twl); break;
    case 8: xf_store<T, 8, 3>(xg, spec + 9 * xg.S + row0, buf, twl); break;
    case 4: xf_store<T, 4, 3>(xg, spec + 9 * xg.S + row0, buf, twl); break;
    default: xf_store<T, 2, 3>(xg, spec + 9 * xg.S + row0, buf, twl); break;
  }
}

// corner o in {0,-1}^3 coded as bits (bit a set: o_a = 0, clear: o_a = -1);
// T1 takes the corners with an even number of -1 offsets
__device__ __forceinline__ int tet_of(int o) { return ((o & 1) + ((o >> 1) & 1) + ((o >> 2) & 1)) & 1 ? 0 : 1; }

// sigma^T1 (s[0..5]) and sigma^T2 (s[6..11]) of one voxel from its 8 corners u8[o][j]
template <typename T, bool ISO>
__device__ __forceinline__ void stencil_sigma(const Desc& d, const HZ_GLB T* C, int ph, const T (&u8)[8][3],
                                              T (&s)[12]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    T G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      if (tet_of(o) != k) continue;
      // w_i(o) = +1/2 if o_i = 0 (bit set), -1/2 if o_i = -1 (bit clear)
      const T w0 = (o & 1) ? (T)0.5 : (T)-0.5, w1 = (o & 2) ? (T)0.5 : (T)-0.5, w2 = (o & 4) ? (T)0.5 : (T)-0.5;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        G[0][j] += w0 * u8[o][j];
        G[1][j] += w1 * u8[o][j];
        G[2][j] += w2 * u8[o][j];
      }
    }
    T e[6];
    e[0] = G[0][0];
    e[1] = G[1][1];
    e[2] = G[2][2];
    e[3] = (T)0.5 * (G[1][2] + G[2][1]);
    e[4] = (T)0.5 * (G[0][2] + G[2][0]);
    e[5] = (T)0.5 * (G[0][1] + G[1][0]);
    T out[6];
    if (ISO) {
      const cpx<T> l = gld(reinterpret_cast<const HZ_GLB cpx<T>*>(C) + ph);
      constitutive_iso<T>(l.x, l.y, d.Ebar, e, out);
    } else {
      constitutive<T>(C + ph * 24, d.Ebar, e, out);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) s[6 * k + c] = out[c];
  }
}

// Strain, constitutive law and corner force in real space.  A block owns a
// kStX x kStY column of corners over TZ planes and streams along z: at voxel
// plane p the corner planes p-1 and p sit in LDS (ring of two), it computes sigma
// of the voxel plane (one halo voxel on the + side in x and y), completes the
// force of corner plane p-1 and starts that of corner plane p.  Corner plane p+1
// is fetched into registers one step ahead, so its latency overlaps the work.
template <typename T, bool ISO>
__global__ __launch_bounds__(kThreads) void k_stencil(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                      SGeo sg) {
  constexpr int UX = kStX + 2, UY = kStY + 2, VX = kStX + 1, VY = kStY + 1;
  constexpr int UP = 3 * UY * UX;                      // corner values per plane
  constexpr int NL = (UP + kThreads - 1) / kThreads;   // per thread
  __shared__ T ub[2][UP];                              // [slot][c][yy][xx]
  __shared__ T sb[12][VY][VX];
  __shared__ double red[6 * 4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d) || (d.iso != 0) != ISO) return;
  const int N1 = sg.N1, N2 = sg.N2, N3 = sg.N3;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = tile % sg.tx, byz = tile / sg.tx;
  const int by = byz % sg.ty, bz = byz / sg.ty;
  const int x0 = bx * kStX, y0 = by * kStY, z0 = bz * sg.TZ;
  const int wx = min(kStX, N1 - x0), wy = min(kStY, N2 - y0), wz = min(sg.TZ, N3 - z0);
  const int Nn = N1 * N2 * N3, NP = N1 * N2;
  const long long S = (long long)(N1 / 2 + 1) * N2 * N3;
  const HZ_GLB T* ur = reinterpret_cast<const HZ_GLB T*>(glb(reinterpret_cast<const cpx<T>*>(d.spec)) + 3 * S);
  HZ_GLB T* gr = reinterpret_cast<HZ_GLB T*>(glb(reinterpret_cast<cpx<T>*>(d.spec)) + 6 * S);
  const HZ_GLB T* C = glb(sizeof(T) == 8 ? reinterpret_cast<const T*>(d.C64) : reinterpret_cast<const T*>(d.C32));
  const HZ_GLB uint16_t* ph = glb(d.phase);
  const int tid = threadIdx.x;
  const int cx = tid % kStX, cy = tid / kStX;  // the corner this thread owns
  const bool own = cx < wx && cy < wy;
  // in-plane offsets of this thread's corner loads (periodic wrap)
  int loff[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int i = tid + k * kThreads;
    loff[k] = -1;
    if (i < UP) {
      const int c = i / (UY * UX), rem = i - c * (UY * UX);
      const int yy = rem / UX, xx = rem - yy * UX;
      int gx = x0 - 1 + xx, gy = y0 - 1 + yy;
      while (gx < 0) gx += N1;
      while (gx >= N1) gx -= N1;
      while (gy < 0) gy += N2;
      while (gy >= N2) gy -= N2;
      loff[k] = c * Nn + gy * N1 + gx;
    }
  }
  // in-plane phase-map offsets of this thread's voxels
  const int nv = (wx + 1) * (wy + 1);
  int voff[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int v = tid + k * kThreads;
    const int vy = v / (wx + 1), vx = v - vy * (wx + 1);
    int gx = x0 + vx, gy = y0 + vy;
    while (gx >= N1) gx -= N1;
    while (gy >= N2) gy -= N2;
    voff[k] = gy * N1 + gx;
  }
  T rg[NL];
  auto fetch = [&](int q) {
    const int qq = q < 0 ? q + N3 : (q >= N3 ? q - N3 : q);
    const HZ_GLB T* base = ur + (long long)qq * NP;
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (loff[k] >= 0) rg[k] = base[loff[k]];
  };
  auto stash = [&](int slot) {
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (loff[k] >= 0) ub[slot][tid + k * kThreads] = rg[k];
  };
  fetch(z0 - 1);
  stash((z0 + 1) & 1);
  fetch(z0);
  stash(z0 & 1);
  fetch(z0 + 1);
  T acc[3] = {0, 0, 0};
  double sacc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 1
  for (int p = z0; p <= z0 + wz; ++p) {
    const int cur = p & 1, prv = cur ^ 1;
    __syncthreads();
    // sigma of voxel plane p over (wx+1) x (wy+1) voxels
    const int pp = p >= N3 ? p - N3 : p;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int v = tid + k * kThreads;
      if (v >= nv) continue;
      const int vy = v / (wx + 1), vx = v - vy * (wx + 1);
      T u8[8][3];
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        // bit a set: o_a = 0, clear: o_a = -1; corner (vx + o1, vy + o2) sits at (vx + o1 + 1, vy + o2 + 1)
        const int ix = vx + ((o & 1) ? 1 : 0), iy = vy + ((o & 2) ? 1 : 0);
        const int sl = (o & 4) ? cur : prv;
#pragma unroll
        for (int j = 0; j < 3; ++j) u8[o][j] = ub[sl][(j * UY + iy) * UX + ix];
      }
      const int phv = ph[(long long)pp * NP + voff[k]];
      T s12[12];
      stencil_sigma<T, ISO>(d, C, phv, u8, s12);
#pragma unroll
      for (int c = 0; c < 12; ++c) sb[c][vy][vx] = s12[c];
      if (vx < wx && vy < wy && p < z0 + wz) {
#pragma unroll
        for (int c = 0; c < 6; ++c) sacc[c] += 0.5 * ((double)s12[c] + (double)s12[6 + c]);
      }
    }
    __syncthreads();
    if (own) {
      // corner (cx, cy) receives sigma of voxel (cx - o1, cy - o2): offset -1 -> voxel +1
      T g1[3] = {0, 0, 0}, g0[3] = {0, 0, 0};
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int k = tet_of(o);
        const int vx = cx + ((o & 1) ? 0 : 1), vy = cy + ((o & 2) ? 0 : 1);
        const T w0 = (o & 1) ? (T)0.5 : (T)-0.5, w1 = (o & 2) ? (T)0.5 : (T)-0.5, w2 = (o & 4) ? (T)0.5 : (T)-0.5;
        const T s0 = sb[6 * k + 0][vy][vx], s1 = sb[6 * k + 1][vy][vx], s2 = sb[6 * k + 2][vy][vx];
        const T s3 = sb[6 * k + 3][vy][vx], s4 = sb[6 * k + 4][vy][vx], s5 = sb[6 * k + 5][vy][vx];
        const T f0 = s0 * w0 + s5 * w1 + s4 * w2;
        const T f1 = s5 * w0 + s1 * w1 + s3 * w2;
        const T f2 = s4 * w0 + s3 * w1 + s2 * w2;
        // o3 = 0 (bit 2 set): voxel plane = corner plane p; o3 = -1: corner plane p - 1
        if (o & 4) {
          g0[0] += f0; g0[1] += f1; g0[2] += f2;
        } else {
          g1[0] += f0; g1[1] += f1; g1[2] += f2;
        }
      }
      if (p > z0) {
        const int at = (p - 1) * NP + (y0 + cy) * N1 + (x0 + cx);
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[(long long)j * Nn + at] = acc[j] + g1[j];
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) acc[j] = g0[j];
    }
    // corner plane p+1 goes where plane p-1 was (no longer read), then fetch p+2
    if (p < z0 + wz) {
      stash(prv);
      if (p + 1 < z0 + wz) fetch(p + 2);
    }
  }
  block_sum<6>(sacc, red);
  if (tid == 0) {
    double* pp = d.part_sig + (long long)tile * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) pp[c] = sacc[c];
  }
}

// ----------------------------------------------------------------------------
// P5: residual r = sigma^T1.conj(D~) + sigma^T2.conj(D~2) (eq. Equilibrium_Q_div_bis),
// formed before the forward z transform as R(l3) = A(l3) + B(l3 + 1) with
// A = sigma.conj(alpha), B = sigma.conj(beta); then the transform of its 3 comps,
// the Green operator in FP64 (eq. Green_tensor) and the update (eq. basic_scheme_dep_2).
// d.cmode 0: u[1-p] = u[p] - Omega r      (p = current slot)
// d.cmode 1: FP64 sweep of the anchor: store r in r32, no update
// d.cmode 2: correction round: r += r32, u[1-p] = u[p] - Omega r
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void sig_dot(const cpx<T> (&s)[6], const cpx<double>* c, cpx<double>* out) {
  // out_i = sum_j s_ij c_j, comps (11,22,33,23,13,12)
  const cpx<double> s0 = to64(s[0]), s1 = to64(s[1]), s2 = to64(s[2]);
  const cpx<double> s3 = to64(s[3]), s4 = to64(s[4]), s5 = to64(s[5]);
  out[0] = s0 * c[0] + s5 * c[1] + s4 * c[2];
  out[1] = s5 * c[0] + s1 * c[1] + s3 * c[2];
  out[2] = s4 * c[0] + s3 * c[1] + s2 * c[2];
}

// STENCIL: the residual's 3 components already sit in spec slot 9 (the stencil form's
// forward-transformed corner forces), so phase A is the first radix pass from HBM.
template <typename T, bool STENCIL>
__global__ __launch_bounds__(kThreads) void k_zcon(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                   ZGeo zg, const Plan* __restrict__ plan3, const cpx<T>* __restrict__ tw3T,
                                                   const cpx<double>* __restrict__ tw1,
                                                   const cpx<double>* __restrict__ tw2,
                                                   const cpx<double>* __restrict__ tw3) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int TX = zg.TX, N2 = zg.N2, N3 = zg.N3;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int h1 = tile / zg.tiles;
  const int h2_0 = (tile % zg.tiles) * TX;
  const int lines = 3 * TX;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = buf + lines * N3;
  for (int i = threadIdx.x; i < N3; i += kThreads) twl[i] = tw3T[i];
  const long long plane = (long long)h1 * N3 * N2 + h2_0;
  const LdsAcc<T> lds{buf, 1, lines};
  const HZ_GLB cpx<T>* sp = glb(reinterpret_cast<const cpx<T>*>(d.spec)) + plane;
  const cpx<double> t1 = tw1[h1];
  const int ne = TX * N3;
  if (STENCIL) {
    __syncthreads();  // twiddles
    const GblAcc<T> src{const_cast<HZ_GLB cpx<T>*>(sp) + 9 * zg.S, (int)zg.S, TX, 1, N2};
    fft_lines<T, emax<T>(), false>(*plan3, lines, zg.rLines, false, twl, 1, lds, src, lds);
  } else {
  // phase A: each thread walks a run of l3 values of one column downwards, so that
  // R(l) = A(l) + B(l+1) needs one extra row of loads per run, not one per element
  const int m = (ne + kThreads - 1) / kThreads;  // run length
  const int nruns = (N3 + m - 1) / m;
  for (int wk = threadIdx.x; wk < TX * nruns; wk += kThreads) {
    const int run = fdiv(wk, zg.rTX), col = wk - run * TX;
    {
      cpx<double> a1[3], b1[3], a2[3], b2[3];
      affine_symbols(t1, tw2[h2_0 + col], a1, b1, a2, b2);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a1[c] = conjg(a1[c]); b1[c] = conjg(b1[c]); a2[c] = conjg(a2[c]); b2[c] = conjg(b2[c]);
      }
      const int l0 = run * m;
      const int l1 = min(l0 + m, N3);  // rows l0 .. l1-1 produced, row l1 (mod N3) read
      cpx<double> Bn[3];
      {
        const int l = l1 == N3 ? 0 : l1;
        const long long o = (long long)l * N2 + col;
        cpx<T> s1[6], s2[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          s1[c] = gld(sp + c * zg.S + o);
          s2[c] = gld(sp + (6 + c) * zg.S + o);
        }
        cpx<double> y1[3], y2[3];
        sig_dot(s1, b1, y1);
        sig_dot(s2, b2, y2);
#pragma unroll
        for (int c = 0; c < 3; ++c) Bn[c] = y1[c] + y2[c];
      }
#pragma unroll 1
      for (int l = l1 - 1; l >= l0; --l) {
        {
          const long long o = (long long)l * N2 + col;
          cpx<T> s1[6], s2[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            s1[c] = gld(sp + c * zg.S + o);
            s2[c] = gld(sp + (6 + c) * zg.S + o);
          }
          cpx<double> x1[3], x2[3], y1[3], y2[3];
          sig_dot(s1, a1, x1);
          sig_dot(s2, a2, x2);
          sig_dot(s1, b1, y1);
          sig_dot(s2, b2, y2);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            lds.put(c * TX + col, l, fr64<T>(x1[c] + x2[c] + Bn[c]));
            Bn[c] = y1[c] + y2[c];
          }
        }
      }
    }
  }
  __syncthreads();
  fft_lines<T, emax<T>(), false>(*plan3, lines, zg.rLines, false, twl, 1, lds, lds, lds);
  }
  __syncthreads();
  // phase C: Green operator and update at q = (h1, h2, h3)
  double part[1] = {0.0};
  const double w = (h1 == 0 || 2 * h1 == zg.N1) ? 1.0 : 2.0;
  for (int e = threadIdx.x; e < ne; e += kThreads) {
    const int h3 = fdiv(e, zg.rTX), col = e - h3 * TX;
    const int h2 = h2_0 + col;
    const long long o = (long long)h3 * N2 + col;
    cpx<double> r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = to64(lds.get(c * TX + col, h3));
    const int MODE = d.cmode;
    if (MODE == 2) {
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = r[c] + to64(gld(glb(reinterpret_cast<const cpx<float>*>(d.r32)) + c * zg.S + plane + o));
    }
    part[0] += 0.25 * w * (r[0].x * r[0].x + r[0].y * r[0].y + r[1].x * r[1].x + r[1].y * r[1].y +
                           r[2].x * r[2].x + r[2].y * r[2].y);
    if (MODE == 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) gst(glb(reinterpret_cast<cpx<float>*>(d.r32)) + c * zg.S + plane + o, fr64<float>(r[c]));
      continue;
    }
    cpx<double> D1[3], D2[3];
    symbols(t1, tw2[h2], tw3[h3], D1, D2);
    // K_il = sum_jk C0_ijkl M_jk,  M_jk = 2 Re(conj(D_j) D_k)
    double Mjk[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) Mjk[j][k] = 2.0 * (D1[j].x * D1[k].x + D1[j].y * D1[k].y);
    double K[3][3];
    if (d.c0_iso) {
      // isotropic lambda0: K = mu0 tr(M) I + (lam0 + mu0) M
      const double tm = d.mu0 * (Mjk[0][0] + Mjk[1][1] + Mjk[2][2]), lm = d.lam0 + d.mu0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l) K[i][l] = lm * Mjk[i][l] + (i == l ? tm : 0.0);
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += d.C0[((i * 3 + j) * 3 + k) * 3 + l] * Mjk[j][k];
          K[i][l] = acc;
        }
    }
    const bool sing = (h1 == 0 && h2 == 0 && h3 == 0) || (2 * h1 == zg.N1 && 2 * h2 == N2 && 2 * h3 == N3);
    // Omega = K^-1 by the adjugate (K symmetric)
    const double a00 = K[1][1] * K[2][2] - K[1][2] * K[2][1];
    const double a01 = K[0][2] * K[2][1] - K[0][1] * K[2][2];
    const double a02 = K[0][1] * K[1][2] - K[0][2] * K[1][1];
    const double a11 = K[0][0] * K[2][2] - K[0][2] * K[2][0];
    const double a12 = K[0][2] * K[1][0] - K[0][0] * K[1][2];
    const double a22 = K[0][0] * K[1][1] - K[0][1] * K[1][0];
    const double det = K[0][0] * a00 + K[0][1] * a01 + K[0][2] * a02;
    const double inv = sing ? 0.0 : 1.0 / det;
    const double O[3][3] = {{a00 * inv, a01 * inv, a02 * inv},
                            {a01 * inv, a11 * inv, a12 * inv},
                            {a02 * inv, a12 * inv, a22 * inv}};
    const int p = cur_slot(d);
    const HZ_GLB cpx<T>* uin = glb(reinterpret_cast<const cpx<T>*>(d.u[p])) + plane;
    HZ_GLB cpx<T>* uout = glb(reinterpret_cast<cpx<T>*>(d.u[1 - p])) + plane;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const cpx<double> dw = {O[i][0] * r[0].x + O[i][1] * r[1].x + O[i][2] * r[2].x,
                              O[i][0] * r[0].y + O[i][1] * r[1].y + O[i][2] * r[2].y};
      gst(uout + i * zg.S + o, fr64<T>(to64(gld(uin + i * zg.S + o)) - dw));
    }
  }
  block_sum<1>(part, red);
  if (threadIdx.x == 0) d.part_res[tile] = part[0];
}

// ----------------------------------------------------------------------------
// Fixed-order sums of the partials and the stop rule (eqs. L2-norm, tolerance).
// d.fmode 0: plain iteration on u.  1: FP64 sweep (measure only).
// 2: correction round (stop at ST_REF or on stagnation).  3: FP32 round 0.
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_finalize(const Desc* __restrict__ descs,
                                                       const int* __restrict__ active, FinGeo fg) {
  __shared__ double red[7 * 4];
  const Desc& d = descs[active[blockIdx.x]];
  if (problem_done(d)) return;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  const int fmode = d.fmode;
  const int parity = cur_slot(d);
  if (fmode != 2) {
    for (int b = threadIdx.x; b < fg.nbx; b += kThreads) {
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] += d.part_sig[(long long)b * 6 + c];
    }
  }
  for (int b = threadIdx.x; b < fg.nbq; b += kThreads) v[6] += d.part_res[b];
  block_sum<7>(v, red);
  if (threadIdx.x != 0) return;
  double* s = d.status;
  const int k = (int)s[ST_K];
  if (fmode == 2) {
    // inner FP32 iteration: residual of U + delta relative to the sweep's ||<sigma>||
    const double err = sqrt(v[6]) / s[ST_NORM];
    s[ST_ERR] = err;
    s[ST_K] = k + 1;
    const bool reached = err <= s[ST_REF];
    const bool bad = !(err == err) || isinf(err) || err > 1e3 * s[ST_FIRST_ERR];
    // stagnation (the FP32 rounding floor): less than 3% gain over 32 inner iterations
    bool stalled = false;
    if (k > 0 && (k % 32) == 0) {
      if (err > 0.97 * s[ST_BEST]) stalled = true;
      else s[ST_BEST] = err;
    }
    if (reached || bad || stalled || k + 1 >= d.inner_max) {
      s[ST_DONE] = bad ? 3.0 : 1.0;
      s[ST_ITERS] = k + 1;       // inner updates applied
      s[ST_PARITY] = 1 - parity;
    }
    return;
  }
  double m[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) m[c] = v[c] * fg.invN;
  const double nrm = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2] +
                          2.0 * (m[3] * m[3] + m[4] * m[4] + m[5] * m[5]));
  const double L2 = sqrt(v[6]);
  const double err = nrm > 0.0 ? L2 / nrm : L2;
  if (k < d.trace_len && d.trace) {
    double* tr = d.trace + (long long)k * 7;
    tr[0] = err;
#pragma unroll
    for (int c = 0; c < 6; ++c) tr[1 + c] = m[c];
  }
  s[ST_ERR] = err;
#pragma unroll
  for (int c = 0; c < 6; ++c) s[ST_MEAN + c] = m[c];
  s[ST_L2SQ] = v[6];
  s[ST_NORM] = nrm;
  if (k == 0) s[ST_FIRST_ERR] = err;
  s[ST_K] = k + 1;
  if (fmode == 1) {
    // a sweep measures once; the host decides what follows
    s[ST_DONE] = 1.0;
    s[ST_ITERS] = k;
    return;
  }
  if (fmode == 3) {
    // plain FP32 iterations of refinement round 0: stop at the target, at the FP32
    // rounding floor (less than 3% gain over 32 iterations) or at the cap
    const bool reached = err <= s[ST_REF];
    const bool bad = !(err == err) || isinf(err) || (k > 0 && err > 1e3 * s[ST_FIRST_ERR]);
    bool stalled = false;
    if (k > 0 && (k % 32) == 0) {
      if (err > 0.97 * s[ST_BEST]) stalled = true;
      else s[ST_BEST] = err;
    }
    if (reached || bad || stalled || k + 1 >= d.inner_max) {
      s[ST_DONE] = bad ? 3.0 : 1.0;
      s[ST_ITERS] = k + 1;
      s[ST_PARITY] = 1 - parity;
    }
    return;
  }
  const bool stop = d.fixed_iters >= 0 ? (k >= d.fixed_iters) : (err < d.tol);
  const bool bad = !(err == err) || isinf(err) || (k > 0 && err > 1e3 * s[ST_FIRST_ERR]);
  if (stop || bad || k >= d.max_iters) {
    s[ST_DONE] = bad ? 3.0 : (stop ? 1.0 : 2.0);
    s[ST_ITERS] = k;
    s[ST_PARITY] = parity;
  }
}

// U64 += delta (refinement), delta in FP32
__global__ __launch_bounds__(kThreads) void k_accumulate(const Desc* __restrict__ descs,
                                                         const int* __restrict__ active,
                                                         long long n3c) {
  const Desc& d = descs[active[blockIdx.y]];
  const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= n3c) return;
  const int p = (int)d.status[ST_PARITY];
  const cpx<float> a = ld<float>(d.u[p], idx);
  cpx<double> b = ld<double>(d.u64, idx);
  b.x += (double)a.x;
  b.y += (double)a.y;
  st<double>(d.u64, idx, b);
}

// zero-fill (used instead of memset so every clear is an ordinary kernel)
__global__ __launch_bounds__(kThreads) void k_zero(const Desc* __restrict__ descs,
                                                   const int* __restrict__ active, int what,
                                                   long long nbytes16) {
  const Desc& d = descs[active[blockIdx.y]];
  const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= nbytes16) return;
  void* p = what == 0 ? d.u[0] : (what == 1 ? d.u[1] : d.u64);
  reinterpret_cast<cpx<double>*>(p)[idx] = cpx<double>{0.0, 0.0};
}

// ----------------------------------------------------------------------------
// launch wrappers
// ----------------------------------------------------------------------------
template <typename T>
hipError_t launch_zexp(const Desc* descs, const int* active, int nact, const ZGeo& zg, const Plan* plan3,
                       const void* tw3T, const void* tw1, const void* tw2, hipStream_t s) {
  const size_t shm = ((size_t)3 * zg.TX * zg.N3 + zg.N3) * sizeof(cpx<T>);
  dim3 grid((unsigned)(zg.H1 * zg.tiles), nact);
  hipLaunchKernelGGL(k_zexp<T>, grid, dim3(kThreads), shm, s, descs, active, zg, plan3, (const cpx<T>*)tw3T,
                     (const cpx<double>*)tw1, (const cpx<double>*)tw2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_yline(const Desc* descs, const int* active, int nact, const YGeo& yg, const Plan* plan2,
                        const void* tw2T, bool inv, hipStream_t s) {
  const size_t shm = ((size_t)yg.TX * yg.N2 + yg.N2) * sizeof(cpx<T>);
  dim3 grid((unsigned)((yg.nlines + yg.TX - 1) / yg.TX), nact);
  if (inv)
    hipLaunchKernelGGL((k_yline<T, true>), grid, dim3(kThreads), shm, s, descs, active, yg, plan2, (const cpx<T>*)tw2T);
  else
    hipLaunchKernelGGL((k_yline<T, false>), grid, dim3(kThreads), shm, s, descs, active, yg, plan2, (const cpx<T>*)tw2T);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xpass(const Desc* descs, const int* active, int nact, const XGeo& xg,
                        const Plan* planM, const void* twN1, hipStream_t s) {
  const size_t shm = ((size_t)6 * xg.TY * xg.H1p + xg.N1) * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY) * (xg.half >= 0 ? 1 : 2)), nact);
  hipLaunchKernelGGL(k_xpass<T>, grid, dim3(kThreads), shm, s, descs, active, xg, planM,
                     (const cpx<T>*)twN1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xfused(const Desc* descs, const int* active, int nact, bool iso, const XGeo& xg,
                         const Plan* planXi, const Plan* planXf, const void* twN1, hipStream_t s) {
  const size_t shm = ((size_t)6 * xg.TY * xg.H1p + xg.N1) * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY) * (xg.half >= 0 ? 1 : 2)), nact);
  if (iso)
    hipLaunchKernelGGL((k_xfused<T, true>), grid, dim3(kThreads), shm, s, descs, active, xg, planXi, planXf,
                       (const cpx<T>*)twN1);
  else
    hipLaunchKernelGGL((k_xfused<T, false>), grid, dim3(kThreads), shm, s, descs, active, xg, planXi, planXf,
                       (const cpx<T>*)twN1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zexp3(const Desc* descs, const int* active, int nact, const ZGeo& zg, const Plan* plan3,
                        const void* tw3T, hipStream_t s) {
  const size_t shm = ((size_t)3 * zg.TX * zg.N3 + zg.N3) * sizeof(cpx<T>);
  dim3 grid((unsigned)(zg.H1 * zg.tiles), nact);
  hipLaunchKernelGGL(k_zexp3<T>, grid, dim3(kThreads), shm, s, descs, active, zg, plan3, (const cpx<T>*)tw3T);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xc2r(const Desc* descs, const int* active, int nact, const XGeo& xg, const Plan* planXi,
                       const void* twN1, hipStream_t s) {
  const size_t shm = ((size_t)3 * xg.TY * xg.H1p + xg.N1) * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY)), nact);
  hipLaunchKernelGGL(k_xc2r<T>, grid, dim3(kThreads), shm, s, descs, active, xg, planXi, (const cpx<T>*)twN1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xr2c(const Desc* descs, const int* active, int nact, const XGeo& xg, const Plan* planXf,
                       const void* twN1, hipStream_t s) {
  const size_t shm = ((size_t)3 * xg.TY * xg.H1p + xg.N1) * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY)), nact);
  hipLaunchKernelGGL(k_xr2c<T>, grid, dim3(kThreads), shm, s, descs, active, xg, planXf, (const cpx<T>*)twN1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const Desc* descs, const int* active, int nact, bool iso, const SGeo& sg, hipStream_t s) {
  dim3 grid((unsigned)(sg.tx * sg.ty * sg.tz), nact);
  if (iso)
    hipLaunchKernelGGL((k_stencil<T, true>), grid, dim3(kThreads), 0, s, descs, active, sg);
  else
    hipLaunchKernelGGL((k_stencil<T, false>), grid, dim3(kThreads), 0, s, descs, active, sg);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zcon(const Desc* descs, const int* active, int nact, bool stencil, const ZGeo& zg,
                       const Plan* plan3, const void* tw3T, const void* tw1, const void* tw2, const void* tw3,
                       hipStream_t s) {
  const size_t shm = ((size_t)3 * zg.TX * zg.N3 + zg.N3) * sizeof(cpx<T>);
  dim3 grid((unsigned)(zg.H1 * zg.tiles), nact);
  if (stencil)
    hipLaunchKernelGGL((k_zcon<T, true>), grid, dim3(kThreads), shm, s, descs, active, zg, plan3, (const cpx<T>*)tw3T,
                       (const cpx<double>*)tw1, (const cpx<double>*)tw2, (const cpx<double>*)tw3);
  else
    hipLaunchKernelGGL((k_zcon<T, false>), grid, dim3(kThreads), shm, s, descs, active, zg, plan3, (const cpx<T>*)tw3T,
                       (const cpx<double>*)tw1, (const cpx<double>*)tw2, (const cpx<double>*)tw3);
  return hipGetLastError();
}

hipError_t launch_finalize(const Desc* descs, const int* active, int nact, const FinGeo& fg,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(nact), dim3(kThreads), 0, s, descs, active, fg);
  return hipGetLastError();
}

hipError_t launch_accumulate(const Desc* descs, const int* active, int nact, long long n3c,
                             hipStream_t s) {
  dim3 grid((unsigned)((n3c + kThreads - 1) / kThreads), nact);
  hipLaunchKernelGGL(k_accumulate, grid, dim3(kThreads), 0, s, descs, active, n3c);
  return hipGetLastError();
}

hipError_t launch_zero(const Desc* descs, const int* active, int nact, int what, long long n16,
                       hipStream_t s) {
  dim3 grid((unsigned)((n16 + kThreads - 1) / kThreads), nact);
  hipLaunchKernelGGL(k_zero, grid, dim3(kThreads), 0, s, descs, active, what, n16);
  return hipGetLastError();
}

template hipError_t launch_zexp<double>(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_zexp<float>(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_yline<double>(const Desc*, const int*, int, const YGeo&, const Plan*, const void*, bool, hipStream_t);
template hipError_t launch_yline<float>(const Desc*, const int*, int, const YGeo&, const Plan*, const void*, bool, hipStream_t);
template hipError_t launch_xpass<double>(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_xpass<float>(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_xfused<double>(const Desc*, const int*, int, bool, const XGeo&, const Plan*, const Plan*, const void*, hipStream_t);
template hipError_t launch_xfused<float>(const Desc*, const int*, int, bool, const XGeo&, const Plan*, const Plan*, const void*, hipStream_t);
template hipError_t launch_zexp3<double>(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_zexp3<float>(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_xc2r<double>(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_xc2r<float>(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_xr2c<double>(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_xr2c<float>(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_stencil<double>(const Desc*, const int*, int, bool, const SGeo&, hipStream_t);
template hipError_t launch_stencil<float>(const Desc*, const int*, int, bool, const SGeo&, hipStream_t);
template hipError_t launch_zcon<double>(const Desc*, const int*, int, bool, const ZGeo&, const Plan*, const void*, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_zcon<float>(const Desc*, const int*, int, bool, const ZGeo&, const Plan*, const void*, const void*, const void*, const void*, hipStream_t);

}  // namespace hz
