// HIP kernels (gfx950) of one iteration of the tetrahedral-stencil basic scheme.
//
// Iteration (Algorithm 1, Sec. 2.6), spectra stored as [comp][h1][h3][h2]:
//   k_expand    u(q) -> 12 strain spectra  eps^T1 = D~ (x)_s u, eps^T2 = D~2 (x)_s u
//   k_lines     inverse z, inverse y            (LDS Stockham, batched over comps)
//   k_xpass     per (l3, l2-tile): C2R along x, sigma = C(phase):(Ebar + eps), R2C along x,
//               FP64 partial sums of <sigma>
//   k_lines     forward y, forward z
//   k_contract  r = sigma^T1.conj(D~) + sigma^T2.conj(D~2), Omega(q) in FP64, u update,
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

// ----------------------------------------------------------------------------
// P1: displacement spectrum -> 12 strain spectra (eqs. desp_T1_dep_Q, desp_T2_dep_Q)
// src: 0 = u[parity] in kernel precision, 1 = FP64 anchor u64
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_expand(const Desc* __restrict__ descs,
                                                     const int* __restrict__ active, int parity,
                                                     int src, Geo g,
                                                     const cpx<double>* __restrict__ tw1,
                                                     const cpx<double>* __restrict__ tw2,
                                                     const cpx<double>* __restrict__ tw3) {
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= g.S) return;
  const int h2 = (int)(idx % g.N2);
  const int h3 = (int)((idx / g.N2) % g.N3);
  const int h1 = (int)(idx / ((long long)g.N2 * g.N3));
  cpx<double> D1[3], D2[3];
  symbols(tw1[h1], tw2[h2], tw3[h3], D1, D2);
  cpx<double> u[3];
  if (src == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = ld<double>(d.u64, c * g.S + idx);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = to64(ld<T>(d.u[parity], c * g.S + idx));
  }
  // symmetric products in component order 11,22,33,23,13,12
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const cpx<double>* D = t == 0 ? D1 : D2;
    cpx<double> e[6];
    e[0] = D[0] * u[0];
    e[1] = D[1] * u[1];
    e[2] = D[2] * u[2];
    e[3] = scale(D[1] * u[2] + D[2] * u[1], 0.5);
    e[4] = scale(D[0] * u[2] + D[2] * u[0], 0.5);
    e[5] = scale(D[0] * u[1] + D[1] * u[0], 0.5);
#pragma unroll
    for (int c = 0; c < 6; ++c) st<T>(d.spec, (t * 6 + c) * g.S + idx, fr64<T>(e[c]));
  }
}

// ----------------------------------------------------------------------------
// y / z passes: batched 1D transforms along a strided axis, LDS Stockham.
// mode 0 (y): lines are contiguous rows of length L = N2; a tile is TX rows.
// mode 1 (z): lines run along h3 with stride N2; a tile is TX adjacent h2 columns
//             of one (comp, h1) plane, so every row of the tile is TX*16 B contiguous.
// ----------------------------------------------------------------------------

template <typename T, bool INV>
__global__ __launch_bounds__(kThreads) void k_lines(const Desc* __restrict__ descs,
                                                    const int* __restrict__ active, LinesGeo lg,
                                                    Plan plan, const cpx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  cpx<T>* data = reinterpret_cast<cpx<T>*>(lg.which == 0 ? d.spec : d.u[lg.parity]);
  const int L = lg.L;
  if (lg.mode == 0) {
    const long long t0 = (long long)blockIdx.x * lg.TX;
    const int lines = (int)((lg.nlines - t0) < lg.TX ? (lg.nlines - t0) : lg.TX);
    cpx<T>* base = data + t0 * L;
    const int n = lines * L;
    for (int f = threadIdx.x; f < n; f += kThreads) buf[f] = base[f];
    __syncthreads();
    lds_fft_chunked<T, emax_of<T>(), INV>(buf, plan, lines, L, 1, true, tw, 1);
    for (int f = threadIdx.x; f < n; f += kThreads) base[f] = buf[f];
  } else {
    const int TX = lg.TX;
    const long long plane = blockIdx.x / lg.tiles_per_plane;
    const int h2_0 = (blockIdx.x % lg.tiles_per_plane) * TX;
    cpx<T>* base = data + plane * (long long)lg.N3 * lg.N2 + h2_0;
    const int n = TX * L;
    for (int f = threadIdx.x; f < n; f += kThreads) {
      const int t = f % TX, j = f / TX;
      buf[f] = base[(long long)j * lg.N2 + t];
    }
    __syncthreads();
    lds_fft_chunked<T, emax_of<T>(), INV>(buf, plan, TX, 1, TX, false, tw, 1);
    for (int f = threadIdx.x; f < n; f += kThreads) {
      const int t = f % TX, j = f / TX;
      base[(long long)j * lg.N2 + t] = buf[f];
    }
  }
}

// ----------------------------------------------------------------------------
// P3: fused x pass.  One block owns TY consecutive rows l2 at one l3 and handles
// T1 then T2: load 6 half-spectrum rows (h1 = 0..N1/2) per row, C2R of length N1
// as a complex transform of length M = N1/2, constitutive law per voxel,
// R2C back (with the 1/N of eq. FT), store.  FP64 partials of <sigma>.
// ----------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void constitutive(const T* __restrict__ C, const double* Eb,
                                             const T (&de)[6], T (&s)[6]) {
  T g[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) g[c] = (T)Eb[c] + de[c];
  g[3] *= (T)2; g[4] *= (T)2; g[5] *= (T)2;  // engineering shears
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T acc = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += C[i * 6 + j] * g[j];
    s[i] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_xpass(const Desc* __restrict__ descs,
                                                    const int* __restrict__ active, XGeo xg,
                                                    Plan planM, const cpx<T>* __restrict__ twN1) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  __shared__ double red[6 * 4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int tiles2 = xg.N2 / xg.TY;
  const int l3 = blockIdx.x / tiles2;
  const int l2_0 = (blockIdx.x % tiles2) * xg.TY;
  const int TY = xg.TY, H1 = xg.H1, H1p = xg.H1p, M = xg.M;
  const long long N3N2 = (long long)xg.N3 * xg.N2;
  const long long rowoff = (long long)l3 * xg.N2 + l2_0;
  const T* C = sizeof(T) == 8 ? reinterpret_cast<const T*>(d.C64) : reinterpret_cast<const T*>(d.C32);
  const uint16_t* ph = d.phase + ((long long)l3 * xg.N2 + l2_0) * xg.N1;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int nload = 6 * TY * H1;
  const int nlines = 6 * TY;
  const int kh = M / 2 + 1;  // pair items per line

  for (int half = 0; half < 2; ++half) {
    const cpx<T>* src = reinterpret_cast<const cpx<T>*>(d.spec) + (long long)half * 6 * xg.S;
    for (int f = threadIdx.x; f < nload; f += kThreads) {
      const int r = f % TY, k = (f / TY) % H1, c = f / (TY * H1);
      buf[(c * TY + r) * H1p + k] = src[c * xg.S + k * N3N2 + rowoff + r];
    }
    __syncthreads();
    // C2R split: Z[k] = X[k] + conj(X[M-k]) + i w^k (X[k] - conj(X[M-k])), w = exp(2 pi i / N1)
    for (int it = threadIdx.x; it < nlines * kh; it += kThreads) {
      const int line = it / kh, kk = it - line * kh;
      cpx<T>* X = buf + line * H1p;
      if (kk == 0) {
        const cpx<T> a = X[0], b = conjg(X[M]);
        X[0] = (a + b) + mul_i(a - b);
      } else {
        const int k1 = kk, k2 = M - kk;
        const cpx<T> a = X[k1], b = X[k2];
        const cpx<T> w1 = conjg(twN1[k1]);
        const cpx<T> z1 = (a + conjg(b)) + mul_i(w1 * (a - conjg(b)));
        if (k2 != k1) {
          const cpx<T> w2 = conjg(twN1[k2]);
          X[k2] = (b + conjg(a)) + mul_i(w2 * (b - conjg(a)));
        }
        X[k1] = z1;
      }
    }
    __syncthreads();
    lds_fft_chunked<T, emax_of<T>(), true>(buf, planM, nlines, H1p, 1, true, twN1, 2);
    // constitutive law on voxel pairs (2n, 2n+1): real / imaginary parts
    for (int it = threadIdx.x; it < TY * M; it += kThreads) {
      const int r = it / M, n = it - r * M;
      T ea[6], eb[6], sa[6], sb[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const cpx<T> z = buf[(c * TY + r) * H1p + n];
        ea[c] = z.x;
        eb[c] = z.y;
      }
      const int pa = ph[r * xg.N1 + 2 * n], pb = ph[r * xg.N1 + 2 * n + 1];
      constitutive<T>(C + pa * 36, d.Ebar, ea, sa);
      constitutive<T>(C + pb * 36, d.Ebar, eb, sb);
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
    lds_fft_chunked<T, emax_of<T>(), false>(buf, planM, nlines, H1p, 1, true, twN1, 2);
    // R2C merge: X[k] = (A - i w^-k B)/2 with A = Z[k] + conj(Z[M-k]), B = Z[k] - conj(Z[M-k])
    const T hs = (T)(0.5 * xg.invN);
    for (int it = threadIdx.x; it < nlines * kh; it += kThreads) {
      const int line = it / kh, kk = it - line * kh;
      cpx<T>* Z = buf + line * H1p;
      if (kk == 0) {
        const cpx<T> z = Z[0];
        Z[0] = cpx<T>{(z.x + z.y) * (T)xg.invN, (T)0};
        Z[M] = cpx<T>{(z.x - z.y) * (T)xg.invN, (T)0};
      } else {
        const int k1 = kk, k2 = M - kk;
        const cpx<T> a = Z[k1], b = Z[k2];
        const cpx<T> x1 = scale((a + conjg(b)) - mul_i(twN1[k1] * (a - conjg(b))), hs);
        if (k2 != k1) Z[k2] = scale((b + conjg(a)) - mul_i(twN1[k2] * (b - conjg(a))), hs);
        Z[k1] = x1;
      }
    }
    __syncthreads();
    cpx<T>* dst = reinterpret_cast<cpx<T>*>(d.spec) + (long long)half * 6 * xg.S;
    for (int f = threadIdx.x; f < nload; f += kThreads) {
      const int r = f % TY, k = (f / TY) % H1, c = f / (TY * H1);
      dst[c * xg.S + k * N3N2 + rowoff + r] = buf[(c * TY + r) * H1p + k];
    }
    __syncthreads();
  }
  block_sum<6>(acc, red);
  if (threadIdx.x == 0) {
    double* p = d.part_sig + (long long)blockIdx.x * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c] = acc[c];
  }
}

// ----------------------------------------------------------------------------
// P5: equilibrium residual, Green operator, update (eqs. Green_tensor, basic_scheme_dep_2)
// MODE 0: u[1-parity] = u[parity] - Omega r
// MODE 1: FP64 sweep of the anchor: store r in r32, no update
// MODE 2: refinement inner step: r += r32, u[1-parity] = u[parity] - Omega r
// ----------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_contract(const Desc* __restrict__ descs,
                                                       const int* __restrict__ active, int parity,
                                                       Geo g, const cpx<double>* __restrict__ tw1,
                                                       const cpx<double>* __restrict__ tw2,
                                                       const cpx<double>* __restrict__ tw3) {
  __shared__ double red[4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
  double part[1] = {0.0};
  if (idx < g.S) {
    const int h2 = (int)(idx % g.N2);
    const int h3 = (int)((idx / g.N2) % g.N3);
    const int h1 = (int)(idx / ((long long)g.N2 * g.N3));
    cpx<double> D1[3], D2[3];
    symbols(tw1[h1], tw2[h2], tw3[h3], D1, D2);
    cpx<double> s1[6], s2[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      s1[c] = to64(ld<T>(d.spec, c * g.S + idx));
      s2[c] = to64(ld<T>(d.spec, (6 + c) * g.S + idx));
    }
    // (sigma . conj(D))_i with sigma_ij from comps (11,22,33,23,13,12)
    const cpx<double> c1[3] = {conjg(D1[0]), conjg(D1[1]), conjg(D1[2])};
    const cpx<double> c2[3] = {conjg(D2[0]), conjg(D2[1]), conjg(D2[2])};
    cpx<double> r[3];
    r[0] = s1[0] * c1[0] + s1[5] * c1[1] + s1[4] * c1[2] + s2[0] * c2[0] + s2[5] * c2[1] + s2[4] * c2[2];
    r[1] = s1[5] * c1[0] + s1[1] * c1[1] + s1[3] * c1[2] + s2[5] * c2[0] + s2[1] * c2[1] + s2[3] * c2[2];
    r[2] = s1[4] * c1[0] + s1[3] * c1[1] + s1[2] * c1[2] + s2[4] * c2[0] + s2[3] * c2[1] + s2[2] * c2[2];
    if (MODE == 2) {
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = r[c] + to64(ld<float>(d.r32, c * g.S + idx));
    }
    const double w = (h1 == 0 || 2 * h1 == g.N1) ? 1.0 : 2.0;
    part[0] = 0.25 * w * (r[0].x * r[0].x + r[0].y * r[0].y + r[1].x * r[1].x + r[1].y * r[1].y +
                          r[2].x * r[2].x + r[2].y * r[2].y);
    if (MODE == 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) st<float>(d.r32, c * g.S + idx, fr64<float>(r[c]));
    } else {
      // K_il = sum_jk C0_ijkl M_jk,  M_jk = 2 Re(conj(D_j) D_k)
      double Mjk[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k) Mjk[j][k] = 2.0 * (D1[j].x * D1[k].x + D1[j].y * D1[k].y);
      double K[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          double a = 0.0;
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) a += d.C0[((i * 3 + j) * 3 + k) * 3 + l] * Mjk[j][k];
          K[i][l] = a;
        }
      const bool sing = (h1 == 0 && h2 == 0 && h3 == 0) ||
                        (2 * h1 == g.N1 && 2 * h2 == g.N2 && 2 * h3 == g.N3);
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
      const void* uin = d.u[parity];
      void* uout = d.u[1 - parity];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const cpx<double> dw = {O[i][0] * r[0].x + O[i][1] * r[1].x + O[i][2] * r[2].x,
                                O[i][0] * r[0].y + O[i][1] * r[1].y + O[i][2] * r[2].y};
        const cpx<double> un = to64(ld<T>(uin, i * g.S + idx)) - dw;
        st<T>(uout, i * g.S + idx, fr64<T>(un));
      }
    }
  }
  block_sum<1>(part, red);
  if (threadIdx.x == 0) d.part_res[blockIdx.x] = part[0];
}

// ----------------------------------------------------------------------------
// Fixed-order sums of the partials and the stop rule (eqs. L2-norm, tolerance).
// MODE 0: plain iteration on u.  MODE 1: FP64 sweep (measure only).
// MODE 2: inner refinement iteration (stop at ST_REF or on stagnation).
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_finalize(const Desc* __restrict__ descs,
                                                       const int* __restrict__ active, FinGeo fg) {
  __shared__ double red[7 * 4];
  const Desc& d = descs[active[blockIdx.x]];
  if (problem_done(d)) return;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  if (fg.mode != 2) {
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
  if (fg.mode == 2) {
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
    if (reached || bad || stalled || k + 1 >= fg.inner_max) {
      s[ST_DONE] = bad ? 3.0 : 1.0;
      s[ST_ITERS] = k + 1;       // inner updates applied
      s[ST_PARITY] = 1 - fg.parity;
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
  if (fg.mode == 1) return;  // the host decides after a sweep
  const bool stop = d.fixed_iters >= 0 ? (k >= d.fixed_iters) : (err < d.tol);
  const bool bad = !(err == err) || isinf(err) || (k > 0 && err > 1e3 * s[ST_FIRST_ERR]);
  if (stop || bad || k >= d.max_iters) {
    s[ST_DONE] = bad ? 3.0 : (stop ? 1.0 : 2.0);
    s[ST_ITERS] = k;
    s[ST_PARITY] = fg.parity;
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
hipError_t launch_expand(const Desc* descs, const int* active, int nact, int parity, int src,
                         const Geo& g, const void* tw1, const void* tw2, const void* tw3,
                         hipStream_t s) {
  dim3 grid((unsigned)((g.S + kThreads - 1) / kThreads), nact);
  hipLaunchKernelGGL(k_expand<T>, grid, dim3(kThreads), 0, s, descs, active, parity, src, g,
                     (const cpx<double>*)tw1, (const cpx<double>*)tw2, (const cpx<double>*)tw3);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lines(const Desc* descs, const int* active, int nact, const LinesGeo& lg,
                        const Plan& plan, const void* tw, bool inv, hipStream_t s) {
  unsigned nblk;
  if (lg.mode == 0) nblk = (unsigned)((lg.nlines + lg.TX - 1) / lg.TX);
  else nblk = (unsigned)((long long)lg.tiles_per_plane * (lg.nlines));  // nlines = planes for mode 1
  const size_t shm = (size_t)lg.TX * lg.L * sizeof(cpx<T>);
  dim3 grid(nblk, nact);
  if (inv)
    hipLaunchKernelGGL((k_lines<T, true>), grid, dim3(kThreads), shm, s, descs, active, lg, plan,
                       (const cpx<T>*)tw);
  else
    hipLaunchKernelGGL((k_lines<T, false>), grid, dim3(kThreads), shm, s, descs, active, lg, plan,
                       (const cpx<T>*)tw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xpass(const Desc* descs, const int* active, int nact, const XGeo& xg,
                        const Plan& planM, const void* twN1, hipStream_t s) {
  const size_t shm = (size_t)6 * xg.TY * xg.H1p * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY)), nact);
  hipLaunchKernelGGL(k_xpass<T>, grid, dim3(kThreads), shm, s, descs, active, xg, planM,
                     (const cpx<T>*)twN1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_contract(int mode, const Desc* descs, const int* active, int nact, int parity,
                           const Geo& g, const void* tw1, const void* tw2, const void* tw3,
                           hipStream_t s) {
  dim3 grid((unsigned)((g.S + kThreads - 1) / kThreads), nact);
  const cpx<double>* a = (const cpx<double>*)tw1;
  const cpx<double>* b = (const cpx<double>*)tw2;
  const cpx<double>* c = (const cpx<double>*)tw3;
  if (mode == 0)
    hipLaunchKernelGGL((k_contract<T, 0>), grid, dim3(kThreads), 0, s, descs, active, parity, g, a, b, c);
  else if (mode == 1)
    hipLaunchKernelGGL((k_contract<T, 1>), grid, dim3(kThreads), 0, s, descs, active, parity, g, a, b, c);
  else
    hipLaunchKernelGGL((k_contract<T, 2>), grid, dim3(kThreads), 0, s, descs, active, parity, g, a, b, c);
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

template hipError_t launch_expand<double>(const Desc*, const int*, int, int, int, const Geo&, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_expand<float>(const Desc*, const int*, int, int, int, const Geo&, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_lines<double>(const Desc*, const int*, int, const LinesGeo&, const Plan&, const void*, bool, hipStream_t);
template hipError_t launch_lines<float>(const Desc*, const int*, int, const LinesGeo&, const Plan&, const void*, bool, hipStream_t);
template hipError_t launch_xpass<double>(const Desc*, const int*, int, const XGeo&, const Plan&, const void*, hipStream_t);
template hipError_t launch_xpass<float>(const Desc*, const int*, int, const XGeo&, const Plan&, const void*, hipStream_t);
template hipError_t launch_contract<double>(int, const Desc*, const int*, int, int, const Geo&, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_contract<float>(int, const Desc*, const int*, int, int, const Geo&, const void*, const void*, const void*, hipStream_t);

}  // namespace hz
