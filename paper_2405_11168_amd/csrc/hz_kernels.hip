// HIP kernels (gfx950) of one iteration of the tetrahedral-stencil basic scheme.
//
// Spectra are stored [comp][h1][h3][h2] (h1 in [0, N1/2], h2 fastest).  Iteration
// (Algorithm 1, Sec. 2.6):
//   k_zexp      u(q) (3 comps) -> inverse z transform of the 3 displacement comps,
//               then the 12 strain comps eps^T1 = D~ (x)_s u, eps^T2 = D~2 (x)_s u
//               formed in the mixed (h1, h2, l3) domain
//   k_yline     inverse y (12 comps)
//   k_xpass     per (l3, l2-tile): C2R along x, sigma = C(phase):(Ebar + eps - eps0), R2C along x,
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
#include "hz_device.h"

namespace hz {

// ----------------------------------------------------------------------------
// P1: inverse z transform of u (3 comps) and the 12 strain spectra
// (eqs. desp_T1_dep_Q, desp_T2_dep_Q) as 2-tap combinations along l3.
// Tile: TX adjacent h2 columns of one h1 plane.  LDS: 3*TX lines x N3, then twiddles.
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zexp(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                   ZGeo zg, const Plan plan3v, const cpx<T>* __restrict__ tw3T,
                                                   const cpx<double>* __restrict__ tw1,
                                                   const cpx<double>* __restrict__ tw2) {
  const Plan* plan3 = &plan3v;  // kernel argument (scalar loads)

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
  stage_table(twl, tw3T, N3);
  const long long plane = (long long)h1 * N3 * N2 + h2_0;
  const LdsAcc<T> lds{buf, 1, lines};
  const void* usrc = d.src == 1 ? d.u64 : u_slot(d, cur_slot(d));
  const GblAcc<T> src{glb(reinterpret_cast<cpx<T>*>(const_cast<void*>(usrc))) + plane, (int)zg.S, TX, 1, N2};
  fft_lines<T, emax<T>(), true>(*plan3, lines, zg.rLines, false, twl, 1, lds, src, lds);
  __syncthreads();
  HZ_GLB cpx<T>* out = glb(reinterpret_cast<cpx<T>*>(d.spec)) + plane;
  const cpx<double> t1 = tw1[h1];
  const bool rot = d.green == GREEN_ROTATED;
  for (int e = threadIdx.x; e < TX * N3; e += kThreads) {
    const int l3 = fdiv(e, zg.rTX), col = e - l3 * TX;
    const int lm = l3 == 0 ? N3 - 1 : l3 - 1;
    cpx<double> a1[3], b1[3], a2[3], b2[3];
    affine_symbols(t1, tw2[h2_0 + col], a1, b1, a2, b2);
    if (rot) {
      rotated_mean(a1, a2);
      rotated_mean(b1, b2);
    }
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
// P1 of the strain-based form (Algorithm 2): the iterate is the 12 strain spectra.
// The contraction of the previous iteration left w = Omega r in u[0]; here
//   eps^Tk <- eps^Tk - D~k (x)_s w      (Gamma.r = D (x)_s (Omega r), eq.
//   Lippmann_Schwinger_strain_3; D~2 carries the sign of the T2 update)
// is applied in q-space, the updated strains are stored back, and they are
// transformed along z into the work spectra, 3 components at a time.
// d.cmode 3 with k = 0 starts from zero strains; any other cmode (the output
// pass) transforms the stored strains unchanged.
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zstrain(const Desc* __restrict__ descs,
                                                      const int* __restrict__ active, ZGeo zg,
                                                      const Plan plan3v,
                                                      const cpx<T>* __restrict__ tw3T,
                                                      const cpx<double>* __restrict__ tw1,
                                                      const cpx<double>* __restrict__ tw2,
                                                      const cpx<double>* __restrict__ tw3) {
  const Plan* plan3 = &plan3v;  // kernel argument (scalar loads)

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
  stage_table(twl, tw3T, N3);
  const bool iter = d.cmode == 3;
  const int k = (int)status_ro(d)[ST_K];
  const bool fresh = iter && k == 0, apply = iter && k > 0;
  const long long plane = (long long)h1 * N3 * N2 + h2_0;
  HZ_GLB cpx<T>* st = glb(reinterpret_cast<cpx<T>*>(d.state)) + plane;
  const HZ_GLB cpx<T>* wv = glb(reinterpret_cast<const cpx<T>*>(d.u[0])) + plane;
  const LdsAcc<T> lds{buf, 1, lines};
  const cpx<double> t1 = tw1[h1];
  const int ne = TX * N3;
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const int tet = g >> 1, c0 = (g & 1) * 3, f0 = tet * 6 + c0;  // first of this group's 3 fields
    __syncthreads();  // twiddles, and the previous group's transform is done with the LDS lines
    for (int e = threadIdx.x; e < ne; e += kThreads) {
      const int h3 = fdiv(e, zg.rTX), col = e - h3 * TX;
      const int o = h3 * N2 + col;
      cpx<T> v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] = fresh ? cpx<T>{0, 0} : gld(st + (f0 + c) * zg.S + o);
      if (apply) {
        cpx<double> D1[3], D2[3];
        symbols(t1, tw2[h2_0 + col], tw3[h3], D1, D2);
        const cpx<double>* D = tet == 0 ? D1 : D2;
        cpx<double> w[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) w[a] = to64(gld(wv + a * zg.S + o));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          // (D (x)_s w) in comps (11,22,33,23,13,12)
          const int comp = c0 + c;
          const int i = comp < 3 ? comp : (comp == 3 ? 1 : 0);
          const int j = comp < 3 ? comp : (comp == 5 ? 1 : 2);
          const cpx<double> s = comp < 3 ? D[i] * w[j] : scale(D[i] * w[j] + D[j] * w[i], 0.5);
          v[c] = fr64<T>(to64(v[c]) - s);
        }
      }
      if (iter) {
#pragma unroll
        for (int c = 0; c < 3; ++c) gst(st + (f0 + c) * zg.S + o, v[c]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) lds.put(c * TX + col, h3, v[c]);
    }
    __syncthreads();
    const GblAcc<T> dst{glb(reinterpret_cast<cpx<T>*>(d.spec)) + plane + (long long)f0 * zg.S, (int)zg.S, TX, 1, N2};
    fft_lines<T, emax<T>(), true>(*plan3, lines, zg.rLines, false, twl, 1, lds, lds, dst);
  }
}

// ----------------------------------------------------------------------------
// y pass: TX contiguous rows of length N2; first radix pass straight from HBM,
// last radix pass straight to HBM, twiddles in LDS.
// ----------------------------------------------------------------------------
template <typename T, bool INV>
__global__ __launch_bounds__(kThreads) void k_yline(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                    YGeo yg, const Plan plan2v, const cpx<T>* __restrict__ tw2T) {
  const Plan* plan2 = &plan2v;  // kernel argument (scalar loads)

  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int N2 = yg.N2;
  const long long t0 = (long long)blockIdx.x * yg.TX;
  const int lines = (int)((yg.nlines - t0) < yg.TX ? (yg.nlines - t0) : yg.TX);
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = buf + yg.TX * yg.pitch;
  stage_table(twl, tw2T, N2);
  const LdsPad<T> lds{buf, yg.pitch, yg.pshift};
  const GblAcc<T> g{glb(reinterpret_cast<cpx<T>*>(d.spec)) + yg.off + t0 * N2, N2, 1, 0, 1};
  if (yg.from_state) {
    void* st = d.src == 1 ? d.u64 : u_slot(d, cur_slot(d));
    const GblAcc<T> src{glb(reinterpret_cast<cpx<T>*>(st)) + t0 * N2, N2, 1, 0, 1};
    fft_lines<T, emax<T>(), INV>(*plan2, lines, 0.f, true, twl, 1, lds, src, g);
  } else {
    fft_lines<T, emax<T>(), INV>(*plan2, lines, 0.f, true, twl, 1, lds, g, g);
  }
}

// ----------------------------------------------------------------------------
// P3: fused x pass.  One block owns TY consecutive rows l2 at one l3 and handles
// T1 then T2: load 6 half-spectrum rows (h1 = 0..N1/2) per row, C2R of length N1
// as a complex transform of length M = N1/2, constitutive law per voxel,
// R2C back (with the 1/N of eq. FT), store.  FP64 partials of <sigma>.
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_xpass(const Desc* __restrict__ descs,
                                                    const int* __restrict__ active, XGeo xg,
                                                    const Plan planMv, const cpx<T>* __restrict__ twN1) {
  const Plan* planM = &planMv;  // kernel argument (scalar loads)

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
  stage_table(twl, twN1, xg.N1);
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
  const Mean<T> Mn = mean_state<T>(d);
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
      constitutive_iso<false, T>(la.x, la.y, Mn, pa, ea, sa);
      constitutive_iso<false, T>(lb.x, lb.y, Mn, pb, eb, sb);
    } else {
      constitutive<false, T>(C + pa * 24, Mn, pa, ea, sa);
      constitutive<false, T>(C + pb * 24, Mn, pb, eb, sb);
    }
    if (Mn.tau) {
      eigenstress<true>(Mn, pa, sa);
      eigenstress<true>(Mn, pb, sb);
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
        const double e0 = 0.5 * ((double)Mn.Eb[c] + (double)ea[c]);
        const double e1 = 0.5 * ((double)Mn.Eb[c] + (double)eb[c]);
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

// ISO: every phase of the material is isotropic; EIG: the problem has eigenstrains
// (separate instantiations keep the register budget of each at two waves per SIMD
// in FP64)
template <typename T, bool ISO, bool EIG>
__global__ __launch_bounds__(kThreads) void k_xfused(const Desc* __restrict__ descs,
                                                     const int* __restrict__ active, XGeo xg,
                                                     const Plan planXiv,
                                                     const Plan planXfv,
                                                     const cpx<T>* __restrict__ twN1) {
  const Plan* planXi = &planXiv;  // kernel argument (scalar loads)
  const Plan* planXf = &planXfv;  // kernel argument (scalar loads)

  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[6 * 4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d) || (d.iso != 0) != ISO || (d.tau64 != nullptr) != EIG) return;
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
  stage_table(twl, twN1, xg.N1);
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
    case 4: xf_middle<T, ISO, EIG, 4>(d, xg, buf, twl, ph, acc); break;
    case 2: xf_middle<T, ISO, EIG, 2>(d, xg, buf, twl, ph, acc); break;
    case 5: xf_middle<T, ISO, EIG, 5>(d, xg, buf, twl, ph, acc); break;
    default: xf_middle<T, ISO, EIG, 3>(d, xg, buf, twl, ph, acc); break;
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
// launch wrappers
// ----------------------------------------------------------------------------
template <typename T>
hipError_t launch_zexp(const Desc* descs, const int* active, int nact, const ZGeo& zg, const Plan* plan3,
                       const void* tw3T, const void* tw1, const void* tw2, hipStream_t s) {
  const size_t shm = ((size_t)3 * zg.TX * zg.N3 + zg.N3) * sizeof(cpx<T>);
  dim3 grid((unsigned)(zg.H1 * zg.tiles), nact);
  const hipError_t e = allow_lds(k_zexp<T>, shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zexp<T>, grid, dim3(kThreads), shm, s, descs, active, zg, *plan3, (const cpx<T>*)tw3T,
                     (const cpx<double>*)tw1, (const cpx<double>*)tw2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_yline(const Desc* descs, const int* active, int nact, const YGeo& yg, const Plan* plan2,
                        const void* tw2T, bool inv, hipStream_t s) {
  const size_t shm = ((size_t)yg.TX * yg.pitch + yg.N2) * sizeof(cpx<T>);
  dim3 grid((unsigned)((yg.nlines + yg.TX - 1) / yg.TX), nact);
  if (inv)
    hipLaunchKernelGGL((k_yline<T, true>), grid, dim3(kThreads), shm, s, descs, active, yg, *plan2, (const cpx<T>*)tw2T);
  else
    hipLaunchKernelGGL((k_yline<T, false>), grid, dim3(kThreads), shm, s, descs, active, yg, *plan2, (const cpx<T>*)tw2T);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xpass(const Desc* descs, const int* active, int nact, const XGeo& xg,
                        const Plan* planM, const void* twN1, hipStream_t s) {
  const size_t shm = ((size_t)6 * xg.TY * xg.H1p + xg.N1) * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY) * (xg.half >= 0 ? 1 : 2)), nact);
  hipLaunchKernelGGL(k_xpass<T>, grid, dim3(kThreads), shm, s, descs, active, xg, *planM,
                     (const cpx<T>*)twN1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xfused(const Desc* descs, const int* active, int nact, int kind, const XGeo& xg,
                         const Plan* planXi, const Plan* planXf, const void* twN1, hipStream_t s) {
  const size_t shm = ((size_t)6 * xg.TY * xg.H1p + xg.N1) * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY) * (xg.half >= 0 ? 1 : 2)), nact);
  const cpx<T>* tw = (const cpx<T>*)twN1;
  switch (kind) {
    case KIND_ISO:
      hipLaunchKernelGGL((k_xfused<T, true, false>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, *planXf, tw);
      break;
    case KIND_ISO | KIND_EIG:
      hipLaunchKernelGGL((k_xfused<T, true, true>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, *planXf, tw);
      break;
    case 0:
      hipLaunchKernelGGL((k_xfused<T, false, false>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, *planXf, tw);
      break;
    default:
      hipLaunchKernelGGL((k_xfused<T, false, true>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, *planXf, tw);
      break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zstrain(const Desc* descs, const int* active, int nact, const ZGeo& zg, const Plan* plan3,
                          const void* tw3T, const void* tw1, const void* tw2, const void* tw3, hipStream_t s) {
  const size_t shm = ((size_t)3 * zg.TX * zg.N3 + zg.N3) * sizeof(cpx<T>);
  dim3 grid((unsigned)(zg.H1 * zg.tiles), nact);
  const hipError_t e = allow_lds(k_zstrain<T>, shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zstrain<T>, grid, dim3(kThreads), shm, s, descs, active, zg, *plan3, (const cpx<T>*)tw3T,
                     (const cpx<double>*)tw1, (const cpx<double>*)tw2, (const cpx<double>*)tw3);
  return hipGetLastError();
}

template hipError_t launch_zstrain<double>(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_zstrain<float>(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_zexp<double>(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_zexp<float>(const Desc*, const int*, int, const ZGeo&, const Plan*, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_yline<double>(const Desc*, const int*, int, const YGeo&, const Plan*, const void*, bool, hipStream_t);
template hipError_t launch_yline<float>(const Desc*, const int*, int, const YGeo&, const Plan*, const void*, bool, hipStream_t);
template hipError_t launch_xpass<double>(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_xpass<float>(const Desc*, const int*, int, const XGeo&, const Plan*, const void*, hipStream_t);
template hipError_t launch_xfused<double>(const Desc*, const int*, int, int, const XGeo&, const Plan*, const Plan*, const void*, hipStream_t);
template hipError_t launch_xfused<float>(const Desc*, const int*, int, int, const XGeo&, const Plan*, const Plan*, const void*, hipStream_t);

}  // namespace hz
