// HIP kernels (gfx950) of the stencil form of the iteration: 3-field z and x
// transforms around the real-space strain / constitutive / corner-force kernel.
#include <type_traits>

#include "hz_device.h"

namespace hz {

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

// The iteration keeps a stencil-form displacement (3 comps, FP64) in the mixed domain
// [3][h1][l3][h2]: its inverse z transform.  Conversion in place, one tile of TX
// columns of one h1 plane per block: INV, u(q) -> mixed domain (a solve that starts
// from a given displacement); otherwise mixed domain -> u(q), the forward transform
// scaled by 1/N3 (a finished problem's reported iterate).
template <bool INV>
__global__ __launch_bounds__(kThreads) void k_zconv3(cpx<double>* __restrict__ u, ZGeo zg,
                                                     const Plan plan3v,
                                                     const cpx<double>* __restrict__ tw3, double scale) {
  const Plan* plan3 = &plan3v;  // kernel argument (scalar loads)

  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TX = zg.TX, N2 = zg.N2, N3 = zg.N3;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int h1 = tile / zg.tiles;
  const int h2_0 = (tile % zg.tiles) * TX;
  const int lines = 3 * TX;
  cpx<double>* buf = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* twl = buf + lines * N3;
  stage_table(twl, tw3, N3);
  __syncthreads();
  const LdsAcc<double> lds{buf, 1, lines};
  const GblAcc<double> g{glb(u) + (long long)h1 * N3 * N2 + h2_0, (int)zg.S, TX, 1, N2};
  if (INV) {
    // in place: a single pass owns whole lines; otherwise every read precedes a barrier
    fft_lines<double, emax<double>(), true>(*plan3, lines, zg.rLines, false, twl, 1, lds, g, g);
    return;
  }
  fft_lines<double, emax<double>(), false>(*plan3, lines, zg.rLines, false, twl, 1, lds, g, lds);
  __syncthreads();
  for (int e = threadIdx.x; e < lines * N3; e += kThreads) {
    const int l3 = fdiv(e, zg.rLines);
    const cpx<double> v = buf[e];
    g.put(e - l3 * lines, l3, {v.x * scale, v.y * scale});
  }
}

// C2R along x of u (slot 0 -> slot 3 real rows): split + first inverse pass (the
// smallest power-of-two radix of N1/2), middle passes, last pass to HBM.
// R0: the plan's first radix (one instantiation each, so the register budget is that
// of the radix actually used)
template <typename T, int R0>
__global__ __launch_bounds__(kThreads) void k_xc2r(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                   XGeo xg, const Plan planXiv,
                                                   const cpx<T>* __restrict__ twN1) {
  const Plan* planXi = &planXiv;  // kernel argument (scalar loads)

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
  stage_table(twl, twN1, xg.N1);
  __syncthreads();
  HZ_GLB cpx<T>* spec = glb(reinterpret_cast<cpx<T>*>(d.spec));
  const Plan& pi = *planXi;
  const int np = pi.np;
  xf_load<T, R0, 3>(xg, spec + row0, buf, twl);
  __syncthreads();
  const LdsAcc<T> lds{buf, xg.H1p, 1};
  int Ns = R0;
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

// R2C along x of the corner force g (slot 6 real rows -> slot 9), with 1/N.
// RL: the plan's last radix (the merge pass).
template <typename T, int RL>
__global__ __launch_bounds__(kThreads) void k_xr2c(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                   XGeo xg, const Plan planXfv,
                                                   const cpx<T>* __restrict__ twN1) {
  const Plan* planXf = &planXfv;  // kernel argument (scalar loads)

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
  stage_table(twl, twN1, xg.N1);
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
  xf_store<T, RL, 3>(xg, spec + 9 * xg.S + row0, buf, twl);
}

// corner o in {0,-1}^3 coded as bits (bit a set: o_a = 0, clear: o_a = -1);
// T1 takes the corners with an even number of -1 offsets
__device__ __forceinline__ int tet_of(int o) { return ((o & 1) + ((o >> 1) & 1) + ((o >> 2) & 1)) & 1 ? 0 : 1; }

// strain of tetrahedron k of one voxel from its 4 corners (u4[i] = corner o_i of Tk,
// in increasing corner code).  The weights w(o) pair the corners: with
// Tk = 1 (codes 000, 011, 101, 110): a = u1 - u0, b = u2 - u3,
// Tk = 0 (codes 001, 010, 100, 111): a = u3 - u2, b = u0 - u1,
// the gradient rows are 2 G_x = a + b, 2 G_y = a - b, 2 G_z = (u2 + u3) - (u0 + u1).
template <typename T, int K>
__device__ __forceinline__ void stencil_strain_k(const T (&u4)[4][3], T (&e)[6]) {
  T H[3][3];  // H[a][j] = 2 du_j/dx_a
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T a = K ? u4[1][j] - u4[0][j] : u4[3][j] - u4[2][j];
    const T b = K ? u4[2][j] - u4[3][j] : u4[0][j] - u4[1][j];
    H[0][j] = a + b;
    H[1][j] = a - b;
    H[2][j] = (u4[2][j] + u4[3][j]) - (u4[0][j] + u4[1][j]);
  }
  e[0] = (T)0.5 * H[0][0];
  e[1] = (T)0.5 * H[1][1];
  e[2] = (T)0.5 * H[2][2];
  e[3] = (T)0.25 * (H[1][2] + H[2][1]);
  e[4] = (T)0.25 * (H[0][2] + H[2][0]);
  e[5] = (T)0.25 * (H[0][1] + H[1][0]);
}

// sigma^Tk of one voxel of an isotropic phase
template <typename T, bool EIG, int K>
__device__ __forceinline__ void stencil_sigma_iso_k(const Mean<T>& Mn, int ph, cpx<T> lm, const T (&u4)[4][3],
                                                    T (&out)[6]) {
  T e[6];
  stencil_strain_k<T, K>(u4, e);
  constitutive_iso<EIG, T>(lm.x, lm.y, Mn, ph, e, out);
}

// Strain, constitutive law and corner force in real space.  A block owns a
// kStX x kStY column of corners over TZ planes and streams along z: at voxel
// plane p the corner planes p-1 and p sit in LDS (ring of two); for T1 and then T2
// it computes sigma^Tk of the voxel plane (one halo voxel on the + side in x and y)
// and the corners gather it, which completes the force of corner plane p-1 and
// starts that of corner plane p.  Corner plane p+1
// is fetched into registers one step ahead, so its latency overlaps the work.
// Occupancy: isotropic phases keep one tetrahedron's stresses in LDS at a time (35 KB
// per block in FP64), which lets 4 blocks share a CU.  The anisotropic variants, held
// to 3 waves per SIMD by their registers anyway, compute both tetrahedra of a voxel
// in one stage (50 KB): the 21 stiffness entries are loaded once per voxel and a
// z step has 2 barriers instead of 4.  The register bounds below are the largest that
// compile without spills (FP64: 4 waves per SIMD for isotropic phases without
// eigenstrains, 3 otherwise; FP32: 5 for the isotropic variant without eigenstrains).
template <typename T, bool ISO, bool EIG>
__global__ __launch_bounds__(kThreads, (ISO && !EIG) ? (sizeof(T) == 4 ? 5 : 4) : (sizeof(T) == 8 ? 3 : 1)) void k_stencil(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                      SGeo sg) {
  constexpr int UX = kStX + 2, UY = kStY + 2, VX = kStX + 1, VY = kStY + 1;
  constexpr int UP = 3 * UY * UX;                      // corner values per plane
  constexpr int NL = (UP + kThreads - 1) / kThreads;   // per thread
  constexpr bool PAIR = !ISO;                          // both tetrahedra per stage
  __shared__ T ub[2][UP];                              // [slot][c][yy][xx]
  __shared__ T sb[PAIR ? 2 : 1][6][VY][VX];            // sigma of one (or both) tetrahedra
  __shared__ double red[6 * 4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d) || (d.iso != 0) != ISO || (d.tau64 != nullptr) != EIG) return;
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
  const Mean<T> Mn = mean_state<T>(d);
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
  // this thread's voxels (in-tile coordinates) and their in-plane phase-map offsets
  const int nv = (wx + 1) * (wy + 1);
  int voff[2], vxs[2], vys[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int v = tid + k * kThreads;
    vys[k] = v / (wx + 1);
    vxs[k] = v - vys[k] * (wx + 1);
    int gx = x0 + vxs[k], gy = y0 + vys[k];
    while (gx >= N1) gx -= N1;
    while (gy >= N2) gy -= N2;
    voff[k] = gy * N1 + gx;
  }
  // the fetch of a plane brings its corners and the phase ids of its voxels; the
  // stiffness entries of the isotropic case follow one step later, so no load sits
  // on a step's critical path
  T rg[NL];
  int rph[2] = {0, 0}, cph[2] = {0, 0};
  cpx<T> clm[2] = {{0, 0}, {0, 0}};
  auto fetch = [&](int q) {
    const int qq = q < 0 ? q + N3 : (q >= N3 ? q - N3 : q);
    const HZ_GLB T* base = ur + (long long)qq * NP;
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (loff[k] >= 0) rg[k] = base[loff[k]];
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (tid + k * kThreads < nv) rph[k] = ph[(long long)qq * NP + voff[k]];
  };
  auto stash = [&](int slot) {
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (loff[k] >= 0) ub[slot][tid + k * kThreads] = rg[k];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      cph[k] = rph[k];
      if (ISO && tid + k * kThreads < nv) clm[k] = gld(reinterpret_cast<const HZ_GLB cpx<T>*>(C) + cph[k]);
    }
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
    T g1[3] = {0, 0, 0}, g0[3] = {0, 0, 0};
    if constexpr (PAIR) {
      // the 4 corners of tetrahedron k of voxel (vx, vy) of plane p
      auto corners = [&](auto kc, int vx, int vy, T (&u4)[4][3]) {
        constexpr int k = decltype(kc)::value;
        int i = 0;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
          if (tet_of(o) != k) continue;
          const int ix = vx + ((o & 1) ? 1 : 0), iy = vy + ((o & 2) ? 1 : 0);
          const int slot = (o & 4) ? cur : prv;
#pragma unroll
          for (int j = 0; j < 3; ++j) u4[i][j] = ub[slot][(j * UY + iy) * UX + ix];
          ++i;
        }
      };
      // corner (cx, cy) receives sigma^Tk of voxel (cx - o1, cy - o2) for o in Tk;
      // with w(o) = +-1/2 the sums carry 2 sigma.w and the 1/2 is applied at the store
      auto gather = [&](auto kc, const T (&sk)[6][VY][VX]) {
        constexpr int k = decltype(kc)::value;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
          if (tet_of(o) != k) continue;
          const int vx = cx + ((o & 1) ? 0 : 1), vy = cy + ((o & 2) ? 0 : 1);
          auto pm = [](bool plus, T x) { return plus ? x : -x; };
          const bool p0 = o & 1, p1 = o & 2, p2 = o & 4;
          const T s0 = sk[0][vy][vx], s1 = sk[1][vy][vx], s2 = sk[2][vy][vx];
          const T s3 = sk[3][vy][vx], s4 = sk[4][vy][vx], s5 = sk[5][vy][vx];
          const T f0 = pm(p0, s0) + pm(p1, s5) + pm(p2, s4);
          const T f1 = pm(p0, s5) + pm(p1, s1) + pm(p2, s3);
          const T f2 = pm(p0, s4) + pm(p1, s3) + pm(p2, s2);
          if (o & 4) {
            g0[0] += f0; g0[1] += f1; g0[2] += f2;
          } else {
            g1[0] += f0; g1[1] += f1; g1[2] += f2;
          }
        }
      };
      using K0 = std::integral_constant<int, 0>;
      using K1 = std::integral_constant<int, 1>;
      __syncthreads();  // plane p stashed, the previous gather done with sb
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        if (tid + sl * kThreads >= nv) continue;
        const int vy = vys[sl], vx = vxs[sl];
        T e0[6], e1[6];
        {
          T u4[4][3];
          corners(K0{}, vx, vy, u4);
          stencil_strain_k<T, 0>(u4, e0);
        }
        {
          T u4[4][3];
          corners(K1{}, vx, vy, u4);
          stencil_strain_k<T, 1>(u4, e1);
        }
        T s0[6], s1[6];
        constitutive_pair<EIG, T>(C + cph[sl] * 24, Mn, cph[sl], e0, e1, s0, s1);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          sb[0][c][vy][vx] = s0[c];
          sb[PAIR ? 1 : 0][c][vy][vx] = s1[c];
        }
        if (vx < wx && vy < wy && p < z0 + wz) {
#pragma unroll
          for (int c = 0; c < 6; ++c) sacc[c] += 0.5 * ((double)s0[c] + (double)s1[c]);
        }
      }
      __syncthreads();
      if (own) {
        gather(K0{}, sb[0]);
        gather(K1{}, sb[PAIR ? 1 : 0]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        __syncthreads();  // k = 0: plane p stashed; k = 1: the gather of tetrahedron 0 is done with sb
        // sigma^Tk of voxel plane p over (wx+1) x (wy+1) voxels
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          if (tid + sl * kThreads >= nv) continue;
          const int vy = vys[sl], vx = vxs[sl];
          T u4[4][3];
          int i = 0;
#pragma unroll
          for (int o = 0; o < 8; ++o) {
            if (tet_of(o) != k) continue;
            const int ix = vx + ((o & 1) ? 1 : 0), iy = vy + ((o & 2) ? 1 : 0);
            const int slot = (o & 4) ? cur : prv;
#pragma unroll
            for (int j = 0; j < 3; ++j) u4[i][j] = ub[slot][(j * UY + iy) * UX + ix];
            ++i;
          }
          T out[6];
          if (k == 0) stencil_sigma_iso_k<T, EIG, 0>(Mn, cph[sl], clm[sl], u4, out);
          else stencil_sigma_iso_k<T, EIG, 1>(Mn, cph[sl], clm[sl], u4, out);
#pragma unroll
          for (int c = 0; c < 6; ++c) sb[0][c][vy][vx] = out[c];
          if (vx < wx && vy < wy && p < z0 + wz) {
#pragma unroll
            for (int c = 0; c < 6; ++c) sacc[c] += 0.5 * (double)out[c];
          }
        }
        __syncthreads();
        if (own) {
          // corner (cx, cy) receives sigma^Tk of voxel (cx - o1, cy - o2) for o in Tk;
          // with w(o) = +-1/2 the sums carry 2 sigma.w and the 1/2 is applied at the store
#pragma unroll
          for (int o = 0; o < 8; ++o) {
            if (tet_of(o) != k) continue;
            const int vx = cx + ((o & 1) ? 0 : 1), vy = cy + ((o & 2) ? 0 : 1);
            auto pm = [](bool plus, T x) { return plus ? x : -x; };
            const bool p0 = o & 1, p1 = o & 2, p2 = o & 4;
            const T s0 = sb[0][0][vy][vx], s1 = sb[0][1][vy][vx], s2 = sb[0][2][vy][vx];
            const T s3 = sb[0][3][vy][vx], s4 = sb[0][4][vy][vx], s5 = sb[0][5][vy][vx];
            const T f0 = pm(p0, s0) + pm(p1, s5) + pm(p2, s4);
            const T f1 = pm(p0, s5) + pm(p1, s1) + pm(p2, s3);
            const T f2 = pm(p0, s4) + pm(p1, s3) + pm(p2, s2);
            if (o & 4) {
              g0[0] += f0; g0[1] += f1; g0[2] += f2;
            } else {
              g1[0] += f0; g1[1] += f1; g1[2] += f2;
            }
          }
        }
      }
    }
    if (own) {
      if (p > z0) {
        const int at = (p - 1) * NP + (y0 + cy) * N1 + (x0 + cx);
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[(long long)j * Nn + at] = (T)0.5 * (acc[j] + g1[j]);
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
// launch wrappers
// ----------------------------------------------------------------------------
hipError_t launch_zconv3(void* u, bool inverse, const ZGeo& zg, const Plan* plan3, const void* tw3, hipStream_t s) {
  const size_t shm = ((size_t)3 * zg.TX * zg.N3 + zg.N3) * sizeof(cpx<double>);
  const dim3 grid((unsigned)(zg.H1 * zg.tiles));
  cpx<double>* p = reinterpret_cast<cpx<double>*>(u);
  const cpx<double>* tw = (const cpx<double>*)tw3;
  if (inverse) hipLaunchKernelGGL(k_zconv3<true>, grid, dim3(kThreads), shm, s, p, zg, *plan3, tw, 1.0);
  else hipLaunchKernelGGL(k_zconv3<false>, grid, dim3(kThreads), shm, s, p, zg, *plan3, tw, 1.0 / zg.N3);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xc2r(const Desc* descs, const int* active, int nact, const XGeo& xg, const Plan* planXi, int r0,
                       const void* twN1, hipStream_t s) {
  const size_t shm = ((size_t)3 * xg.TY * xg.H1p + xg.N1) * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY)), nact);
  const cpx<T>* tw = (const cpx<T>*)twN1;
  switch (r0) {
    case 16: hipLaunchKernelGGL((k_xc2r<T, 16>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, tw); break;
    case 8: hipLaunchKernelGGL((k_xc2r<T, 8>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, tw); break;
    case 4: hipLaunchKernelGGL((k_xc2r<T, 4>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, tw); break;
    case 2: hipLaunchKernelGGL((k_xc2r<T, 2>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xr2c(const Desc* descs, const int* active, int nact, const XGeo& xg, const Plan* planXf, int rl,
                       const void* twN1, hipStream_t s) {
  const size_t shm = ((size_t)3 * xg.TY * xg.H1p + xg.N1) * sizeof(cpx<T>);
  dim3 grid((unsigned)(xg.N3 * (xg.N2 / xg.TY)), nact);
  const cpx<T>* tw = (const cpx<T>*)twN1;
  switch (rl) {
    case 16: hipLaunchKernelGGL((k_xr2c<T, 16>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXf, tw); break;
    case 8: hipLaunchKernelGGL((k_xr2c<T, 8>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXf, tw); break;
    case 4: hipLaunchKernelGGL((k_xr2c<T, 4>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXf, tw); break;
    case 2: hipLaunchKernelGGL((k_xr2c<T, 2>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXf, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const Desc* descs, const int* active, int nact, int kind, const SGeo& sg, hipStream_t s) {
  dim3 grid((unsigned)(sg.tx * sg.ty * sg.tz), nact);
  switch (kind) {
    case KIND_ISO: hipLaunchKernelGGL((k_stencil<T, true, false>), grid, dim3(kThreads), 0, s, descs, active, sg); break;
    case KIND_ISO | KIND_EIG: hipLaunchKernelGGL((k_stencil<T, true, true>), grid, dim3(kThreads), 0, s, descs, active, sg); break;
    case 0: hipLaunchKernelGGL((k_stencil<T, false, false>), grid, dim3(kThreads), 0, s, descs, active, sg); break;
    default: hipLaunchKernelGGL((k_stencil<T, false, true>), grid, dim3(kThreads), 0, s, descs, active, sg); break;
  }
  return hipGetLastError();
}

template hipError_t launch_xc2r<double>(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template hipError_t launch_xc2r<float>(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template hipError_t launch_xr2c<double>(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template hipError_t launch_xr2c<float>(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template hipError_t launch_stencil<double>(const Desc*, const int*, int, int, const SGeo&, hipStream_t);
template hipError_t launch_stencil<float>(const Desc*, const int*, int, int, const SGeo&, hipStream_t);

}  // namespace hz
