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
// smallest power-of-two radix of N1/2, else its smallest odd one), middle passes, last
// pass to HBM; a one-pass plan (N1/2 prime or 1) copies the split pass's lines out.
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
  HZ_GLB cpx<T>* spec = glb(reinterpret_cast<cpx<T>*>(d.spec));
  {
    // the corner-force rows that the stencil kernel accumulates from two blocks (the
    // last corner row of each of its tiles in y) start from zero
    HZ_GLB T* g = reinterpret_cast<HZ_GLB T*>(spec + 6 * xg.S);
    const long long N = (long long)xg.N1 * xg.N2 * xg.N3;
#pragma unroll 1
    for (int r = 0; r < TY; ++r) {
      const int l2 = l2_0 + r;
      if (l2 % kStY != kStY - 1 && l2 != xg.N2 - 1) continue;
      HZ_GLB T* row = g + (long long)(row0 + r) * xg.N1;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        for (int x = threadIdx.x; x < xg.N1; x += kThreads) row[c * N + x] = (T)0;
    }
  }
  __syncthreads();
  const Plan& pi = *planXi;
  const int np = pi.np;
  xf_load<T, R0, 3>(xg, spec + row0, buf, twl);
  __syncthreads();
  const LdsAcc<T> lds{buf, xg.H1p, 1};
  // real row (l3, l2) of comp c as M complex values z[n] = x[2n] + i x[2n+1]
  const int half_n = (xg.N1 / 2) * xg.N2 * xg.N3;
  const GblAcc<T> out{spec + 3 * xg.S + (long long)row0 * M, half_n, TY, M, 1};
  if (np == 1) {
    // one pass (M prime or 1): the split pass left the lines in natural order
#pragma unroll 1
    for (int e = threadIdx.x; e < 3 * TY * M; e += kThreads) {
      const int t = fdiv(e, xg.rM), j = e - t * M;
      out.put(t, j, lds.get(t, j));
    }
    return;
  }
  int Ns = R0;
#pragma unroll 1
  for (int p = 1; p < np - 1; ++p) {
    pass_any<T, emax<T>(), true>(pi.radix[p], M, Ns, 3 * TY, true, twl, 2, lds, lds, true, pi.rLR[p], pi.rNs[p], 0.f);
    __syncthreads();
    Ns *= pi.radix[p];
  }
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
  if (np == 1) {
    // one pass (M prime or 1): the merge pass reads the lines in natural order
#pragma unroll 1
    for (int e = threadIdx.x; e < 3 * TY * M; e += kThreads) {
      const int t = fdiv(e, xg.rM), j = e - t * M;
      lds.put(t, j, in.get(t, j));
    }
    __syncthreads();
    xf_store<T, RL, 3>(xg, spec + 9 * xg.S + row0, buf, twl);
    return;
  }
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

// corner o in {0,-1}^3 coded as bits (bit a set: o_a = 0, clear: o_a = -1).  T1 takes the
// corners with an even number of -1 offsets (codes 001, 010, 100, 111), T2 the others
// (000, 011, 101, 110); the weight of corner o is w(o) = o + (1/2, 1/2, 1/2).

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

// sigma^T1 and sigma^T2 of one voxel from its 8 corners c[o] (o = corner code)
template <typename T, bool ISO, bool EIG>
__device__ __forceinline__ void voxel_sigma(const T (&c)[8][3], const HZ_GLB T* __restrict__ C, cpx<T> lm, int ph,
                                            const Mean<T>& Mn, T (&s1)[6], T (&s2)[6]) {
  T e1[6], e2[6];
  {
    T u4[4][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      u4[0][j] = c[1][j];
      u4[1][j] = c[2][j];
      u4[2][j] = c[4][j];
      u4[3][j] = c[7][j];
    }
    stencil_strain_k<T, 0>(u4, e1);
  }
  {
    T u4[4][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      u4[0][j] = c[0][j];
      u4[1][j] = c[3][j];
      u4[2][j] = c[5][j];
      u4[3][j] = c[6][j];
    }
    stencil_strain_k<T, 1>(u4, e2);
  }
  if constexpr (ISO) {
    constitutive_iso<EIG, T>(lm.x, lm.y, Mn, ph, e1, s1);
    constitutive_iso<EIG, T>(lm.x, lm.y, Mn, ph, e2, s2);
  } else {
    constitutive_pair<EIG, T>(C + ph * 24, Mn, ph, e1, e2, s1, s2);
  }
}

// Rows of a stress for the corner forces: with X, Y, Z the rows of sigma (sigma e_a),
// 2 sigma.w(o) = +-X +-Y +-Z with the signs of o + 1/2; P = X + Y, M = X - Y.
template <typename T>
__device__ __forceinline__ void stress_rows(const T (&s)[6], T (&P)[3], T (&M)[3], T (&Z)[3]) {
  const T X[3] = {s[0], s[5], s[4]}, Y[3] = {s[5], s[1], s[3]};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    P[j] = X[j] + Y[j];
    M[j] = X[j] - Y[j];
  }
  Z[0] = s[4];
  Z[1] = s[3];
  Z[2] = s[2];
}

// Raw buffer access to one plane of a real field: the plane's address sits in a
// buffer resource (scalar registers) and each lane adds a 32-bit byte offset, so no
// 64-bit address is formed per lane; an offset past the plane reads 0 and is not
// written.  Word 3 of the resource is the gfx9 raw-buffer setting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, 0x00020000);
}
__device__ __forceinline__ double buf_ld(double, __amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ float buf_ld(float, __amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                        (int)off, 0, 0);
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}

// Lane shifts across the wavefront (DPP): with kShr1 lane i takes the value of lane
// i - 1, with kShl1 that of lane i + 1; the lane without a source (0, resp. 63) takes
// `edge`.  Every lane of the wave must be active.
constexpr int kShr1 = 0x138, kShl1 = 0x130;
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v, double edge) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(edge), __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(edge), __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v, float edge) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// waves per SIMD the register budget is set for: FP64 needs about 166 VGPRs (3 waves),
// FP32 about 105 (4 waves); no variant spills at these bounds except the anisotropic
// FP64 one with eigenstrains (a few loop-invariant addresses)
template <typename T>
constexpr int stencil_waves() { return sizeof(T) == 8 ? 3 : 4; }
// Strain, constitutive law and corner force in real space.  A block owns a tile of
// 64 x kStY corners in x and y over TZ planes along z: wave w owns corner row y0 + w,
// lane l the corner column x = x0 + l, and the wave streams along z.  At voxel plane p
// a lane holds the 8 corners of voxel (x, y, p) -- its own column and, by a lane shift,
// column x - 1, in its row and the row below (both loaded by the wave), planes p - 1 and
// p -- and computes sigma of both tetrahedra and the voxel's contribution 2 sigma.w(o)
// to each corner x + o.  The contributions to one corner plane are summed per corner
// offset (dx, dy) = (-o1, -o2) over the two voxel planes that touch it, A_dxdy, and
//   g(x, y, p-1) = 1/2 [A00(x, y) + A10(x+1, y) + A01(x, y+1) + A11(x+1, y+1)]:
// A10 and A11 of column x + 1 come by a lane shift, the row y + 1 terms from the wave of
// that row through LDS (one barrier per z step, double buffered).  The voxel column
// right of the tile is computed once per wave before the z loop, with its lanes spread
// over the planes, and the corners of column x0 - 1 are staged there too.  The last
// corner row of a tile takes terms from two blocks: the wave of that row adds its part
// and the first wave of the next tile in y adds the row y + 1 terms, both as atomic adds
// onto a row the C2R kernel has zeroed.  With exactly two addends the result does not
// depend on their order, so every run gives the same bits.
template <typename T, bool ISO, bool EIG>
__global__ __launch_bounds__(kThreads, stencil_waves<T>()) void k_stencil(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                      SGeo sg, int tab_bytes) {
  static_assert(kStX == 64 && kStY * 64 == kThreads, "one wave per corner row");
  // anisotropic phases: the stiffness table in LDS when it fits tab_bytes, so the per-voxel
  // rows are LDS gathers instead of HBM/L2 gathers issued at the point of use
  extern __shared__ __align__(16) unsigned char smem_dyn[];
  cpx<T>* ctab = reinterpret_cast<cpx<T>*>(smem_dyn);
  __shared__ T lh[kStY][kStZ + 2][6];     // u at column x0 - 1: row below (0..2), own row (3..5)
  __shared__ T hr[kStY][kStZ + 1][4][3];  // halo voxel column: contribution to column x0+wx-1, [dy*2 + dz]
  __shared__ T xb[2][kStY][3][64];        // row y + 1 terms of corner row y
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
  const HZ_GLB cpx<T>* Clm = reinterpret_cast<const HZ_GLB cpx<T>*>(C);
  const Mean<T> Mn = mean_state<T>(d);
  const HZ_GLB uint16_t* ph = glb(d.phase);
  const bool tab = !ISO && d.n_phases * 24 * (int)sizeof(T) <= tab_bytes;
  if (tab) {
    for (int i = threadIdx.x; i < d.n_phases * 12; i += kThreads) ctab[i] = gld(Clm + i);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool wact = w < wy, xact = lane < wx;
  const int y = y0 + (wact ? w : 0);  // waves past the tile's last row shadow its first (results unused)
  const int ym = y == 0 ? N2 - 1 : y - 1;
  // lanes past a ragged tile's last column take the voxel column right of the tile
  // (periodic), so the lane after the last one holds that column's terms
  const int x = xact ? x0 + lane : (x0 + wx == N1 ? 0 : x0 + wx);
  auto plane = [&](int q) { return q < 0 ? q + N3 : (q >= N3 ? q - N3 : q); };

  // ---- the corners of column x0 - 1, and the voxel column x0 + wx (periodic), one
  // lane per plane: lane l holds corner plane z0 - 1 + l, l <= wz + 1
  {
    const int xl = x0 == 0 ? N1 - 1 : x0 - 1;
    const int xh = x0 + wx == N1 ? 0 : x0 + wx, xhm = x0 + wx - 1;
    const int l = min(lane, wz + 1);
    const int q = plane(z0 - 1 + l);
    const HZ_GLB T* b = ur + (long long)q * NP;
    T L[6], R[2][2][3];  // R[row: below/own][column: xhm/xh][comp]
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      L[j] = b[j * Nn + ym * N1 + xl];
      L[3 + j] = b[j * Nn + y * N1 + xl];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        R[r][0][j] = b[j * Nn + (r ? y : ym) * N1 + xhm];
        R[r][1][j] = b[j * Nn + (r ? y : ym) * N1 + xh];
      }
    }
    const int hph = ph[(long long)q * NP + y * N1 + xh];
    const cpx<T> hlm = ISO ? gld(Clm + hph) : cpx<T>{0, 0};
    if (wact && lane <= wz + 1) {
#pragma unroll
      for (int k = 0; k < 6; ++k) lh[w][lane][k] = L[k];
    }
    // voxel (xh, y, q) of lane l >= 1 (voxel plane z0 + l - 1): the plane below from lane l - 1
    T c[8][3];
#pragma unroll
    for (int o = 0; o < 8; ++o)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T v = R[(o >> 1) & 1][o & 1][j];
        c[o][j] = (o & 4) ? v : lane_shift<kShr1>(v, v);
      }
    T s1[6], s2[6];
    voxel_sigma<T, ISO, EIG>(c, C, hlm, hph, Mn, s1, s2);
    T P1[3], M1[3], Z1[3], P2[3], M2[3], Z2[3];
    stress_rows(s1, P1, M1, Z1);
    stress_rows(s2, P2, M2, Z2);
    if (wact && lane >= 1 && lane <= wz + 1) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        hr[w][lane - 1][0][j] = Z2[j] - M2[j];   // dy 0, dz 0: T2 corner 110
        hr[w][lane - 1][1][j] = -M1[j] - Z1[j];  // dy 0, dz 1: T1 corner 010
        hr[w][lane - 1][2][j] = Z1[j] - P1[j];   // dy 1, dz 0: T1 corner 100
        hr[w][lane - 1][3][j] = -P2[j] - Z2[j];  // dy 1, dz 1: T2 corner 000
      }
    }
  }
  __syncthreads();

  // ---- z streaming.  Corner plane q sits in buffer U[(q - z0 + 1) % 3] (rows: own,
  // below; column x -- column x - 1 comes by a lane shift where it is used), the phase
  // id and isotropic moduli of voxel plane q in PH, LM at the same index.  At step i
  // (voxel plane p = z0 + i) the buffers hold planes p - 1, p and p + 1 (in flight); once
  // the stresses are known, plane p - 1's buffer takes the loads of plane p + 2, issued
  // before this step's stores so that waiting for them later does not wait for the
  // stores.  The loop is unrolled three times, so no loaded value is ever copied.
  // byte offsets of this lane's corner in its row and the row below, within a plane
  // (the grid's real fields stay below 4 GiB: 12 S < 2^31 complex elements per load)
  const unsigned oo = (unsigned)((y * N1 + x) * (int)sizeof(T)), ob = (unsigned)((ym * N1 + x) * (int)sizeof(T));
  const unsigned oph = (unsigned)((y * N1 + x) * 2);
  T U[3][2][3];
  int PH[3] = {0, 0, 0};
  cpx<T> LM[3] = {{0, 0}, {0, 0}, {0, 0}};
  const int plane_bytes = NP * (int)sizeof(T);
  // corner plane q (q clamped to the segment's last one, so every call loads)
  auto load = [&](int q, T (&B)[2][3]) {
    const HZ_GLB T* base = ur + (long long)plane(min(q, z0 + wz)) * NP;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const __amdgpu_buffer_rsrc_t r = plane_rsrc((const void*)(base + (long long)j * Nn), plane_bytes);
      B[0][j] = buf_ld(T(), r, oo);
      B[1][j] = buf_ld(T(), r, ob);
    }
  };
  // phase id of voxel (x, y, q), q clamped to the segment's last voxel plane
  auto phase_at = [&](int q) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc((const void*)(ph + (long long)plane(min(q, z0 + wz)) * NP), 2 * NP);
    return (int)__builtin_amdgcn_raw_buffer_load_b16(r, (int)oph, 0, 0);
  };
  auto moduli = [&](int phase) { return gld(Clm + phase); };
  // the same issue order as in the loop: planes z0 - 1 and z0, phase ids, moduli,
  // then plane z0 + 1 last (the one needed latest)
  load(z0 - 1, U[0]);
  load(z0, U[1]);
  __builtin_amdgcn_sched_barrier(0);
  PH[1] = phase_at(z0);
  PH[2] = phase_at(z0 + 1);
  if constexpr (ISO) LM[1] = moduli(PH[1]);
  __builtin_amdgcn_sched_barrier(0);
  load(z0 + 1, U[2]);  // wz >= 1
  T Ap[4][3];  // [dx*2 + dy]: contributions of voxel plane p - 1 to corner plane p - 1
  double sacc[6] = {0, 0, 0, 0, 0, 0};
  // one z step; returns true after the segment's last voxel plane
  auto step = [&](const int i, auto bc) -> bool {
    constexpr int b0 = decltype(bc)::value, b1 = (b0 + 1) % 3, b2 = (b0 + 2) % 3;
    const int p = z0 + i;
    const T(&uo0)[3] = U[b0][0];
    const T(&ub0)[3] = U[b0][1];
    const T(&uo1)[3] = U[b1][0];
    const T(&ub1)[3] = U[b1][1];
    const int phc = PH[b1];
    const cpx<T> lmc = LM[b1];
    const T* e0 = lh[w][i];      // column x0 - 1, plane p - 1
    const T* e1 = lh[w][i + 1];  // plane p
    T s1[6], s2[6];
    {
      T u4[4][3], e[6];  // T1: corners 001, 010, 100, 111
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        u4[0][j] = ub0[j];
        u4[1][j] = lane_shift<kShr1>(uo0[j], e0[3 + j]);
        u4[2][j] = lane_shift<kShr1>(ub1[j], e1[j]);
        u4[3][j] = uo1[j];
      }
      stencil_strain_k<T, 0>(u4, e);
      if constexpr (ISO) constitutive_iso<EIG, T>(lmc.x, lmc.y, Mn, phc, e, s1);
      else {
#pragma unroll
        for (int k = 0; k < 6; ++k) s1[k] = e[k];  // the strain, until both are known
      }
    }
    {
      T u4[4][3], e[6];  // T2: corners 000, 011, 101, 110
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        u4[0][j] = lane_shift<kShr1>(ub0[j], e0[j]);
        u4[1][j] = uo0[j];
        u4[2][j] = ub1[j];
        u4[3][j] = lane_shift<kShr1>(uo1[j], e1[3 + j]);
      }
      stencil_strain_k<T, 1>(u4, e);
      if constexpr (ISO) constitutive_iso<EIG, T>(lmc.x, lmc.y, Mn, phc, e, s2);
      else {
        const T e1s[6] = {s1[0], s1[1], s1[2], s1[3], s1[4], s1[5]};
        if (tab) {
          const cpx<T>* row = ctab + phc * 12;
          constitutive_pair_ld<EIG, T>([&](int k) { return row[k]; }, Mn, phc, e1s, e, s1, s2);
        } else {
          constitutive_pair<EIG, T>(C + phc * 24, Mn, phc, e1s, e, s1, s2);
        }
      }
    }
    // issue order: moduli of plane p + 1 (needed first), phase ids of plane p + 2,
    // corners of plane p + 2 (needed last); past the segment's end the loads repeat its
    // last plane (unused), which keeps the step free of branches around them
    if constexpr (ISO) LM[b2] = moduli(PH[b2]);
    __builtin_amdgcn_sched_barrier(0);
    PH[b0] = phase_at(p + 2);
    __builtin_amdgcn_sched_barrier(0);
    load(p + 2, U[b0]);
    if (i < wz && wact && xact) {
#pragma unroll
      for (int k = 0; k < 6; ++k) sacc[k] += 0.5 * ((double)s1[k] + (double)s2[k]);
    }
    T P1[3], M1[3], Z1[3], P2[3], M2[3], Z2[3];
    stress_rows(s1, P1, M1, Z1);
    stress_rows(s2, P2, M2, Z2);
    T X0[3], X1[3];
    if (i > 0) {
      // corner plane p - 1 is complete: add the voxel plane p terms (dz = 1); column
      // x + 1's A10, A11 by a lane shift (lane 63 of a full tile: the halo column)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T H10 = hr[w][i - 1][0][j] + hr[w][i][1][j];
        const T H11 = hr[w][i - 1][2][j] + hr[w][i][3][j];
        const T A10 = Ap[2][j] - (M1[j] + Z1[j]);  // T1 corner 010
        const T A11 = Ap[3][j] - (P2[j] + Z2[j]);  // T2 corner 000
        X0[j] = (Ap[0][j] + (P2[j] - Z2[j])) + lane_shift<kShl1>(A10, H10);  // T2 corner 011
        X1[j] = (Ap[1][j] + (M1[j] - Z1[j])) + lane_shift<kShl1>(A11, H11);  // T1 corner 001
        xb[i & 1][w][j][lane] = X1[j];
      }
    }
    // voxel plane p's terms of corner plane p (dz = 0)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Ap[0][j] = P1[j] + Z1[j];  // T1 corner 111
      Ap[1][j] = M2[j] + Z2[j];  // T2 corner 101
      Ap[2][j] = Z2[j] - M2[j];  // T2 corner 110
      Ap[3][j] = Z1[j] - P1[j];  // T1 corner 100
    }
    __syncthreads();
    if (i > 0 && wact && xact) {
      HZ_GLB T* gp = gr + (long long)(p - 1) * NP;
      if (w + 1 < wy) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
          buf_st((T)0.5 * (X0[j] + xb[i & 1][w + 1][j][lane]), plane_rsrc((void*)(gp + (long long)j * Nn), plane_bytes),
                 oo);
      } else {
#pragma unroll
        for (int j = 0; j < 3; ++j) unsafeAtomicAdd((T*)(gp + (long long)j * Nn + y * N1 + x), (T)0.5 * X0[j]);
      }
      if (w == 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j) unsafeAtomicAdd((T*)(gp + (long long)j * Nn + ym * N1 + x), (T)0.5 * X1[j]);
      }
    }
    return i == wz;
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  using B2 = std::integral_constant<int, 2>;
#pragma unroll 1
  for (int i = 0;; i += 3) {
    if (step(i, B0{})) break;
    if (step(i + 1, B1{})) break;
    if (step(i + 2, B2{})) break;
  }
  block_sum<6>(sacc, red);
  if (threadIdx.x == 0) {
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
  const hipError_t e = inverse ? allow_lds(k_zconv3<true>, shm) : allow_lds(k_zconv3<false>, shm);
  if (e != hipSuccess) return e;
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
    case 7: hipLaunchKernelGGL((k_xc2r<T, 7>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, tw); break;
    case 5: hipLaunchKernelGGL((k_xc2r<T, 5>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, tw); break;
    case 3: hipLaunchKernelGGL((k_xc2r<T, 3>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, tw); break;
    case 1: hipLaunchKernelGGL((k_xc2r<T, 1>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXi, tw); break;
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
    case 7: hipLaunchKernelGGL((k_xr2c<T, 7>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXf, tw); break;
    case 5: hipLaunchKernelGGL((k_xr2c<T, 5>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXf, tw); break;
    case 3: hipLaunchKernelGGL((k_xr2c<T, 3>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXf, tw); break;
    case 1: hipLaunchKernelGGL((k_xr2c<T, 1>), grid, dim3(kThreads), shm, s, descs, active, xg, *planXf, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Largest stiffness table the anisotropic variants copy to LDS (24 slots per phase):
// 200 rotated grains.  Beside the kernel's static buffers (about 32 KB FP64, 16 KB FP32)
// a table that size leaves FP32 at its 4 work-groups per CU and takes FP64 from 3 to 2,
// which still measured faster at 200 grains than gathering the rows from L2 at 3.
template <typename T>
constexpr int stencil_tab_cap() { return sizeof(T) == 8 ? 38400 : 24 * 1024; }

// max_phases: the most phases among the launch's problems; the launch reserves LDS for
// that table if it fits the cap, else none (each block checks its own problem)
template <typename T>
hipError_t launch_stencil(const Desc* descs, const int* active, int nact, int kind, int max_phases, const SGeo& sg,
                          hipStream_t s) {
  dim3 grid((unsigned)(sg.tx * sg.ty * sg.tz), nact);
  const int need = max_phases * 24 * (int)sizeof(T);
  const int tb = (kind & KIND_ISO) || need > stencil_tab_cap<T>() ? 0 : need;
  if (kind == 0) {
    const hipError_t e = allow_lds(k_stencil<T, false, false>, tb + 32 * 1024);
    if (e != hipSuccess) return e;
  } else if (kind == KIND_EIG) {
    const hipError_t e = allow_lds(k_stencil<T, false, true>, tb + 32 * 1024);
    if (e != hipSuccess) return e;
  }
  switch (kind) {
    case KIND_ISO: hipLaunchKernelGGL((k_stencil<T, true, false>), grid, dim3(kThreads), 0, s, descs, active, sg, 0); break;
    case KIND_ISO | KIND_EIG: hipLaunchKernelGGL((k_stencil<T, true, true>), grid, dim3(kThreads), 0, s, descs, active, sg, 0); break;
    case 0: hipLaunchKernelGGL((k_stencil<T, false, false>), grid, dim3(kThreads), tb, s, descs, active, sg, tb); break;
    default: hipLaunchKernelGGL((k_stencil<T, false, true>), grid, dim3(kThreads), tb, s, descs, active, sg, tb); break;
  }
  return hipGetLastError();
}

template hipError_t launch_xc2r<double>(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template hipError_t launch_xc2r<float>(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template hipError_t launch_xr2c<double>(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template hipError_t launch_xr2c<float>(const Desc*, const int*, int, const XGeo&, const Plan*, int, const void*, hipStream_t);
template hipError_t launch_stencil<double>(const Desc*, const int*, int, int, int, const SGeo&, hipStream_t);
template hipError_t launch_stencil<float>(const Desc*, const int*, int, int, int, const SGeo&, hipStream_t);

}  // namespace hz
