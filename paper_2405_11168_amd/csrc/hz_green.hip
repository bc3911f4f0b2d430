// HIP kernels (gfx950) of the continuous-frequency comparison operator (Sec. 3.2):
// the displacement-based basic scheme with one strain field per voxel and the
// gradient symbol D(q) = i xi(q), xi the frequency of the centred representative of
// q (xi = 0 at the highest frequency of an even axis, so the strain stays real).
// The x and y passes are those of the spectral form (its two strain fields simply
// coincide); these kernels replace its two z kernels, FP64 only.
//
// Why 6 lines per column.  i xi_3 is not a short stencil along l3, so unlike the
// tetrahedral and rotated symbols (affine in exp(-i q3)) the z derivative cannot be
// taken after the transform.  Instead the transform carries u and i xi_3 u together
// (inverse), and the residual's xi_3 part and the rest separately (forward):
//   eps_ij = (G_i u_j + G_j u_i)/2 with G_1 u = i xi_1 U, G_2 u = i xi_2 U, G_3 u = V,
//   U, V the inverse z transforms of u and i xi_3 u;
//   r_i = sum_j S_ij conj(G_j) = A_i - i xi_3 B_i with A_i = -i (xi_1 S_i1 + xi_2 S_i2),
//   B_i = S_i3 formed before the forward transform, S = sigma^T1 + sigma^T2.
// A block owns the TX columns of a z tile of the spectral form (so the residual
// partial sums keep their count and order) and works through them `sub` columns at
// a time, 6 sub lines of N3 in LDS.
#include "hz_device.h"

namespace hz {

// xi(h) = 2 pi h~ / N, h~ in (-N/2, N/2); 0 at h = N/2
__device__ __forceinline__ double xi_of(int h, int N) {
  const int ht = 2 * h < N ? h : (2 * h == N ? 0 : h - N);
  return (2.0 * 3.14159265358979323846) * (double)ht / (double)N;
}
// i x a
__device__ __forceinline__ cpx<double> ix(double x, cpx<double> a) { return {-x * a.y, x * a.x}; }

__global__ __launch_bounds__(kThreads) void k_zexp_cont(const Desc* __restrict__ descs,
                                                        const int* __restrict__ active, ZGeo zg, int sub,
                                                        float rl6, const Plan plan3v,
                                                        const cpx<double>* __restrict__ tw3T) {
  const Plan* plan3 = &plan3v;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int TX = zg.TX, N2 = zg.N2, N3 = zg.N3;
  const long long S = zg.S;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int h1 = tile / zg.tiles;
  const int h2t = (tile % zg.tiles) * TX;
  const int lines = 6 * sub;
  cpx<double>* buf = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* twl = buf + lines * N3;
  stage_table(twl, tw3T, N3);
  const LdsAcc<double> lds{buf, 1, lines};
  const cpx<double>* u = reinterpret_cast<const cpx<double>*>(d.src == 1 ? d.u64 : u_slot(d, cur_slot(d)));
  cpx<double>* out = reinterpret_cast<cpx<double>*>(d.spec);
  const double x1 = xi_of(h1, zg.N1);
#pragma unroll 1
  for (int r0 = 0; r0 < TX; r0 += sub) {
    const long long plane = (long long)h1 * N3 * N2 + h2t + r0;
    for (int e = threadIdx.x; e < 3 * sub * N3; e += kThreads) {
      const int col = e % sub, rest = e / sub;
      const int h3 = rest % N3, c = rest / N3;
      const cpx<double> v = u[c * S + plane + (long long)h3 * N2 + col];
      lds.put(c * sub + col, h3, v);
      lds.put((3 + c) * sub + col, h3, ix(xi_of(h3, N3), v));
    }
    __syncthreads();
    fft_lines<double, emax<double>(), true>(*plan3, lines, rl6, false, twl, 1, lds, lds, lds);
    __syncthreads();
    for (int e = threadIdx.x; e < sub * N3; e += kThreads) {
      const int col = e % sub, l3 = e / sub;
      const double x2 = xi_of(h2t + r0 + col, N2);
      cpx<double> G[3][3];  // G[i][j] = (D_i u_j) in the mixed (h1, h2, l3) domain
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const cpx<double> U = lds.get(j * sub + col, l3);
        G[0][j] = ix(x1, U);
        G[1][j] = ix(x2, U);
        G[2][j] = lds.get((3 + j) * sub + col, l3);
      }
      cpx<double> e6[6];
      e6[0] = G[0][0];
      e6[1] = G[1][1];
      e6[2] = G[2][2];
      e6[3] = scale(G[1][2] + G[2][1], 0.5);
      e6[4] = scale(G[0][2] + G[2][0], 0.5);
      e6[5] = scale(G[0][1] + G[1][0], 0.5);
      const long long o = plane + (long long)l3 * N2 + col;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        out[c * S + o] = e6[c];        // both strain fields of the spectral form
        out[(6 + c) * S + o] = e6[c];  // carry the one strain of this scheme
      }
    }
    __syncthreads();  // the next column group reuses the lines
  }
}

__global__ __launch_bounds__(kThreads) void k_zcon_cont(const Desc* __restrict__ descs,
                                                        const int* __restrict__ active, ZGeo zg, int sub,
                                                        float rl6, const Plan plan3v,
                                                        const cpx<double>* __restrict__ tw3T) {
  const Plan* plan3 = &plan3v;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d)) return;
  const int TX = zg.TX, N1 = zg.N1, N2 = zg.N2, N3 = zg.N3;
  const long long S = zg.S;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int h1 = tile / zg.tiles;
  const int h2t = (tile % zg.tiles) * TX;
  const int lines = 6 * sub;
  cpx<double>* buf = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* twl = buf + lines * N3;
  stage_table(twl, tw3T, N3);
  const LdsAcc<double> lds{buf, 1, lines};
  const cpx<double>* sp = reinterpret_cast<const cpx<double>*>(d.spec);
  const int p = cur_slot(d);
  const cpx<double>* uin = reinterpret_cast<const cpx<double>*>(u_slot(d, p));
  cpx<double>* uout = reinterpret_cast<cpx<double>*>(u_slot(d, 1 - p));
  const double x1 = xi_of(h1, N1);
  const bool h1_edge = h1 == 0 || 2 * h1 == N1;
  const double w = h1_edge ? 1.0 : 2.0;  // half-spectrum weight of the norm
  double part[1] = {0.0};
#pragma unroll 1
  for (int r0 = 0; r0 < TX; r0 += sub) {
    const long long plane = (long long)h1 * N3 * N2 + h2t + r0;
    for (int e = threadIdx.x; e < sub * N3; e += kThreads) {
      const int col = e % sub, l3 = e / sub;
      const long long o = plane + (long long)l3 * N2 + col;
      cpx<double> s[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) s[c] = sp[c * S + o] + sp[(6 + c) * S + o];
      // comps (11,22,33,23,13,12): S_i1 = (s0, s5, s4), S_i2 = (s5, s1, s3), S_i3 = (s4, s3, s2)
      const double x2 = xi_of(h2t + r0 + col, N2);
      const cpx<double> Si1[3] = {s[0], s[5], s[4]}, Si2[3] = {s[5], s[1], s[3]}, Si3[3] = {s[4], s[3], s[2]};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const cpx<double> a = {x1 * Si1[i].x + x2 * Si2[i].x, x1 * Si1[i].y + x2 * Si2[i].y};
        lds.put(i * sub + col, l3, ix(-1.0, a));  // -i (xi1 S_i1 + xi2 S_i2)
        lds.put((3 + i) * sub + col, l3, Si3[i]);
      }
    }
    __syncthreads();
    fft_lines<double, emax<double>(), false>(*plan3, lines, rl6, false, twl, 1, lds, lds, lds);
    __syncthreads();
    for (int e = threadIdx.x; e < sub * N3; e += kThreads) {
      const int col = e % sub, h3 = e / sub;
      const int h2 = h2t + r0 + col;
      const double x2 = xi_of(h2, N2), x3 = xi_of(h3, N3);
      cpx<double> r[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) r[i] = lds.get(i * sub + col, h3) + ix(-x3, lds.get((3 + i) * sub + col, h3));
      part[0] += 0.25 * w * (r[0].x * r[0].x + r[0].y * r[0].y + r[1].x * r[1].x + r[1].y * r[1].y +
                             r[2].x * r[2].x + r[2].y * r[2].y);
      // K_il = sum_jk lambda0_ijkl M_jk with M_jk = 2 xi_j xi_k (both strain fields)
      const double xv[3] = {x1, x2, x3};
      double M[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k) M[j][k] = 2.0 * xv[j] * xv[k];
      double K[3][3];
      if (d.c0_iso) {
        const double tm = d.mu0 * (M[0][0] + M[1][1] + M[2][2]), lm = d.lam0 + d.mu0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int l = 0; l < 3; ++l) K[a][l] = lm * M[a][l] + (a == l ? tm : 0.0);
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
              for (int k = 0; k < 3; ++k) acc += d.C0[((a * 3 + j) * 3 + k) * 3 + l] * M[j][k];
            K[a][l] = acc;
          }
      }
      // xi = 0: every index at 0 or at the highest frequency of its axis
      const bool sing = h1_edge && (h2 == 0 || 2 * h2 == N2) && (h3 == 0 || 2 * h3 == N3);
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
      const long long o = plane + (long long)h3 * N2 + col;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const cpx<double> dw = {O[a][0] * r[0].x + O[a][1] * r[1].x + O[a][2] * r[2].x,
                                O[a][0] * r[0].y + O[a][1] * r[1].y + O[a][2] * r[2].y};
        uout[a * S + o] = uin[a * S + o] - dw;
      }
    }
    __syncthreads();
  }
  block_sum<1>(part, red);
  if (threadIdx.x == 0) d.part_res[tile] = part[0];
}

hipError_t launch_zexp_cont(const Desc* descs, const int* active, int nact, const ZGeo& zg, int sub, float rl6,
                            const Plan* plan3, const void* tw3T, hipStream_t s) {
  const size_t shm = ((size_t)6 * sub * zg.N3 + zg.N3) * sizeof(cpx<double>);
  dim3 grid((unsigned)(zg.H1 * zg.tiles), nact);
  hipLaunchKernelGGL(k_zexp_cont, grid, dim3(kThreads), shm, s, descs, active, zg, sub, rl6, *plan3,
                     (const cpx<double>*)tw3T);
  return hipGetLastError();
}

hipError_t launch_zcon_cont(const Desc* descs, const int* active, int nact, const ZGeo& zg, int sub, float rl6,
                            const Plan* plan3, const void* tw3T, hipStream_t s) {
  const size_t shm = ((size_t)6 * sub * zg.N3 + zg.N3) * sizeof(cpx<double>);
  dim3 grid((unsigned)(zg.H1 * zg.tiles), nact);
  hipLaunchKernelGGL(k_zcon_cont, grid, dim3(kThreads), shm, s, descs, active, zg, sub, rl6, *plan3,
                     (const cpx<double>*)tw3T);
  return hipGetLastError();
}

}  // namespace hz
