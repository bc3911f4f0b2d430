// HIP kernels (gfx950) shared by both realisations: forward z transform with the
// Green-operator update (P5), the stop rule, and the refinement helpers.
#include "hz_device.h"

namespace hz {

// ----------------------------------------------------------------------------
// P5: residual r = sigma^T1.conj(D~) + sigma^T2.conj(D~2) (eq. Equilibrium_Q_div_bis),
// formed before the forward z transform as R(l3) = A(l3) + B(l3 + 1) with
// A = sigma.conj(alpha), B = sigma.conj(beta); then the transform of its 3 comps,
// the Green operator in FP64 (eq. Green_tensor) and the update (eq. basic_scheme_dep_2).
// d.cmode 0: u[1-p] = u[p] - Omega r      (p = current slot)
// d.cmode 1: FP64 sweep of the anchor: store r in r32, no update
// d.cmode 2: correction round: r += r32, u[1-p] = u[p] - Omega r
// d.cmode 3: strain-based form: u[0] = Omega r (the next P1 applies it to the strains)
// The stencil form keeps u in the mixed domain (inverse z transform of u(q)), so its
// update subtracts the inverse z transform of Omega r (linearity of the transform).
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
// C0ISO: the reference medium is isotropic (problems of the other kind skip the
// block); the generic variant contracts the full lambda0 tensor.
template <typename T, bool STENCIL, bool C0ISO>
__global__ __launch_bounds__(kThreads) void k_zcon(const Desc* __restrict__ descs, const int* __restrict__ active,
                                                   ZGeo zg, const Plan plan3v, const cpx<T>* __restrict__ tw3T,
                                                   const cpx<double>* __restrict__ tw1,
                                                   const cpx<double>* __restrict__ tw2,
                                                   const cpx<double>* __restrict__ tw3) {
  const Plan* plan3 = &plan3v;  // kernel argument (scalar loads)

  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  const Desc& d = descs[active[blockIdx.y]];
  if (problem_done(d) || (d.c0_iso != 0) != C0ISO) return;
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
  const HZ_GLB cpx<T>* sp = glb(reinterpret_cast<const cpx<T>*>(d.spec)) + plane;
  const cpx<double> t1 = tw1[h1];
  const int ne = TX * N3;
  const bool rot = !STENCIL && d.green == GREEN_ROTATED;  // the stencil form is tetrahedral
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
      if (rot) {
        rotated_mean(a1, a2);
        rotated_mean(b1, b2);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a1[c] = conjg(a1[c]); b1[c] = conjg(b1[c]); a2[c] = conjg(a2[c]); b2[c] = conjg(b2[c]);
      }
      const int l0 = run * m;
      const int l1 = min(l0 + m, N3);  // rows l0 .. l1-1 produced, row l1 (mod N3) read
      // the two tetrahedra one after the other (6 loads live at a time): T1 writes its
      // part of R, T2 adds its own to the same elements of the same thread
      auto half = [&](const cpx<double>(&A)[3], const cpx<double>(&B)[3], const int f, const bool add) {
        cpx<double> Bn[3];
        {
          const int l = l1 == N3 ? 0 : l1;
          const long long o = (long long)l * N2 + col;
          cpx<T> s[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) s[c] = gld(sp + (f + c) * zg.S + o);
          sig_dot(s, B, Bn);
        }
#pragma unroll 1
        for (int l = l1 - 1; l >= l0; --l) {
          const long long o = (long long)l * N2 + col;
          cpx<T> s[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) s[c] = gld(sp + (f + c) * zg.S + o);
          cpx<double> x[3], y[3];
          sig_dot(s, A, x);
          sig_dot(s, B, y);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const cpx<double> v = x[c] + Bn[c];
            lds.put(c * TX + col, l, add ? fr64<T>(to64(lds.get(c * TX + col, l)) + v) : fr64<T>(v));
            Bn[c] = y[c];
          }
        }
      };
      half(a1, b1, 0, false);
      half(a2, b2, 6, true);
    }
  }
  __syncthreads();
  fft_lines<T, emax<T>(), false>(*plan3, lines, zg.rLines, false, twl, 1, lds, lds, lds);
  }
  __syncthreads();
  // phase C: Green operator and update at q = (h1, h2, h3).  Elements go in chunks
  // of CH per thread with the chunk's HBM loads (u, and r of the sweep) issued
  // first, so their latency overlaps instead of stalling every element.
  double part[1] = {0.0};
  const double w = (h1 == 0 || 2 * h1 == zg.N1) ? 1.0 : 2.0;
  const int MODE = d.cmode;
  const int p = cur_slot(d);
  const HZ_GLB cpx<T>* uin = glb(reinterpret_cast<const cpx<T>*>(u_slot(d, p))) + plane;
  HZ_GLB cpx<T>* uout = glb(reinterpret_cast<cpx<T>*>(u_slot(d, MODE == 3 ? 0 : 1 - p))) + plane;
  const HZ_GLB cpx<float>* r32in = glb(reinterpret_cast<const cpx<float>*>(d.r32)) + plane;
  HZ_GLB cpx<float>* r32out = glb(reinterpret_cast<cpx<float>*>(d.r32)) + plane;
  constexpr int CH = 4;
#pragma unroll 1
  for (int e0 = threadIdx.x; e0 < ne; e0 += CH * kThreads) {
    cpx<T> uv[CH][3];
    cpx<float> rv[CH][3];
    cpx<double> t2v[CH], t3v[CH];  // e^{-i q2}, e^{-i q3} of the chunk's elements
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int e = e0 + i * kThreads;
      if (e >= ne) break;
      const int h3 = fdiv(e, zg.rTX), col = e - h3 * TX;
      const int o = h3 * N2 + col;
      t2v[i] = tw2[h2_0 + col];
      t3v[i] = tw3[h3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (!STENCIL && (MODE == 0 || MODE == 2)) uv[i][c] = gld(uin + c * zg.S + o);
        if (MODE == 2) rv[i][c] = gld(r32in + c * zg.S + o);
      }
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int e = e0 + i * kThreads;
      if (e >= ne) break;
      const int h3 = fdiv(e, zg.rTX), col = e - h3 * TX;
      const int h2 = h2_0 + col;
      const int o = h3 * N2 + col;
      cpx<double> r[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = to64(lds.get(c * TX + col, h3));
      if (MODE == 2) {
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = r[c] + to64(rv[i][c]);
      }
      part[0] += 0.25 * w * (r[0].x * r[0].x + r[0].y * r[0].y + r[1].x * r[1].x + r[1].y * r[1].y +
                             r[2].x * r[2].x + r[2].y * r[2].y);
      if (MODE == 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) gst(r32out + c * zg.S + o, fr64<float>(r[c]));
        continue;
      }
      cpx<double> D1[3], D2[3];
      symbols(t1, t2v[i], t3v[i], D1, D2);
      // M_jk = Re(conj(D1_j) D1_k + conj(D2_j) D2_k): with D~2 = -conj(D) times the phase
      // (tetrahedral) and with D1 = D2 (rotated) alike it is 2 Re(conj(D1_j) D1_k)
      if (rot) rotated_mean(D1, D2);
      // K_il = sum_jk C0_ijkl M_jk,  M_jk = 2 Re(conj(D_j) D_k)
      double Mjk[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k) Mjk[j][k] = 2.0 * (D1[j].x * D1[k].x + D1[j].y * D1[k].y);
      double K[3][3];
      if (C0ISO) {
        // isotropic lambda0: K = mu0 tr(M) I + (lam0 + mu0) M
        const double tm = d.mu0 * (Mjk[0][0] + Mjk[1][1] + Mjk[2][2]), lm = d.lam0 + d.mu0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int l = 0; l < 3; ++l) K[a][l] = lm * Mjk[a][l] + (a == l ? tm : 0.0);
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
              for (int k = 0; k < 3; ++k) acc += d.C0[((a * 3 + j) * 3 + k) * 3 + l] * Mjk[j][k];
            K[a][l] = acc;
          }
      }
      const int npi = (2 * h1 == zg.N1) + (2 * h2 == N2) + (2 * h3 == N3);
      // Omega := 0 at q = 0 and where D vanishes: (pi,pi,pi) for the tetrahedral
      // stencil, every q with two components at pi for the rotated one
      const bool sing = (h1 == 0 && h2 == 0 && h3 == 0) || npi >= (rot ? 2 : 3);
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
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const cpx<double> dw = {O[a][0] * r[0].x + O[a][1] * r[1].x + O[a][2] * r[2].x,
                                O[a][0] * r[0].y + O[a][1] * r[1].y + O[a][2] * r[2].y};
        if (STENCIL) {
          // Omega r replaces r in its LDS line (same element, same thread)
          lds.put(a * TX + col, h3, fr64<T>(dw));
        } else {
          gst(uout + a * zg.S + o, fr64<T>(MODE == 3 ? dw : to64(uv[i][a]) - dw));
        }
      }
    }
  }
  if (STENCIL && (MODE == 0 || MODE == 2)) {
    // mixed-domain update: inverse z transform of Omega r on the lines in LDS, then
    // u[1-p] = u[p] - that, element by element (loads issued CT at a time: the
    // transform's registers are free by then)
    __syncthreads();
    fft_lines<T, emax<T>(), true>(*plan3, lines, zg.rLines, false, twl, 1, lds, lds, lds);
    __syncthreads();
    const int nl = lines * N3;
    constexpr int CT = 12;
#pragma unroll 1
    for (int e0 = threadIdx.x; e0 < nl; e0 += CT * kThreads) {
      cpx<T> v[CT];
      int off[CT];
#pragma unroll
      for (int i = 0; i < CT; ++i) {
        const int e = e0 + i * kThreads;
        if (e >= nl) break;
        const int l3 = fdiv(e, zg.rLines), t = e - l3 * lines;
        const int c = fdiv(t, zg.rTX);
        off[i] = c * (int)zg.S + l3 * N2 + (t - c * TX);
        v[i] = gld(uin + off[i]);
      }
#pragma unroll
      for (int i = 0; i < CT; ++i) {
        const int e = e0 + i * kThreads;
        if (e >= nl) break;
        gst(uout + off[i], v[i] - buf[e]);
      }
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
  // under applied stress the residual is measured against the fixed scale d.sref
  // (||sigma^a||, or the eigenstress scale when no stress is applied) instead of
  // ||<sigma>||, which tends to sigma^a
  const bool stress = d.loading == 1;
  const double nrm = stress ? d.sref
                            : sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2] +
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
  if (k == 0) {
    s[ST_FIRST_ERR] = err;
    s[ST_L2_FIRST] = L2;
  }
  s[ST_K] = k + 1;
  if (fmode == 1) {
    // a sweep measures once; the host decides what follows
    s[ST_DONE] = 1.0;
    s[ST_ITERS] = k;
    return;
  }
  if (fmode == 3) {
    // plain FP32 iterations of refinement round 0: stop at the target, at the FP32
    // rounding floor (less than 3% gain over 32 iterations) or at the cap; with a
    // fixed count only at the cap
    const bool fixed = d.fixed_iters >= 0;
    const bool reached = !fixed && err <= s[ST_REF];
    const bool bad = !(err == err) || isinf(err) || (k > 0 && err > 1e3 * s[ST_FIRST_ERR]);
    bool stalled = false;
    if (!fixed && k > 0 && (k % 32) == 0) {
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
  if (s[ST_K1E6] < 0.0 && err < 1e-6) s[ST_K1E6] = k;  // time-to-1e-6 of FP64 iterations
  bool conv = err < d.tol;
  double mis[6];
  if (stress) {
    // the loop on the mean strain has converged too: <sigma> = sigma^a (eq. equi_epsilon_bar)
#pragma unroll
    for (int c = 0; c < 6; ++c) mis[c] = d.sig_a[c] - m[c];
    const double dm = sqrt(mis[0] * mis[0] + mis[1] * mis[1] + mis[2] * mis[2] +
                           2.0 * (mis[3] * mis[3] + mis[4] * mis[4] + mis[5] * mis[5]));
    conv = conv && dm <= d.tol * d.sref;
  }
  const bool stop = d.fixed_iters >= 0 ? (k >= d.fixed_iters) : conv;
  // watchdog: NaN/Inf, eps grown to 1e3 times its first value, or the residual norm L2
  // back above its first value and 10 times the smallest seen.  Iterates that run away
  // (a reference medium too soft for the basic scheme) make L2 grow geometrically while
  // <sigma> grows with them, so eps alone grows only slowly; with stiff inclusions eps
  // can rise transiently by tens of times because <sigma> falls from the Voigt average
  // by up to the contrast, while L2 only decreases, so the rule reads L2, not eps.
  const double best = k == 0 ? L2 : fmin(s[ST_BEST], L2);
  s[ST_BEST] = best;
  const bool bad = !(err == err) || isinf(err) ||
                   (k > 0 && (err > 1e3 * s[ST_FIRST_ERR] || (L2 > s[ST_L2_FIRST] && L2 > 10.0 * best)));
  if (stop || bad || k >= d.max_iters) {
    s[ST_DONE] = bad ? 3.0 : (stop ? 1.0 : 2.0);
    s[ST_ITERS] = k;
    s[ST_PARITY] = parity;
    return;
  }
  if (stress) {
    // step 6 of Algorithm 1: since <lambda>:Ebar + <lambda:deps> - <lambda:eps0> is
    // <sigma>_k, the update is Ebar <- Ebar + lambda0^-1:(sigma^a - <sigma>_k)
    double e[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double a = s[ST_EBAR + i];
#pragma unroll
      for (int j = 0; j < 6; ++j) a += d.S0[i * 6 + j] * mis[j];
      e[i] = a;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) s[ST_EBAR + i] = e[i];
  }
}

// U64 += delta (refinement), delta in FP32
__global__ __launch_bounds__(kThreads) void k_accumulate(const Desc* __restrict__ descs,
                                                         const int* __restrict__ active,
                                                         long long n3c) {
  const Desc& d = descs[active[blockIdx.y]];
  const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= n3c) return;
  const int p = (int)status_ro(d)[ST_PARITY];
  const cpx<float> a = ld<float>(u_slot(d, p), idx);
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
template <typename T, bool STENCIL, bool C0ISO>
hipError_t launch_zcon1(const Desc* descs, const int* active, int nact, const ZGeo& zg, const Plan* plan3,
                        const void* tw3T, const void* tw1, const void* tw2, const void* tw3, hipStream_t s) {
  const size_t shm = ((size_t)3 * zg.TX * zg.N3 + zg.N3) * sizeof(cpx<T>);
  dim3 grid((unsigned)(zg.H1 * zg.tiles), nact);
  const hipError_t e = allow_lds(k_zcon<T, STENCIL, C0ISO>, shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_zcon<T, STENCIL, C0ISO>), grid, dim3(kThreads), shm, s, descs, active, zg, *plan3,
                     (const cpx<T>*)tw3T, (const cpx<double>*)tw1, (const cpx<double>*)tw2, (const cpx<double>*)tw3);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zcon(const Desc* descs, const int* active, int nact, bool stencil, int c0, const ZGeo& zg,
                       const Plan* plan3, const void* tw3T, const void* tw1, const void* tw2, const void* tw3,
                       hipStream_t s) {
  hipError_t e = hipSuccess;
  if (c0 & 1) {
    e = stencil ? launch_zcon1<T, true, true>(descs, active, nact, zg, plan3, tw3T, tw1, tw2, tw3, s)
                : launch_zcon1<T, false, true>(descs, active, nact, zg, plan3, tw3T, tw1, tw2, tw3, s);
    if (e != hipSuccess) return e;
  }
  if (c0 & 2) {
    e = stencil ? launch_zcon1<T, true, false>(descs, active, nact, zg, plan3, tw3T, tw1, tw2, tw3, s)
                : launch_zcon1<T, false, false>(descs, active, nact, zg, plan3, tw3T, tw1, tw2, tw3, s);
  }
  return e;
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

template hipError_t launch_zcon<double>(const Desc*, const int*, int, bool, int, const ZGeo&, const Plan*, const void*, const void*, const void*, const void*, hipStream_t);
template hipError_t launch_zcon<float>(const Desc*, const int*, int, bool, int, const ZGeo&, const Plan*, const void*, const void*, const void*, const void*, hipStream_t);

}  // namespace hz
