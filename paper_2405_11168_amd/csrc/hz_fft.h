// Complex arithmetic, radix butterflies and the LDS-resident Stockham transform
// used by every FFT pass of the solver (gfx950, wave64).
#pragma once
#include "hz_internal.h"

namespace hz {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cpx<T> conjg(cpx<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward sign) or +i (inverse sign)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> rot(cpx<T> a) {
  return INV ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.y, a.x}; }

// cos/sin(2 pi m / R) for the odd radices, m = 0..R-1
template <int R> struct Trig;
template <> struct Trig<3> {
  static constexpr double c[3] = {1.0, -0.5, -0.5};
  static constexpr double s[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
};
template <> struct Trig<5> {
  static constexpr double c[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410,
                                  -0.80901699437494742410, 0.30901699437494742410};
  static constexpr double s[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917,
                                  -0.58778525229247312917, -0.95105651629515357212};
};
template <> struct Trig<7> {
  static constexpr double c[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                  -0.90096886790241912624, -0.90096886790241912624,
                                  -0.22252093395631440429, 0.62348980185873353053};
  static constexpr double s[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                  0.43388373911755812048, -0.43388373911755812048,
                                  -0.97492791218182360702, -0.78183148246802980871};
};

// In-register DFT of length R: a[k] <- sum_n a[n] exp(-+2 pi i n k / R)
template <typename T, int R, bool INV> struct Dft;

template <typename T, bool INV> struct Dft<T, 2, INV> {
  static __device__ __forceinline__ void run(cpx<T>* a) {
    cpx<T> t = a[0] - a[1];
    a[0] = a[0] + a[1];
    a[1] = t;
  }
};

template <typename T, bool INV> struct Dft<T, 4, INV> {
  static __device__ __forceinline__ void run(cpx<T>* a) {
    cpx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
    cpx<T> t2 = a[1] + a[3], t3 = rot<T, INV>(a[1] - a[3]);
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + t3;
    a[3] = t1 - t3;
  }
};

template <typename T, bool INV> struct Dft<T, 8, INV> {
  static __device__ __forceinline__ void run(cpx<T>* a) {
    cpx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cpx<T> o[4] = {a[1], a[3], a[5], a[7]};
    Dft<T, 4, INV>::run(e);
    Dft<T, 4, INV>::run(o);
    const T h = (T)0.70710678118654752440;
    // w8^1, w8^2, w8^3 with w8 = exp(-+ 2 pi i / 8)
    o[1] = INV ? cpx<T>{h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)}
               : cpx<T>{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
    o[2] = rot<T, INV>(o[2]);
    o[3] = INV ? cpx<T>{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)}
               : cpx<T>{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = e[k] + o[k];
      a[k + 4] = e[k] - o[k];
    }
  }
};

// odd prime radix: X_k = a0 + sum_{n<=h} [c(nk)(a_n + a_{R-n}) -+ i s(nk)(a_n - a_{R-n})]
template <typename T, int R, bool INV> struct DftOdd {
  static __device__ __forceinline__ void run(cpx<T>* a) {
    constexpr int H = (R - 1) / 2;
    cpx<T> t[H + 1], d[H + 1];
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      t[n] = a[n] + a[R - n];
      d[n] = a[n] - a[R - n];
    }
    cpx<T> x0 = a[0];
#pragma unroll
    for (int n = 1; n <= H; ++n) x0 = x0 + t[n];
    cpx<T> out[R];
    out[0] = x0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cpx<T> re = a[0], im = {0, 0};
#pragma unroll
      for (int n = 1; n <= H; ++n) {
        const T c = (T)Trig<R>::c[(n * k) % R];
        const T s = (T)Trig<R>::s[(n * k) % R];
        re = re + scale(t[n], c);
        im = im + scale(d[n], s);
      }
      // forward: X_k = re - i im, X_{R-k} = re + i im ; inverse swaps
      cpx<T> ri = mul_i(im);
      out[k] = INV ? re + ri : re - ri;
      out[R - k] = INV ? re - ri : re + ri;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = out[k];
  }
};
template <typename T, bool INV> struct Dft<T, 3, INV> : DftOdd<T, 3, INV> {};
template <typename T, bool INV> struct Dft<T, 5, INV> : DftOdd<T, 5, INV> {};
template <typename T, bool INV> struct Dft<T, 7, INV> : DftOdd<T, 7, INV> {};

// One Stockham radix-R pass over `lines` transforms of length L held in LDS.
// Element (t, j) of line t sits at buf[t*sL + j*sJ].  Ns = product of the
// radices already applied.  Inputs j, j+L/R, ..., outputs (j/Ns)*Ns*R + j%Ns + m*Ns.
// Every thread keeps its butterflies in registers across one barrier, so the
// pass is in place.  Twiddles come from tw[] = exp(-2 pi i n / (L*tstride)).
template <typename T, int R, int BMAX, bool INV>
__device__ __forceinline__ void stockham_pass(cpx<T>* buf, int L, int Ns, int lines, int sL,
                                              int sJ, bool jfast, const cpx<T>* __restrict__ tw,
                                              int tstride) {
  const int LR = L / R;
  const int nb = lines * LR;
  const int tid = threadIdx.x;
  cpx<T> v[BMAX][R];
  const int span = Ns * R;
  const int tws = (L / span) * tstride;
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int b = tid + i * kThreads;
    if (b < nb) {
      int t, j;
      if (jfast) {
        t = b / LR;
        j = b - t * LR;
      } else {
        j = b / lines;
        t = b - j * lines;
      }
      const int k = j % Ns;
#pragma unroll
      for (int m = 0; m < R; ++m) v[i][m] = buf[t * sL + (j + m * LR) * sJ];
      if (Ns > 1) {
#pragma unroll
        for (int m = 1; m < R; ++m) {
          cpx<T> w = tw[m * k * tws];
          if (INV) w.y = -w.y;
          v[i][m] = v[i][m] * w;
        }
      }
      Dft<T, R, INV>::run(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int b = tid + i * kThreads;
    if (b < nb) {
      int t, j;
      if (jfast) {
        t = b / LR;
        j = b - t * LR;
      } else {
        j = b / lines;
        t = b - j * lines;
      }
      const int k = j % Ns;
      const int base = (j / Ns) * span + k;
#pragma unroll
      for (int m = 0; m < R; ++m) buf[t * sL + (base + m * Ns) * sJ] = v[i][m];
    }
  }
  __syncthreads();
}

// Full transform of `lines` lines of length plan.L in LDS (unnormalised).
// EMAX bounds the elements per thread: lines * L <= EMAX * kThreads.  The plan
// lists radices grouped as 8s, 4s, 2s, 7s, 5s, 3s; one loop per radix keeps the
// register allocation of each pass separate.
template <typename T, int EMAX, bool INV>
__device__ void lds_fft(cpx<T>* buf, const Plan& plan, int lines, int sL, int sJ, bool jfast,
                        const cpx<T>* __restrict__ tw, int tstride) {
  int Ns = 1, s = 0;
  const int L = plan.L;
#define HZ_PASSES(R)                                                                            \
  for (; s < plan.np && plan.radix[s] == R; ++s) {                                              \
    stockham_pass<T, R, (EMAX + R - 1) / R, INV>(buf, L, Ns, lines, sL, sJ, jfast, tw, tstride); \
    Ns *= R;                                                                                    \
  }
  HZ_PASSES(8)
  HZ_PASSES(4)
  HZ_PASSES(2)
  HZ_PASSES(7)
  HZ_PASSES(5)
  HZ_PASSES(3)
#undef HZ_PASSES
}

// Transform `lines` lines whose total may exceed EMAX*kThreads elements: the
// lines are processed in chunks that each respect the per-thread bound.
// Line t starts at buf + t*sL (element stride sJ).
template <typename T, int EMAX, bool INV>
__device__ void lds_fft_chunked(cpx<T>* buf, const Plan& plan, int lines, int sL, int sJ, bool jfast,
                                const cpx<T>* __restrict__ tw, int tstride) {
  const int per = max(1, (EMAX * kThreads) / plan.L);
  for (int t0 = 0; t0 < lines; t0 += per) {
    const int n = min(per, lines - t0);
    lds_fft<T, EMAX, INV>(buf + t0 * sL, plan, n, sL, sJ, jfast, tw, tstride);
  }
}

template <typename T>
constexpr int emax_of() { return sizeof(T) == 8 ? 8 : 16; }

}  // namespace hz
