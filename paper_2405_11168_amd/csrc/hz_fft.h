// Complex arithmetic, radix butterflies and the Stockham line transforms used by
// every FFT pass of the solver (gfx950, wave64).
//
// A transform of `lines` lines of length L = prod(radix) runs as Stockham
// passes.  The first pass may read straight from global memory and the last
// pass may write straight to global memory, so a two-pass length (e.g.
// 128 = 16 x 8) touches LDS once: HBM -> registers -> LDS -> registers -> HBM.
#pragma once
#include "hz_internal.h"

namespace hz {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

// Global-memory pointers.  Buffer pointers read from a descriptor are generic to
// the compiler, which then emits flat memory instructions (they count against the
// LDS wait counter too and need 64-bit address arithmetic per lane); casting them
// to the global address space gives global loads/stores with scalar bases.
#define HZ_GLB __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ HZ_GLB T* glb(T* p) { return (HZ_GLB T*)p; }
template <typename T>
__device__ __forceinline__ const HZ_GLB T* glb(const T* p) { return (const HZ_GLB T*)p; }
// complex element load/store through a global pointer (one 8- or 16-byte access)
template <typename T> struct Vec2;
template <> struct Vec2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <typename T>
__device__ __forceinline__ cpx<T> gld(const HZ_GLB cpx<T>* p) {
  const typename Vec2<T>::type v = *reinterpret_cast<const HZ_GLB typename Vec2<T>::type*>(p);
  return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void gst(HZ_GLB cpx<T>* p, cpx<T> a) {
  typename Vec2<T>::type v;
  v.x = a.x;
  v.y = a.y;
  *reinterpret_cast<HZ_GLB typename Vec2<T>::type*>(p) = v;
}

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
// cos/sin(2 pi e / 16), e = 0..9 (the exponents a radix-16 butterfly needs)
struct Trig16 {
  static constexpr double c[10] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173, 0.0,
                                   -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613, -1.0,
                                   -0.92387953251128675613};
  static constexpr double s[10] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613, 1.0,
                                   0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173, 0.0,
                                   -0.38268343236508977173};
};

// In-register DFT of length R: a[k] <- sum_n a[n] exp(-+2 pi i n k / R)
template <typename T, int R, bool INV> struct Dft;

template <typename T, bool INV> struct Dft<T, 1, INV> {
  static __device__ __forceinline__ void run(cpx<T>*) {}
};

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

// 16 = 4 x 4: DFT4 over n1 (stride 4), twiddle w16^(n2 k1), DFT4 over n2
template <typename T, bool INV> struct Dft<T, 16, INV> {
  static __device__ __forceinline__ void run(cpx<T>* a) {
    cpx<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cpx<T> z[4] = {a[n2], a[n2 + 4], a[n2 + 8], a[n2 + 12]};
      Dft<T, 4, INV>::run(z);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) {
        const int e = n2 * k1;
        if (e == 0) {
          y[n2][k1] = z[k1];
        } else {
          const cpx<T> w = {(T)Trig16::c[e], INV ? (T)Trig16::s[e] : -(T)Trig16::s[e]};
          y[n2][k1] = z[k1] * w;
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cpx<T> z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<T, 4, INV>::run(z);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = z[k2];
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

// ---------------------------------------------------------------------------
// element accessors: get(t, j) / put(t, j, v) for element j of line t
// ---------------------------------------------------------------------------
template <typename T>
struct LdsAcc {
  static constexpr bool kLds = true;
  cpx<T>* buf;
  int sL, sJ;
  __device__ __forceinline__ cpx<T> get(int t, int j) const { return buf[t * sL + j * sJ]; }
  __device__ __forceinline__ void put(int t, int j, cpx<T> v) const { buf[t * sL + j * sJ] = v; }
};

// LDS lines of unit element stride with one element of padding after every 16: the
// first Stockham pass writes a butterfly's outputs to consecutive positions, so the
// lanes of a wave write R elements apart, which without the padding puts them all on
// the same banks.  Element j of line t sits at t * sL + j + (j >> sh): sh = 4 pads
// (line pitch lds_pitch(L)), sh = 31 leaves the line unpadded (pitch L).
template <typename T>
struct LdsPad {
  static constexpr bool kLds = true;
  cpx<T>* buf;
  int sL, sh;
  __device__ __forceinline__ cpx<T> get(int t, int j) const { return buf[t * sL + j + (j >> sh)]; }
  __device__ __forceinline__ void put(int t, int j, cpx<T> v) const { buf[t * sL + j + (j >> sh)] = v; }
};

// global line storage: element (t, j) at p[(t / G) * B + (t % G) * sl + j * sj]
// (32-bit offsets: a problem's spectra stay below 2^31 elements)
template <typename T>
struct GblAcc {
  static constexpr bool kLds = false;
  HZ_GLB cpx<T>* p;
  int B, G, sl, sj;
  __device__ __forceinline__ int at(int t, int j) const {
    const int q = t / G;
    return q * B + (t - q * G) * sl + j * sj;
  }
  __device__ __forceinline__ cpx<T> get(int t, int j) const { return gld(p + at(t, j)); }
  __device__ __forceinline__ void put(int t, int j, cpx<T> v) const { gst(p + at(t, j), v); }
};

// floor(a / d) for 0 <= a < 2^19 given r = (1 + 2^-20)/d rounded up (see Plan)
__device__ __forceinline__ int fdiv(int a, float r) { return (int)((float)a * r); }

__device__ __forceinline__ void line_map(int b, int lines, int LR, float rLR, float rlines, bool jfast, int& t,
                                         int& j) {
  if (jfast) {
    t = fdiv(b, rLR);
    j = b - t * LR;
  } else {
    j = fdiv(b, rlines);
    t = b - j * lines;
  }
}

// One radix-R Stockham pass: inputs j, j+L/R, ...; outputs (j/Ns)*Ns*R + j%Ns + m*Ns.
// Twiddles exp(-+2 pi i m k / (Ns R)) come from tw[] = exp(-2 pi i n / (L*tstride)).
// `inplace` puts a barrier between reading src and writing dst (same LDS buffer).
template <typename T, int R, int BMAX, bool INV, class SRC, class DST>
__device__ __forceinline__ void pass_gen(int L, int Ns, int lines, bool jfast, const cpx<T>* __restrict__ tw,
                                         int tstride, const SRC& src, const DST& dst, bool inplace, float rLR,
                                         float rNs, float rlines) {
  const int LR = L / R;
  const int nb = lines * LR;
  const int tid = threadIdx.x;
  const int span = Ns * R;
  const int tws = (L / span) * tstride;
  cpx<T> v[BMAX][R];
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int b = tid + i * kThreads;
    if (b < nb) {
      int t, j;
      line_map(b, lines, LR, rLR, rlines, jfast, t, j);
#pragma unroll
      for (int m = 0; m < R; ++m) v[i][m] = src.get(t, j + m * LR);
    }
  }
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int b = tid + i * kThreads;
    if (b < nb) {
      if (Ns > 1) {
        int t, j;
        line_map(b, lines, LR, rLR, rlines, jfast, t, j);
        const int k = j - fdiv(j, rNs) * Ns;
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
  if (inplace) __syncthreads();
#pragma unroll
  for (int i = 0; i < BMAX; ++i) {
    const int b = tid + i * kThreads;
    if (b < nb) {
      int t, j;
      line_map(b, lines, LR, rLR, rlines, jfast, t, j);
      const int q = fdiv(j, rNs);
      const int k = j - q * Ns;
      const int base = q * span + k;
#pragma unroll
      for (int m = 0; m < R; ++m) dst.put(t, base + m * Ns, v[i][m]);
    }
  }
}

template <int EMAX, int R>
constexpr int bmax() { return (EMAX + R - 1) / R; }

template <typename T, int EMAX, bool INV, class SRC, class DST>
__device__ __forceinline__ void pass_any(int R, int L, int Ns, int lines, bool jfast, const cpx<T>* __restrict__ tw,
                                         int tstride, const SRC& src, const DST& dst, bool inplace, float rLR,
                                         float rNs, float rl) {
#define HZ_CASE(RR)                                                                                      \
  case RR:                                                                                               \
    pass_gen<T, RR, bmax<EMAX, RR>(), INV>(L, Ns, lines, jfast, tw, tstride, src, dst, inplace, rLR, rNs, rl); \
    break;
  switch (R) {
    HZ_CASE(16)
    HZ_CASE(8)
    HZ_CASE(4)
    HZ_CASE(2)
    HZ_CASE(7)
    HZ_CASE(5)
    default:
      pass_gen<T, 3, bmax<EMAX, 3>(), INV>(L, Ns, lines, jfast, tw, tstride, src, dst, inplace, rLR, rNs, rl);
      break;
  }
#undef HZ_CASE
}

// Whole transform of `lines` lines (lines * L <= EMAX * kThreads), unnormalised.
// src -> [first pass] -> lds -> [middle passes] -> lds -> [last pass] -> dst.
// The plan lists radices grouped 16s, 8s, 4s, 2s, 7s, 5s, 3s; the middle passes
// run one loop per radix so each keeps its own register allocation.  When dst
// is LDS the caller synchronises before reading it; when src is LDS the caller
// synchronised after filling it.
template <typename T, int EMAX, bool INV, class LDS, class SRC, class DST>
__device__ __forceinline__ void fft_lines(const Plan& plan, int lines, float rlines, bool jfast,
                                          const cpx<T>* __restrict__ tw, int tstride, const LDS& lds,
                                          const SRC& src, const DST& dst) {
  const int np = plan.np, L = plan.L;
  if (np == 0) {  // L == 1: copy
    for (int t = threadIdx.x; t < lines; t += kThreads) dst.put(t, 0, src.get(t, 0));
    return;
  }
  if (np == 1) {
    pass_any<T, EMAX, INV>(plan.radix[0], L, 1, lines, jfast, tw, tstride, src, dst, SRC::kLds && DST::kLds,
                           plan.rLR[0], plan.rNs[0], rlines);
    return;
  }
  pass_any<T, EMAX, INV>(plan.radix[0], L, 1, lines, jfast, tw, tstride, src, lds, SRC::kLds, plan.rLR[0],
                         plan.rNs[0], rlines);
  __syncthreads();
  int Ns = plan.radix[0], s = 1;
#define HZ_MID(R)                                                                                         \
  for (; s < np - 1 && plan.radix[s] == R; ++s) {                                                         \
    pass_gen<T, R, bmax<EMAX, R>(), INV>(L, Ns, lines, jfast, tw, tstride, lds, lds, true, plan.rLR[s],    \
                                         plan.rNs[s], rlines);                                            \
    __syncthreads();                                                                                      \
    Ns *= R;                                                                                              \
  }
  HZ_MID(16)
  HZ_MID(8)
  HZ_MID(4)
  HZ_MID(2)
  HZ_MID(7)
  HZ_MID(5)
  HZ_MID(3)
#undef HZ_MID
  pass_any<T, EMAX, INV>(plan.radix[np - 1], L, Ns, lines, jfast, tw, tstride, lds, dst, DST::kLds,
                         plan.rLR[np - 1], plan.rNs[np - 1], rlines);
}

// elements per thread in one transform call (bounds register use)
template <typename T>
constexpr int emax() { return sizeof(T) == 8 ? 16 : 32; }

}  // namespace hz
