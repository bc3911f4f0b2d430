// Internal structures shared by the HIP kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <set>
#include <utility>

namespace hz {

constexpr int kThreads = 256;   // work-group size of every kernel (4 wave64)
constexpr int kMaxPasses = 16;

// Factorisation of a transform length into Stockham radix passes.
// Index arithmetic in the kernels divides by these lengths through exact float
// reciprocals: floor(a / d) = int(float(a) * r) with r = (1 + 2^-20) / d rounded up,
// exact for 0 <= a < 2^19.
struct Plan {
  int L;
  int np;
  int radix[kMaxPasses];
  float rLR[kMaxPasses];   // 1 / (L / radix[s])
  float rNs[kMaxPasses];   // 1 / (radix[0] * ... * radix[s-1])
};

// Spectral storage is [comp][h1][h3][h2] with h1 in [0, N1/2] outermost, so the
// y and z transforms read unit-stride rows and no tile is ragged in h1.
struct Geo {
  int N1, N2, N3;
  int H1;          // N1/2 + 1
  long long S;     // H1 * N3 * N2 : complex elements per component
  long long N;     // N1 * N2 * N3
};

// Dynamic LDS of a work-group beyond 64 KB (gfx950 has 160 KB per CU; the z kernels of
// some grids and the stencil kernel with a stiffness table take more) needs the kernel's
// limit raised before the launch: once per kernel and device, to 96 KB, so launches
// (also under stream capture) make no further runtime call.
constexpr int kLdsDynMax = 96 * 1024;
inline hipError_t allow_lds_once(const void* kernel) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count({kernel, dev})) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsDynMax);
  if (e == hipSuccess) done.insert({kernel, dev});
  return e;
}
template <class F>
inline hipError_t allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 65536 - 512) return hipSuccess;  // room for the kernels' static LDS
  if (bytes > (size_t)kLdsDynMax) return hipErrorInvalidValue;
  return allow_lds_once(reinterpret_cast<const void*>(kernel));
}

// Gradient discretisation: the tetrahedral stencil, or one of the comparison
// operators of the paper's experiments (same values as HZ_GREEN_* of the C ABI)
enum { GREEN_TETRA = 0, GREEN_ROTATED = 1, GREEN_CONTINUOUS = 2 };

// Material kind of a problem, which selects the instantiation of the kernels that
// apply the constitutive law: every phase isotropic, and eigenstrains present.
enum { KIND_ISO = 1, KIND_EIG = 2 };

// Pitch of an LDS line of L complex values stored with one element of padding after
// every 16 (the y transforms' layout wherever such a line fits).
__host__ __device__ constexpr int lds_pitch(int L) { return L + (L >> 4); }

// Per-problem descriptor.  One launch serves many same-shape problems (load
// cases of one grid, or requests of a serving group); blockIdx.y picks one.
struct Desc {
  void* spec;            // 12 strain/stress spectra, kernel precision
  void* u[2];            // displacement spectra (3 comps), ping-pong, kernel precision
  void* u64;             // refinement: FP64 anchor U (3 comps)
  void* r32;             // refinement: FP64-sweep residual stored in FP32 (3 comps)
  void* state;           // strain-based form: the 12 strain spectra (the iterate), kernel precision
  const uint16_t* phase; // [N3][N2][N1]
  const double* C64;     // [n_phases][24] Voigt upper triangle (21 used), or (lambda, mu) pairs if iso
  const float* C32;      // same in FP32
  int iso;               // 1: every phase isotropic, tables hold (lambda, mu)
  int c0_iso;            // 1: reference medium isotropic with (lam0, mu0)
  double lam0, mu0;
  double* part_sig;      // [nbx][6] FP64 partial sums of (sigma^T1 + sigma^T2)/2
  double* part_res;      // [nbq] FP64 partial sums of w |r/2|^2
  double* status;        // [kStatusLen] device-side state, see St below
  double* eps_out;       // optional real-space output fields [6][N] FP64
  double* sig_out;
  double* trace;         // optional [max_iters+1][7]: eps_k, <sigma>_k
  const double* tau64;   // optional [n_phases][8] eigenstress lambda_p:eps0_p (tensor comps), or null
  const float* tau32;    // same in FP32
  double sig_a[6];       // applied stress (stress loading), tensor comps
  double S0[36];         // stress loading: lambda0^-1 acting on tensor comps, row-major
  double sref;           // stress loading: fixed stress scale of the stop rule
  int loading;           // 0 applied mean strain, 1 applied stress (Sec. 2.5)
  int n_phases;          // rows of the stiffness tables
  double C0[81];         // reference medium, full 3x3x3x3 tensor
  double tol;
  int max_iters;
  int fixed_iters;
  int trace_len;
  int cmode;             // contraction: 0 update u, 1 FP64 sweep (store r), 2 update with r32 added,
                         // 3 strain-based form: store w = Omega r in u[0] (applied to the strains next)
  int fmode;             // stop rule: 0 plain, 1 sweep (measure only), 2 correction round, 3 FP32 round 0
  int src;               // expansion source: 0 u[parity], 1 FP64 anchor u64
  int inner_max;         // iteration cap of FP32 rounds
  int green;             // GREEN_TETRA, or a comparison operator (spectral form only)
};
// The ping-pong slot of the current iterate is status[ST_K] & 1: every problem
// counts its own measured iterates, so problems that started at different times
// can share a launch.

// Layout of Desc::status (doubles; integers stored exactly)
enum St {
  ST_DONE = 0,       // 1 once the stop rule fired (kernels of later iterations skip)
  ST_ITERS = 1,      // iterate index k at which it stopped
  ST_PARITY = 2,     // u[] slot holding u_k
  ST_ERR = 3,        // eps_k of the last measured iterate
  ST_MEAN = 4,       // 4..9 <sigma>_k
  ST_L2SQ = 10,      // sum w |r/2|^2
  ST_K = 11,         // iterations measured so far
  ST_FIRST_ERR = 12, // eps_0 (divergence watchdog)
  ST_NORM = 13,      // ||<sigma>|| used for the criterion
  ST_REF = 14,       // inner refinement: reference residual level to reach
  ST_BEST = 15,      // smallest residual seen (watchdog; inner refinement: best at a 32-step mark)
  ST_EBAR = 16,      // 16..21 mean strain Ebar of the current iterate (tensor comps): the
                     // applied strain, zero in a correction round, or under applied stress
                     // the iterate of the loop on the mean strain (updated on the device)
  ST_K1E6 = 22,      // FP64 iterations: first iterate k with eps_k < 1e-6 in this state, or -1
  ST_L2_FIRST = 23,  // FP64 iterations: the residual norm L2 of the state's first iterate (watchdog)
};
constexpr int kStatusLen = 24;

// z pass geometry (expand + inverse z, or forward z + contraction): a tile is TX
// adjacent h2 columns of one h1 plane, all N3 elements, 3 displacement components.
struct ZGeo {
  int N1, N2, N3, H1, TX, tiles;   // tiles = N2 / TX
  float rTX, rLines, rTiles;       // reciprocals of TX, 3 TX, tiles
  long long S;
};

// y pass geometry: contiguous rows of length N2, TX rows per tile
struct YGeo {
  int N2, TX;
  long long nlines;                 // fields * H1 * N3
  long long off;                    // first line's element offset in the spectra (complex elements)
  int from_state;                   // 1: read the lines from the problem's displacement state
                                    // (stencil form), write them to the spectra at off
  int pitch, pshift;                // LDS line pitch; element j at j + (j >> pshift): 4 pads
                                    // after every 16 elements, 31 leaves the line unpadded
};

// Stencil form (same iterates as the Fourier form, eqs. DA1-DA2 in real space).
// Its displacement state u[] (and the FP64 anchor) is held in the mixed domain
// [3][h1][l3][h2] (inverse z transform of u(q)); it is converted from u(q) when a
// solve starts from a given displacement and back to u(q) when a problem finishes.
// Spectra slots of one load, in complex elements of the 12-field buffer:
//   0..2  u: inverse y of the mixed-domain state, half spectrum along x  [3][h1][l3][l2]
//   3..5  u on the corner grid, real                                [3][l3][l2][l1]
//   6..8  corner force g = sum_T sigma^T(c - o) . w(o), real        [3][l3][l2][l1]
//   9..11 g: forward x (1/N) then forward y                         [3][h1][l3][h2]
// Real fields of N values start at element offset slot*S + c*N/2.
// stencil tile: 64 corners along x (one per lane of a wave), one corner row per wave
// along y (kStY = kThreads / 64), and at most kStZ corner planes per block along z
#ifndef HZ_STZ
#define HZ_STZ 32
#endif
constexpr int kStX = 64, kStY = kThreads / 64, kStZ = HZ_STZ;
struct SGeo {
  int N1, N2, N3;
  int TZ;                 // corner planes per block (z segment)
  int tx, ty, tz;         // tiles along x, y, z
};

// fused x pass geometry
struct XGeo {
  int N1, N2, N3, H1, H1p, TY, M;
  float rTY, rKH, rM;     // reciprocals of TY, M/2+1, M
  long long S;
  double invN;
  int fields;            // write real-space eps/sigma (T1/T2 averages)
  int half;              // -1: both tetrahedra (two blocks per row tile); 0/1: only T1/T2
  float rNI, rLRm;       // fused form: reciprocals of (M/r0)/2 + 1 and of M/r_last
};

struct FinGeo {
  int nbx, nbq;
  double invN;
};

}  // namespace hz
