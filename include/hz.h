/*
 * hz.h -- C ABI of the MI355X (gfx950) solver for the tetrahedral-stencil
 * FFT homogenization method of A. Finel, "A fast and robust discrete
 * FFT-based solver for computational homogenization" (arXiv 2405.11168).
 *
 * The library iterates the displacement-based basic scheme of the paper's
 * Algorithm 1 (Sec. 2.6) on a periodic N1 x N2 x N3 voxel grid:
 *
 *   1. eps^T1(q) = D(q) (x)_s u(q),  eps^T2(q) = -conj(D(q)) (x)_s u(q)   (eq. deps_dep_Q)
 *   2. inverse FFT of the twelve strain components                          (eq. IFT_1)
 *   3. sigma^Tk(r) = lambda(r) : (Ebar + eps^Tk(r) - eps0(r))                (eq. linear_elasticity_Kk)
 *   4. forward FFT                                                          (eq. FT)
 *   5. u(q) <- u(q) - Omega(q).{sigma^T1(q).conj(D(q)) - sigma^T2(q).D(q)}   (eq. basic_scheme_dep_2)
 *
 * with D of eq. Dq, Omega of eq. Green_tensor (set to 0 at q = 0 and q = (pi,pi,pi)),
 * and the convergence measure eps = L2/||<sigma>|| of eqs. L2-norm and tolerance.
 * Under an applied stress (Sec. 2.5) the mean strain Ebar is an unknown too:
 *
 *   6. Ebar <- lambda0^-1 : {sigma^a + (lambda0 - <lambda>):Ebar - <lambda:deps> + <lambda:eps0>}
 *
 * starting from Ebar = lambda0^-1 : sigma^a.  Per-phase eigenstrains eps0 are optional.
 * Every step runs in hand-written HIP kernels on device-resident fields.
 *
 * Conventions
 *   - Grid sizes: every N_i even and >= 2 (Sec. 2.1), prime factors in {2,3,5,7};
 *     N1 <= 4096, N2, N3 <= 2048.
 *   - Phase map: uint16 [n3][n2][n1], x fastest.
 *   - Stiffness: engineering-shear Voigt 6x6, row-major, order (11,22,33,23,13,12):
 *     sigma_I = C_IJ gamma_J with gamma = (e11,e22,e33,2e23,2e13,2e12).
 *   - Macroscopic strains E and mean stresses: tensor components (11,22,33,23,13,12).
 *   - Voxel size d = 1 (results do not depend on it).
 *
 * Ownership
 *   - The caller owns every host array; the library copies what it needs.
 *   - All device memory the solver touches is one caller-owned workspace
 *     (hz_workspace_bytes / hz_bind_workspace); the library never allocates
 *     device memory.  Work is issued on the caller's HIP stream.
 *   - A handle is used by one host thread at a time; handles are independent.
 *
 * Errors: every int-returning call returns HZ_OK (0) or one of the codes
 * below; no C++ exception crosses the ABI and hz_last_error() gives a
 * thread-local message for the last failing call.
 */
#ifndef HZ_H
#define HZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HZ_OK 0
#define HZ_NOT_CONVERGED 1   /* max_iters reached; outputs written from the last iterate  */
#define HZ_STAGNATED 2       /* reserved, not returned: a refinement that stops gaining (3
                                FP64 sweeps in a row under 10%, or a correction that
                                diverges) continues as plain FP64 iterations from its FP64
                                anchor U instead (hz_info.precision_used = HZ_FP64)        */
#define HZ_PENDING 3         /* hz_server_query: the request has not finished yet          */
#define HZ_EINVAL (-1)       /* NULL pointer, size <= 0, unsupported size or option        */
#define HZ_EODD (-2)         /* a grid dimension is odd (the scheme needs even N_i)        */
#define HZ_ENOMATERIAL (-3)  /* hz_set_material not called                                */
#define HZ_ENOTSPD (-4)      /* a stiffness is not positive semi-definite, or the
                                reference medium is not positive definite                */
#define HZ_EWORKSPACE (-5)   /* workspace not bound or too small                           */
#define HZ_EHIP (-6)         /* a HIP runtime call failed                                  */
#define HZ_EDIVERGED (-7)    /* residual became NaN/Inf, eps grew by 1e3, or the residual
                                norm grew back above its first value and 10 times its
                                smallest (reference medium too soft)                      */

typedef struct hz_grid_s* hz_grid;

/* Arithmetic of the iteration.  HZ_FP64: every kernel in FP64.
 * HZ_FP32_REFINE: fields and FFTs in FP32 on a correction, anchored by FP64
 * sweeps of the full pipeline; the stop decision is always an FP64 residual. */
#define HZ_FP64 0
#define HZ_FP32_REFINE 1

/* Realisation of the iteration; both give the same iterates (eq. Dq is the
 * Fourier symbol of the real-space stencils of eqs. DA1-DA2).
 * HZ_SCHEME_SPECTRAL: Algorithm 1 as written, the 12 strain/stress components
 *   through the transforms.
 * HZ_SCHEME_STENCIL: strains and corner forces by the 4-corner stencils in real
 *   space, so only the 3 displacement and 3 force components are transformed
 *   (available for every grid the library accepts, see hz_scheme_available).
 * HZ_SCHEME_AUTO: the stencil form where available, else the spectral one. */
#define HZ_SCHEME_AUTO 0
#define HZ_SCHEME_SPECTRAL 1
#define HZ_SCHEME_STENCIL 2
#define HZ_SCHEME_STRAIN 3   /* the strain-based Algorithm 2: the 12 strain spectra are the iterate,
                                updated by Gamma(q).r (eq. Lippmann_Schwinger_strain_3); the same
                                iterates as Algorithm 1 at more bytes per iteration.  HZ_FP64 and
                                hz_solve only; needs a workspace bound for 2 n_loads loads;
                                hz_get_displacement is not available after it. */

/* Loading (Sec. 2.3 and Sec. 2.5).  Under HZ_LOAD_STRESS the six numbers of a load
 * are the applied stress sigma^a; the run stops at the first iterate k with
 *   L2_k / s < tol  and  ||<sigma>_k - sigma^a|| <= tol * s
 * where s = ||sigma^a|| (Frobenius), or ||<lambda:eps0>|| when sigma^a = 0 (then
 * <sigma> tends to zero, and the measure of eq. tolerance is undefined), or 1 when
 * both vanish.  HZ_LOAD_STRESS needs HZ_FP64. */
#define HZ_LOAD_STRAIN 0
#define HZ_LOAD_STRESS 1

/* Discretisation of the gradient (the Green operator).
 * HZ_GREEN_TETRA: the paper's tetrahedral stencil (eqs. Dq, DA1-DA2, Green_tensor).
 * The two others are the comparison discretisations of Sec. 3.2 and Appendix B: one
 * strain field per voxel, eps = Ebar + D (x)_s u, the inverse displacement Green
 * function conj(D).lambda0.D (eq. inverse_displacement_Green_function_rotated), the
 * equilibrium residual r = sigma(q).conj(D) and the update u <- u - Omega.r; the
 * stop measure is eps_k = ||r|| / ||<sigma>|| (eq. tolerance for one strain field).
 * HZ_GREEN_ROTATED: Willot's rotated scheme, D of eq. Dq_rotated (differences over the
 *   8 corners of a voxel); Omega := 0 where D vanishes: q = 0 and every q with two
 *   components equal to pi (Willot's recipe, Sec. 3.2).
 * HZ_GREEN_CONTINUOUS: the continuous-frequency gradient of Moulinec-Suquet,
 *   D = i xi(q) with xi = 2 pi h~ / N on the representative h~ in (-N/2, N/2); at the
 *   highest frequency of an even axis xi = 0, so the strain stays real (the paper's
 *   runs use Moulinec-Suquet's strain-based recipe there instead, which has no
 *   displacement form); Omega := 0 where xi = 0.  Needs N3 <= 680.
 * Both need HZ_FP64 and the spectral scheme (HZ_SCHEME_AUTO selects it); hz_solve,
 * hz_solve_static and hz_effective_stiffness only (not served).  hz_get_displacement
 * then returns exp(i (q1 + q2 + q3)) u(q) for u(q) of eq. Dq_rotated (rotated), and
 * u(q) itself (continuous). */
#define HZ_GREEN_TETRA 0
#define HZ_GREEN_ROTATED 1
#define HZ_GREEN_CONTINUOUS 2

typedef struct {
  double tol;               /* stop at the first iterate k with eps_k < tol (eq. tolerance)   */
  int32_t max_iters;        /* cap on updates, <= 1000000 (<= 4096 with a trace): FP64 updates,
                               or for HZ_FP32_REFINE the FP32 inner updates plus the FP64
                               updates of a fallback to plain FP64 iterations                 */
  int32_t precision;        /* HZ_FP64 or HZ_FP32_REFINE                                        */
  int32_t ref_mode;         /* 0: automatic reference medium; 1: use ref_C                      */
  double ref_C[36];         /* reference medium lambda0, Voigt 6x6, when ref_mode = 1           */
  int32_t fixed_iters;      /* >= 0: run exactly this many updates, ignore tol (parity tests,
                               fixed-work timing).  HZ_FP32_REFINE: >= 1 FP32 updates from
                               u = 0 (no stop rule, no corrections), then one FP64 sweep that
                               measures eps and <sigma> of the result; not served            */
  int32_t check_every;      /* host looks at the device stop flags every this many iterations  */
  double* trace_residual;   /* optional [n_loads][max_iters+1]: eps_k of every iterate (FP64);
                               needs max_iters (or fixed_iters) <= 4096                       */
  double* trace_mean;       /* optional [n_loads][max_iters+1][6]: <sigma>_k                    */
  double inner_rho;         /* refinement: inner loop stops at rho * eps of its FP64 sweep      */
  int32_t inner_max;        /* refinement: cap on inner iterations per outer round              */
  int32_t scheme;           /* HZ_SCHEME_AUTO, _SPECTRAL, _STENCIL or _STRAIN                     */
  int32_t loading;          /* HZ_LOAD_STRAIN (E is the mean strain) or HZ_LOAD_STRESS            */
  const double* u_init;     /* optional [n_loads][3][n1/2+1][n3][n2] complex (re,im) FP64 in the
                               layout and phase convention of hz_get_displacement: iterate 0 is
                               this displacement instead of 0 (resume from a checkpoint).  HZ_FP64,
                               spectral or stencil scheme, hz_solve only; NULL: start from 0.
                               The resumed iterates equal those of an uninterrupted solve bit for
                               bit in the spectral scheme and to rounding in the stencil scheme,
                               which holds the displacement as its inverse z transform while it
                               iterates                                                         */
  const double* Ebar_init;  /* optional [n_loads][6]: under HZ_LOAD_STRESS, the mean strain of
                               iterate 0 (hz_info.Ebar of the checkpoint); NULL: lambda0^-1:sigma^a */
  int32_t fields_on_device; /* 0: eps_out / sig_out of hz_solve are host arrays; 1: device
                               arrays (caller-owned, 8-byte aligned), written on the bound
                               stream before hz_solve returns                                  */
  int32_t green;            /* HZ_GREEN_TETRA, HZ_GREEN_ROTATED or HZ_GREEN_CONTINUOUS           */
} hz_opts;

typedef struct {
  int32_t status;           /* HZ_OK, HZ_NOT_CONVERGED, HZ_STAGNATED or HZ_EDIVERGED           */
  int32_t iters;            /* updates applied to the reported iterate                          */
  int32_t outer_rounds;     /* FP64 sweeps (refinement); 0 for HZ_FP64                          */
  int32_t precision_used;   /* HZ_FP32_REFINE, or HZ_FP64: an FP64 solve, or a refinement that
                               fell back to FP64 iterations for the rest of its budget          */
  double residual;          /* eps of the reported iterate, measured in FP64                    */
  double seconds;           /* device time from solve start to the reported iterate            */
  double seconds_to_1e6;    /* device time to the first FP64-verified eps < 1e-6 (an FP64
                               iterate or an FP64 sweep of the refinement), or -1             */
  double wall_seconds;      /* host wall time: the hz_solve call, or a served request from
                               submission to the step that saw it finish (queueing included)     */
  double Ebar[6];           /* mean strain of the reported iterate (tensor comps): the applied
                               strain, or the converged loop of Sec. 2.5 under applied stress     */
} hz_info;

/* Fill *o with defaults: tol 1e-8, max_iters 2000, HZ_FP64, automatic reference,
 * fixed_iters -1, check_every 8, no traces, inner_rho 1e-3, inner_max 400,
 * HZ_SCHEME_AUTO, HZ_LOAD_STRAIN, no initial guess, host field outputs, HZ_GREEN_TETRA. */
void hz_default_opts(hz_opts* o);

/* Create a grid handle for an n1 x n2 x n3 periodic cell (Sec. 2.1).
 * Returns HZ_EODD for an odd size, HZ_EINVAL for other unsupported sizes. */
int hz_create_grid(int32_t n1, int32_t n2, int32_t n3, hz_grid* out);

/* Set the microstructure: the stiffness field lambda(r) of the constitutive law
 * sigma = lambda(r):(eps - eps0) (eq. linear_elasticity, Sec. 2.1), piecewise
 * constant over the voxels of the simple-cubic grid, as n_phases stiffness matrices
 * C_voigt[n_phases][6][6] and the phase id of every voxel phase[n3][n2][n1]
 * (< n_phases).  Each matrix must be symmetric and positive semi-definite
 * (HZ_ENOTSPD otherwise); zero stiffness (voids) is allowed.  Host arrays are
 * copied; device copies are made by hz_bind_workspace.  Clears eigenstrains set
 * before.  HZ_EINVAL for NULL pointers, n_phases outside [1, 65536] or a phase id
 * out of range. */
int hz_set_material(hz_grid g, int32_t n_phases, const double* C_voigt, const uint16_t* phase);

/* Per-phase eigenstrains eps0[n_phases][6] (tensor comps; eq. linear_elasticity:
 * sigma = lambda:(eps - eps0)), for the material currently set; NULL clears them.
 * Copied; hz_set_material clears them.  Like a material change, it takes effect at
 * the next hz_bind_workspace (requests already submitted to a server keep theirs).
 * HZ_ENOMATERIAL before hz_set_material, HZ_EINVAL for a row count other than the
 * material's phase count or a non-finite entry. */
int hz_set_eigenstrain(hz_grid g, int32_t n_phases, const double* eps0);

/* Bytes of device workspace needed to solve up to n_loads load cases at once
 * in the given precision; negative error code on invalid arguments. */
int64_t hz_workspace_bytes(hz_grid g, int32_t precision, int32_t n_loads);

/* Bind a caller-owned device buffer (>= hz_workspace_bytes(g, precision, n_loads),
 * 256-byte aligned) and the HIP stream (hipStream_t, may be NULL) all work is issued
 * on, and upload the material and tables into it.  Must follow hz_set_material;
 * call again after changing the material. */
int hz_bind_workspace(hz_grid g, void* dev_ptr, int64_t bytes, void* hip_stream,
                      int32_t precision, int32_t n_loads);

/* Solve n_loads problems: applied mean strains E[n_loads][6] (HZ_LOAD_STRAIN, Sec. 2.3:
 * the mean strain equals the applied strain) or applied stresses (HZ_LOAD_STRESS,
 * Sec. 2.5), tensor comps.
 * Outputs (each may be NULL):
 *   sigma_mean[n_loads][6]  <sigma> of the reported iterate (FP64)
 *   eps_out, sig_out        [n_loads][6][n3][n2][n1] FP64 fields of eq. final_fields,
 *                           host arrays, or device arrays with o->fields_on_device
 *   info[n_loads]
 * Returns the worst per-load status (negative codes first). */
int hz_solve(hz_grid g, int32_t n_loads, const double* E, const hz_opts* o,
             double* sigma_mean, double* eps_out, double* sig_out, hz_info* info);

/* hz_solve on the library's own static device workspace instead of a bound one, for
 * callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same arguments, outputs and
 * status as hz_solve, plus the HIP stream (hipStream_t of the current device, may be
 * NULL) the work is issued on.  No workspace needs to be bound; the grid's own
 * binding, and the loads hz_get_displacement reads, are left as they were.
 * Memory: one static array of 256 MiB per GPU (allocated when the library's code is
 * loaded on that device, held until the process ends); the problem must fit it,
 * i.e. hz_workspace_bytes(g, o->precision, n_loads) (2 n_loads for
 * HZ_SCHEME_STRAIN) <= 268435456, else HZ_EWORKSPACE.  The call uses no device or
 * pinned-host allocator (no hipMalloc, hipHostMalloc, hipFree); host bookkeeping uses
 * the C++ heap.  Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents (each solve clears what it needs zeroed itself): calls that overlap
 * on one GPU, from several threads or on several streams, race. */
int hz_solve_static(hz_grid g, void* hip_stream, int32_t n_loads, const double* E, const hz_opts* o,
                    double* sigma_mean, double* eps_out, double* sig_out, hz_info* info);

/* Effective stiffness: the six unit load cases (gamma_J = 1) solved as one batch;
 * column J of C_eff (row-major 6x6 engineering Voigt) is <sigma> of case J, the
 * volume average of the stress field of eq. final_fields at the reported iterate.
 * Needs a workspace bound for n_loads >= 6, strain loading and a material without
 * eigenstrains (HZ_EINVAL otherwise).  info may be NULL; traces in *o are [6][...]. */
int hz_effective_stiffness(hz_grid g, const hz_opts* o, double C_eff[36], hz_info info[6]);

/* Copy the displacement spectrum of load `load` after the last solve to host:
 * out[3][n1/2+1][n3][n2] complex (interleaved re,im) FP64, in the library's phase
 * convention u~(q) = exp(i q.(1/2,1/2,1/2)) u(q) (u(q) of eq. FT_u). */
int hz_get_displacement(hz_grid g, int32_t load, double* out);

/* 1 if the grid's sizes allow the given scheme (HZ_SCHEME_SPECTRAL and
 * HZ_SCHEME_STENCIL: every grid hz_create_grid accepts, the stencil form's x
 * transforms taking an odd first radix, or one pass, where N1/2 has no factor 2),
 * 0 if not, negative error code on invalid arguments. */
int hz_scheme_available(hz_grid g, int32_t scheme);

/* Reference medium the automatic rule picks for a set of phases: isotropic with
 * nu0 = 0 and Mandel modulus at the midpoint of the smallest and largest Mandel
 * eigenvalue over all phases (pure host function). */
int hz_reference_medium(int32_t n_phases, const double* C_voigt, double C0_out[36]);

/* Per-kernel device timing with HIP events on the bound stream.
 * hz_profile(g, 1) starts recording every launch (and clears totals); hz_profile(g, 2 + i)
 * records only the launches of entry i of hz_profile_read (one kernel kind and precision,
 * so the other launches carry no events); hz_profile(g, 0) stops.  HZ_EINVAL for other
 * values.  hz_profile_read fills up to max entries: name (static string), total ms,
 * launches; returns the number of entries (kernel kinds x 2 precisions). */
int hz_profile(hz_grid g, int32_t enable);
int hz_profile_read(hz_grid g, int32_t max, const char** names, double* total_ms, int64_t* launches);

void hz_destroy_grid(hz_grid g);
const char* hz_last_error(void);

/* ------------------------------------------------------------------------
 * Solve server: continuous batching of homogenization requests.
 *
 * A request is one grid's material (as set when it is submitted) with n_loads
 * applied strains and its own options; requests on different grids, shapes,
 * materials and precisions run together.  hz_server_step performs one tick:
 * it admits queued requests in arrival order while their buffers fit the
 * server's workspace and slots, runs check_every iterations of every active
 * load (one launch per pass for all loads of one grid shape and kernel
 * precision), reads the device stop flags once and retires the requests whose
 * loads have all stopped, freeing their memory for the queue.  Each load keeps
 * its own buffers, descriptor and device-side stop rule, so a request's
 * results do not depend on what else is being served.
 *
 * Memory: one caller-owned device buffer; the first hz_server_bytes(max_problems)
 * bytes hold the server tables, the rest is an arena for per-shape tables,
 * per-material tables (shared by requests on the same material) and per-load
 * buffers (hz_request_bytes).  The library allocates no device memory.
 * A server is driven from one host thread; it owns its stream's ordering.
 * After an HZ_EHIP error the server must be destroyed.
 * ------------------------------------------------------------------------ */
typedef struct hz_server_s* hz_server;

/* Bytes of the fixed server tables for up to max_problems loads in flight. */
int64_t hz_server_bytes(int32_t max_problems);

/* Arena bytes one request needs: its per-load buffers plus the shape and
 * material tables (the latter two are shared when already resident). */
int64_t hz_request_bytes(hz_grid g, int32_t precision, int32_t n_loads);

/* Create a server on a caller-owned device buffer (256-byte aligned) and HIP
 * stream (may be NULL).  max_problems bounds the loads in flight (<= 4096);
 * check_every is the number of iterations per tick. */
int hz_server_create(void* dev_ptr, int64_t bytes, void* hip_stream, int32_t max_problems,
                     int32_t check_every, hz_server* out);

/* Queue a request: the material currently set on g, with its eigenstrains (shared,
 * copy-on-write: a later hz_set_material or hz_set_eigenstrain on g does not affect
 * it), n_loads loads E[n_loads][6] and options o (tol, max_iters, precision,
 * reference medium, inner_rho, inner_max, scheme, loading; fixed_iters and traces
 * are not served).  Writes the request id.
 * HZ_EWORKSPACE if the request could never fit the workspace or slots. */
int hz_server_submit(hz_server s, hz_grid g, int32_t n_loads, const double* E, const hz_opts* o,
                     int64_t* id);

/* One tick (admit, iterate, retire); *completed = requests finished in it. */
int hz_server_step(hz_server s, int32_t* completed);

/* HZ_PENDING while queued or running; once finished, fills sigma_mean[n_loads][6]
 * and info[n_loads] (seconds counted from the tick the request started) and
 * returns its worst per-load status as hz_solve does.  Either output may be NULL. */
int hz_server_query(hz_server s, int64_t id, double* sigma_mean, hz_info* info);

/* Forget a finished request, or withdraw a queued one (a running one: HZ_EINVAL). */
int hz_server_release(hz_server s, int64_t id);

/* Requests waiting for admission and requests running. */
int hz_server_pending(hz_server s, int32_t* queued, int32_t* running);

/* Spread the iterate groups of a tick (the loads of one grid shape and kernel
 * precision; one launch per pass each) over n_streams streams: the server's own and
 * n_streams - 1 non-blocking streams of default priority that the library creates
 * and destroys with the server.  Each tick forks them from the server's stream with
 * an event, gives each group to the stream with the least estimated work so far,
 * issues one iteration of every group in turn, and joins them back into the server's
 * stream before it reads the stop flags, so groups of different shapes run on the
 * device at the same time.  n_streams = 1 (the default) runs the groups one after
 * another on the server's stream.  Groups hold disjoint loads: results do not depend
 * on n_streams.  1 <= n_streams <= 8, else HZ_EINVAL. */
int hz_server_set_streams(hz_server s, int32_t n_streams);

/* Wait for the stream and free the server's host state (the workspace stays the caller's). */
void hz_server_destroy(hz_server s);

#ifdef __cplusplus
}
#endif

#endif /* HZ_H */
