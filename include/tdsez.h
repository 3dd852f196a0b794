/*
 * tdsez.h -- C ABI of the MI355X (gfx950) Crank-Nicolson propagation library
 * for the single-active-electron time-dependent Schroedinger equation on
 * B-spline Galerkin matrices, after Dahbi & Zair, "Unified Strong-Field
 * Dynamics Simulations from Atoms to Heterostructures" (arXiv 2608.18472).
 *
 * Problem statement (the paper's section II and section V):
 *   i M dc/dt = H(t) c                                 (section II.C, eq. matrixODE)
 *   H(t) = T_BDD + V + E(t) D,  T_BDD = 1/2 <grad B_J, m^-1 grad B_I>
 *                                                      (section II.A-II.C, eq. laser)
 *   (M + i dt/2 H^{n+1/2}) c^{n+1} = (M - i dt/2 H^{n+1/2}) c^n,
 *   H^{n+1/2} = (H^n + H^{n+1})/2                      (section V.B, eq. cn_system)
 * with the per-step observables of section IV.A: the M-norm, the dipole
 * d = c^H D c and the Ehrenfest acceleration a = -<m^-1 (dV/dx + E)> + a_Q
 * (eq. pdm_acceleration), an optional complex absorbing potential
 * (section V.A) and the extended time series of section V.D (energies,
 * velocity, autocorrelation, populations).  The mass matrix is called S
 * here (the paper's M).
 *
 * Conventions for every entry point
 *   - Return value: TDSEZ_OK (0) or an error code; tdsez_last_error() gives a
 *     thread-local message for the last non-OK status of the calling thread.
 *     No C++ exception ever crosses this boundary.
 *   - Host inputs are copied before the call returns; the caller keeps
 *     ownership.  Device pointers (marked "device") are caller-owned memory
 *     on the current HIP device; the library never frees them.  Handles own
 *     their device storage and release it in the matching destroy call.
 *   - Work on device pointers is enqueued on the HIP stream `stream` (NULL =
 *     the null stream) and is asynchronous unless stated otherwise.  Errors
 *     that can only be seen on the device (a non-finite state, norm drift)
 *     are latched in the handle and returned by tdsez_batch_status().
 *   - Units: Hartree atomic units.  Complex vectors are interleaved
 *     (re, im) doubles (complex128).
 *   - Unknowns: B-splines of order k = p + 1 on the open knot vector built
 *     from strictly increasing breakpoints (end breakpoints repeated k times);
 *     the first and last B-spline are dropped (homogeneous Dirichlet,
 *     section II.C), so N = (nbreaks - 1) + p - 2.
 *   - Band convention for host copies: a real symmetric banded matrix M is
 *     its upper half band, diagonal-major: band[d*N + i] = M[i][i+d] for
 *     d = 0..p, i = 0..N-1-d (entries with i+d >= N are zero).
 */
#ifndef TDSEZ_H
#define TDSEZ_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tdsez_status {
    TDSEZ_OK = 0,
    TDSEZ_EINVAL = 1,       /* invalid argument (sizes, knots, order, pointers) */
    TDSEZ_ENOMEM = 2,       /* device or host allocation failed */
    TDSEZ_EHIP = 3,         /* a HIP runtime call failed (message has the HIP error) */
    TDSEZ_ENOCONV = 4,      /* an iterative procedure did not converge */
    TDSEZ_ENONFINITE = 5,   /* a NaN/Inf appeared in a state (latched on device) */
    TDSEZ_ENORMDRIFT = 6,   /* |nu_n / nu_0 - 1| exceeded the batch tolerance */
    TDSEZ_EUNSUPPORTED = 7  /* valid but unsupported request (e.g. order > 8) */
} tdsez_status;

/* Arithmetic of the propagation.
 *   TDSEZ_FP64: bands, factorisations, solves, state and reductions in FP64.
 *   TDSEZ_FP32_REFINED: bands stored and the banded factorisation/solve done
 *     in FP32.  Each step solves for the increment from the previous state
 *     (right-hand side (B_n - A_n) c_n = -i dt H^{n+1/2} c_n formed in FP64,
 *     state accumulated in FP64), then runs `refine` iterative-refinement
 *     sweeps (default 1, see tdsez_batch_set): the residual
 *     B_n c_n - A_n c of the current iterate is formed in FP64 arithmetic
 *     and solved with the same FP32 factorisation.  The residual reads S, H0
 *     and D as their FP32 roundings hi with one signed 8-bit code q per
 *     entry, entry = hi (1 + q 2^-31), q the nearest integer to
 *     (v - hi) / (hi 2^-31) clamped to [-127, 127] for the FP64 entry v
 *     (within 2^-32 |hi| of v; 5 bytes per entry read instead of 8), so
 *     the sweeps converge to the Crank-Nicolson step of those bands; the
 *     absorber W is read in FP64.  Without a sweep the FP32
 *     rounding of the factorisation acts like a perturbed mass matrix and
 *     the phase error grows linearly in time.  State, observables and time
 *     series stay FP64. */
typedef enum tdsez_precision { TDSEZ_FP64 = 0, TDSEZ_FP32_REFINED = 1 } tdsez_precision;

/* Observable selection bits.  The output series always has 3 columns per
 * step, obs[n*3 + 0..2] = (nu_n, d_n, a_n) for n = 0..nsteps; unselected
 * columns are written as 0.
 *   nu_n = c_n^H S c_n                         (M-norm, section V.B)
 *   d_n  = Re c_n^H D c_n                      (dipole, section IV.A)
 *   a_n  = -Re c_n^H G c_n - E_n Re c_n^H Mi c_n + c_n^H Q c_n,
 *          G = <B| m^-1 dV/dx |B>, Mi = <B| m^-1 |B>, Q the a_Q form of
 *          tdsez_set_aq                      (eq. pdm_acceleration)
 * None of them is divided by nu_n.  For a system with a position-dependent
 * mass, TDSEZ_OBS_ACCEL needs the a_Q form (tdsez_set_aq); without it the
 * propagation calls return TDSEZ_EUNSUPPORTED. */
enum { TDSEZ_OBS_NORM = 1, TDSEZ_OBS_DIPOLE = 2, TDSEZ_OBS_ACCEL = 4 };

/* Extended per-step series (the time series the paper's section V.D writes
 * every step), selected by TDSEZ_EXT_SERIES in the *_ext propagation calls:
 * ext[n*ncols + k], ncols = 10 + npop (tdsez_ext_columns), n = 0..nsteps:
 *   k = 0  E_kin = c^H T c              1  E_pot = c^H V c
 *       2  E_int = E_n d_n              3  E_tot = E_kin + E_pot + E_int
 *       4  <m^-1> = c^H Mi c            5  <v> = c^H Vel c (eq. vel_elem)
 *       6  a_Q = c^H Q c (0 without tdsez_set_aq)
 *       7  <W> = c^H W c (0 without an absorber; d nu/dt = -2 <W>)
 *       8, 9  Re, Im of the autocorrelation c_0^H S c_n (M-weighted overlap
 *             with the call's initial state)
 *       10 + j  population |(S phi_j)^T c_n|^2 of projection state j
 *               (tdsez_set_projectors)
 * Expectation values are not divided by the norm.  Computed in FP64 from
 * the FP64 bands in both precisions. */
enum { TDSEZ_EXT_SERIES = 1 };

/* Band selectors for tdsez_get_band.  TDSEZ_BAND_K is the real
 * antisymmetric K with Vel = -(i/2) K (eq. vel_elem), returned as its upper
 * half band K[i][i+d]; W and Q exist after tdsez_set_cap / tdsez_set_aq. */
enum { TDSEZ_BAND_S = 0, TDSEZ_BAND_T = 1, TDSEZ_BAND_V = 2, TDSEZ_BAND_D = 3,
       TDSEZ_BAND_G = 4, TDSEZ_BAND_MI = 5, TDSEZ_BAND_H0 = 6, TDSEZ_BAND_K = 7,
       TDSEZ_BAND_W = 8, TDSEZ_BAND_Q = 9 };

typedef struct tdsez_system_s* tdsez_system; /* one assembled 1D problem */
typedef struct tdsez_batch_s* tdsez_batch;   /* propagation plan for several systems */

/* Message for the last non-OK status returned to this thread ("" if none). */
const char* tdsez_last_error(void);

/* Library ABI version (major*100 + minor). */
int tdsez_version(void);

/* Gauss-Legendre nodes and weights on [-1, 1] (nq in 1..32), ascending.
 * The inner products of section II.C are Gauss quadratures per knot span. */
tdsez_status tdsez_gauss_legendre(int nq, double* x_out, double* w_out);

/* Physical quadrature points at which the caller must sample m^-1(x), V(x)
 * and V'(x) for tdsez_assemble: x_out[e*nq + q] is the q-th Gauss point of
 * span [breaks[e], breaks[e+1]], e = 0..nbreaks-2 (host arrays).
 * EINVAL if nbreaks < 2, nq outside 1..32 or breaks not strictly increasing. */
tdsez_status tdsez_quad_points(const double* breaks, int nbreaks, int nq, double* x_out);

/* Galerkin assembly on the GPU (section V.A element formulas for the overlap
 * matrix, the BenDaniel-Duke kinetic matrix, the potential and dipole
 * matrices; G and Mi for the acceleration).  Inputs are host arrays:
 * breakpoints (nbreaks, strictly increasing), order k = p + 1 in 2..8,
 * nq Gauss points per span, and the caller's samples of m^-1, V, V' at the
 * points of tdsez_quad_points (each (nbreaks-1)*nq doubles; dV_q may be NULL
 * when the acceleration is not needed, minv_q may be NULL for m = 1).
 * Creates a system handle that owns FP64 device bands of S, T, V, D, G, Mi.
 * Runs on the null stream and returns when assembly is complete.
 * EINVAL on bad sizes/knots/order, EUNSUPPORTED for order > 8, EHIP/ENOMEM
 * on device failures. */
tdsez_status tdsez_assemble(const double* breaks, int nbreaks, int order, int nq,
                            const double* minv_q, const double* V_q, const double* dV_q,
                            tdsez_system* out);

/* Complex absorbing potential (section V.A, CAP element formula: the CAP
 * matrix is -i W with W_ab = sum_q w_q eta(x_q) N_a N_b).  eta_q: host
 * samples of the mask eta >= 0 at the points of tdsez_quad_points of the
 * system's breakpoints and nq (copied); NULL removes the absorber.  With an
 * absorber H^{n+1/2} = H0 + Ebar_n D - i W in eq. cn_system, so
 * A_n = S + (dt/2) W + i (dt/2)(H0 + Ebar_n D) stays complex symmetric with a
 * positive definite real part and the same factorisation applies.  Affects
 * batches created afterwards (and the one-system plan of tdsez_propagate).
 * The adjoint refuses systems with an absorber (EUNSUPPORTED).  Synchronous.
 * EINVAL for a negative or non-finite sample. */
tdsez_status tdsez_set_cap(tdsez_system sys, const double* eta_q);

/* The a_Q term of the acceleration (eq. pdm_acceleration, eq.
 * aQ_definition) as a quadratic form.  For a smooth inverse mass mu = m^-1
 * in one dimension, (i/4) <[p mu p, p mu + mu p]> equals
 *   a_Q = 1/2 <psi'| g |psi'> - 1/4 <psi| h |psi>,
 *   g = mu mu_1,  h = mu_1 mu_2 + mu mu_3   (mu_k: k-th derivative of mu),
 * assembled as Q_ab = sum_q w_q (g N'_a N'_b / 2 - h N_a N_b / 4).  g_q, h_q:
 * host samples at the quadrature points (either may be NULL for zero; both
 * NULL removes the form).  Interface terms of a discontinuous mass are not
 * part of this form (g = h = 0 inside layers of constant mass).  Affects
 * batches created afterwards.  Synchronous. */
tdsez_status tdsez_set_aq(tdsez_system sys, const double* g_q, const double* h_q);

/* Projection states of the population series (section V.D
 * "populations"): npop (0..8) real host vectors phi_j, phi + j*N, normally
 * S-normalised eigenstates (tdsez_ground_state); the library stores S phi_j.
 * npop = 0 removes them.  Affects batches created afterwards.  Synchronous. */
tdsez_status tdsez_set_projectors(tdsez_system sys, int npop, const double* phi);

/* Columns of the system's extended series: 10 + npop. */
tdsez_status tdsez_ext_columns(tdsez_system sys, int* ncols);

/* N (unknowns after Dirichlet removal) and half-bandwidth p: the size of the
 * Galerkin system of section II.C (eq. matrixODE) after the homogeneous
 * Dirichlet conditions, and the band half-width p of every matrix of
 * section V.A (B-splines of degree p overlap p neighbours). */
tdsez_status tdsez_system_size(tdsez_system sys, int* ndof, int* halfbw);

/* Copy one assembled band to host memory, (p+1)*N doubles in the header's
 * band convention; `which` is a TDSEZ_BAND_* selector (the element
 * matrices of section V.A, the velocity K of eq. vel_elem, the absorber W
 * of the CAP element formula, the a_Q form of eq. aQ_definition).
 * Synchronous. */
tdsez_status tdsez_get_band(tdsez_system sys, int which, double* host_out);

/* Lowest `nev` eigenpairs of the generalised problem H0 c = e S c
 * (section II.C eq. gen_ev), computed on the GPU in FP64 by shift-and-invert
 * subspace iteration with Rayleigh-Ritz (section V.C uses shift-and-invert).
 * sigma must lie below the lowest wanted eigenvalue (H0 - sigma S positive
 * definite); passing sigma >= 1e300 picks min_q V(x_q) - 1e-3 (|min V| + 1),
 * which is a valid lower bound for the assembled pencil.  tol: relative
 * residual |H0 v - e S v| / (|H0 v| + |e| |S v|) of every wanted pair.
 * Outputs (host): eps_out[nev] ascending; c_out[nev*N], vector j at
 * c_out + j*N, real, S-normalised, largest-magnitude component positive
 * (the real, phase-realigned form of section IV.C).
 * ENOCONV if maxit iterations do not reach tol.  Synchronous. */
tdsez_status tdsez_ground_state(tdsez_system sys, int nev, double sigma, double tol, int maxit,
                                double* eps_out, double* c_out);

/* Ground states of every system of a batch in one launch (one workgroup per
 * system, FP64): the lowest eigenpair of H0 c = e S c (section II.C eq.
 * gen_ev) by shift-and-invert power iteration with K = H0 - sigma S
 * factorised once per system.  sigma as in tdsez_ground_state (>= 1e300
 * picks each system's own min_q V(x_q) - 1e-3 (|min V| + 1)).  Writes
 * eps_out[s] (host) and the real, S-normalised ground state of system s
 * (largest-magnitude component positive, imaginary parts 0) into the
 * device complex128 buffer psi_packed at element psi_off[s] (host offsets).
 * EINVAL if K is not positive definite, ENOCONV if some system misses tol
 * (relative residual as in tdsez_ground_state) after maxit iterations.
 * Synchronous. */
tdsez_status tdsez_ground_state_batched(tdsez_batch b, double sigma, double tol, int maxit,
                                        double* eps_out, double* psi_packed, const long* psi_off);

/* Create a propagation plan for nsys systems (copied handles are borrowed:
 * the systems must outlive the batch): the batched form of the
 * Crank-Nicolson step of section V.B (eq. cn_system), one independent
 * system per workgroup.  Packs every system's bands into the propagation
 * layout in FP64 and FP32 and sizes the device workspaces.  Synchronous. */
tdsez_status tdsez_batch_create(const tdsez_system* sys, int nsys, tdsez_batch* out);

/* Tuning knobs of a batch.  key: "refine" (FP64-residual refinement sweeps
 * per step of TDSEZ_FP32_REFINED calls, integer 0..4, default 1; TDSEZ_FP64
 * calls run none; the residual's bands are described at
 * TDSEZ_FP32_REFINED), "refine_tol" (latch ENOCONV when the relative FP64
 * residual ||r|| / sqrt(||S dx||^2 + ||a (W + i H) v||^2) entering the last
 * refinement sweep of a step exceeds the value, r = B_n c_n - A_n c,
 * dx = c - c_n, v = c + c_n, a = dt/2; default 1e-2; the propagation goes on,
 * the first such step is reported by tdsez_batch_status), "norm_tol" (latch ENORMDRIFT
 * when |nu_n/nu_0 - 1| > value; 0 disables, default 0), "chunks" (force the
 * partition count of every system, 0 = plan, default 0; capped at 64 for a
 * one-wave system, at 128 or 256 for a system marked by tdsez_batch_split,
 * by max_waves), "max_waves" (2 or 4, default 2: the most waves a system
 * marked by tdsez_batch_split may run on; re-packs the batch and clears the
 * autotuner's plans), "profile" (1 turns on per-phase cycle counters read by
 * tdsez_batch_profile, 0 off). */
tdsez_status tdsez_batch_set(tdsez_batch b, const char* key, double value);

/* Partition autotuner (fills the batch's plan cache).  The partitioned solve
 * of section V.B's Crank-Nicolson system splits each system into P chunks;
 * the best P balances the per-chunk sweeps against the serial chain over the
 * P separator blocks and depends on N, p, the precision and the rest of the
 * batch.  Runs short profiled propagations of the whole batch (scratch
 * inputs; the caller's buffers are not touched) for up to five chunk-length
 * rules, the default rule first, until budget_ms of wall time is spent, and
 * keeps for every system the chunk count with the fewest cycles per step.
 * Later calls of either precision use the tuned plan; tdsez_batch_set
 * "chunks" overrides and clears it.  Synchronous (default stream).  EINVAL
 * for budget_ms <= 0 or an unknown precision. */
tdsez_status tdsez_autotune(tdsez_batch b, tdsez_precision prec, double budget_ms);

/* Chunk count P of every system under the batch's current plan (host array
 * of nsys ints). */
tdsez_status tdsez_batch_chunks(tdsez_batch b, int* chunks_out);

/* Two waves for the costliest systems.  A batch launch ends when its
 * longest system ends; in the partitioned solve of section V.B's
 * Crank-Nicolson system the per-step time of one system is bounded below by
 * the serial chain over its P separator blocks and the lane-serial sweep of
 * its N/P-row chunks, with P at most 64 (one chunk per lane of one wave).
 * This call marks the `count` systems with the largest cost N (p + 1)
 * nsteps[s] to run on a workgroup of two waves: up to 128 chunks, chunk
 * length rule L = sqrt(0.3 N), and the separator system eliminated from both
 * ends at once (each wave half of the chain, joined at the middle block).
 * A marked system whose two-wave plan has at most 64 chunks stays on one
 * wave with its one-wave plan.  With the batch key max_waves = 4 a marked
 * system whose four-wave rule L = sqrt(0.15 N) gives more than 128 chunks
 * runs on four waves instead (up to 256 chunks), and its separator system
 * is solved by block cyclic reduction: log2(P) levels, each level's block
 * eliminations shared by the four waves.
 * Multi-wave systems run in launches of their own (four-wave first, on the
 * caller's stream), concurrently with the one-wave launch on internal side
 * streams forked from and joined back into it (all at the default
 * priority), so the `stream` semantics of the propagation calls are
 * unchanged and the calls stay capturable into a graph.  Results equal the
 * one-wave results up to rounding.  count = 0 restores one wave per system.
 * Re-packs the batch and clears the autotuner's plans (run tdsez_autotune
 * afterwards to tune the new plan; it keeps the marks).  The adjoint runs
 * every system on the waves of its plan.  count = TDSEZ_SPLIT_AUTO chooses the count from the
 * current device: with S = 4 x its compute units (SIMDs) the batch's waves
 * are to fill them with a margin of 16 %, count = clamp(floor(1.16 S) -
 * nsys, 0, nsys) (a measured optimum: on a 1024-SIMD device the 1024-system
 * batch runs fastest with 100 to 220 marked systems, 160 in the middle).
 * nsteps: host array of nsys step counts (may be NULL when count = 0).
 * Synchronous.  EINVAL for count outside 0..nsys (other than
 * TDSEZ_SPLIT_AUTO) or a negative step count. */
enum { TDSEZ_SPLIT_AUTO = -1 };
tdsez_status tdsez_batch_split(tdsez_batch b, const int* nsteps, int count);

/* 1 for every system that runs on more than one wave under the current
 * plan, else 0 (host array of nsys ints). */
tdsez_status tdsez_batch_two_wave(tdsez_batch b, int* flags_out);

/* Waves (1, 2 or 4) of every system under the current plan (host array of
 * nsys ints); see tdsez_batch_split. */
tdsez_status tdsez_batch_waves(tdsez_batch b, int* waves_out);

/* Crank-Nicolson propagation of every system of the batch in one persistent
 * kernel launch (one workgroup per system; multi-wave systems in concurrent
 * launches of their own, see tdsez_batch_split), section V.B eq. cn_system with
 * H^{n+1/2} = H0 + (E_n + E_{n+1})/2 D.
 *   psi_packed (device, in/out): complex128 states; system s starts at
 *       element psi_off[s] (host array of nsys offsets, in complex elements)
 *       and has N_s elements; on return it holds c_{nsteps_s}.
 *   E_packed (device): FP64 samples E_0..E_{nsteps_s} of system s at
 *       E_packed + E_off[s] (host offsets, in doubles).
 *   dt, nsteps (host arrays, nsys each): time step (> 0) and step count (>= 0).
 *   obs_packed (device, out): FP64 series, system s at obs_packed + obs_off[s]
 *       (host offsets, in doubles), (nsteps_s + 1) x 3 as described at
 *       TDSEZ_OBS_*; may be NULL when obs == 0.
 * Workgroups start in order of decreasing cost N (p + 1) nsteps, so a batch
 * with more systems than the device holds at once runs longest first.
 * Asynchronous on `stream`.  Calls on one batch must not overlap (they share
 * the batch's working state, and its side streams and events when it holds
 * multi-wave systems); different batches may run concurrently.  EINVAL on bad
 * arguments (detected on the host); device-side failures are latched
 * (tdsez_batch_status). */
tdsez_status tdsez_propagate_batched(tdsez_batch b, double* psi_packed, const long* psi_off,
                                     const double* E_packed, const long* E_off,
                                     const double* dt, const int* nsteps, tdsez_precision prec,
                                     unsigned obs, double* obs_packed, const long* obs_off,
                                     void* stream);

/* tdsez_propagate_batched with the extended per-step series: ext =
 * TDSEZ_EXT_SERIES (or 0 for none); ext_packed (device, out): FP64, system s
 * at ext_packed + ext_off[s] (host offsets, in doubles), (nsteps_s + 1) x
 * (10 + npop_s) as described at TDSEZ_EXT_SERIES.  Asynchronous on `stream`;
 * EINVAL for unknown bits or a NULL buffer with ext != 0. */
tdsez_status tdsez_propagate_batched_ext(tdsez_batch b, double* psi_packed, const long* psi_off,
                                         const double* E_packed, const long* E_off, const double* dt,
                                         const int* nsteps, tdsez_precision prec, unsigned obs,
                                         double* obs_packed, const long* obs_off, unsigned ext,
                                         double* ext_packed, const long* ext_off, void* stream);

/* Single-system convenience form of tdsez_propagate_batched (the library
 * keeps a one-system plan inside the system handle, created by the first
 * call).  The system runs on four waves when its four-wave plan has more
 * than 128 chunks (N above about 2460), else on two when its two-wave plan
 * has more than 64 (N above about 1230; see tdsez_batch_split) or when 65
 * chunks of at least 2p rows fit (N above about 65 (2p - 1): a lone system is
 * latency-bound, so it takes the shorter chunks), else on one.  psi: device
 * complex128 [N] in/out; E: device FP64 [nsteps+1]; obs_out: device FP64
 * [(nsteps+1)*3] or NULL.  Asynchronous on `stream`. */
tdsez_status tdsez_propagate(tdsez_system sys, double* psi, const double* E, double dt, int nsteps,
                             tdsez_precision prec, unsigned obs, double* obs_out, void* stream);

/* tdsez_propagate for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It allocates nothing, on its first call included: the
 * working storage of the partitioned solve (packed bands, state, factor
 * rows, separator system, descriptor) lives in one file-scope device array
 * of 64 MiB per GPU, held until the process ends, and is filled from the
 * system's bands on every call; the kernels and the plan are those of
 * tdsez_propagate on one workgroup (up to four waves), so the results are
 * the same wherever tdsez_propagate keeps one workgroup (where it spreads a
 * long chain over several, see tdsez_system_set, they agree to rounding).  A system that needs more
 * than 64 MiB (N above about 50 000 at order 8) is refused with EINVAL.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams, threads or processes' graphs replayed
 * concurrently) race; calls ordered on one stream do not.  dev_status
 * (device int[4], caller-owned, may be NULL): cleared by the call, then
 * receives the first latched device error (code, -, step, -) as
 * tdsez_batch_status reports it.  No absorber, extended series or a_Q form
 * (EUNSUPPORTED).  Arguments as tdsez_propagate; asynchronous on `stream`. */
tdsez_status tdsez_propagate_noalloc(tdsez_system sys, double* psi, const double* E, double dt, int nsteps,
                                     tdsez_precision prec, unsigned obs, double* obs_out, int* dev_status,
                                     void* stream);

/* tdsez_propagate with the extended series (ext_out: device FP64
 * [(nsteps+1) * (10 + npop)], see TDSEZ_EXT_SERIES). */
tdsez_status tdsez_propagate_ext(tdsez_system sys, double* psi, const double* E, double dt, int nsteps,
                                 tdsez_precision prec, unsigned obs, double* obs_out, unsigned ext,
                                 double* ext_out, void* stream);

/* Gradient of a real function J of the observable series by the discrete
 * adjoint of the Crank-Nicolson recursion of section V.B (the paper gives no
 * adjoint; this is the exact gradient of the discrete recursion).  With
 * lambda_N = g_N and, for n = N-1..0,
 *   z_n = B_n^-1 lambda_{n+1},   lambda_n = g_n + A_n z_n,
 *   g_n = 2 J_nu,n S c_n + 2 J_d,n D c_n - 2 J_a,n (G c_n + E_n Mi c_n),
 * the outputs are
 *   dJdE[n] = (a Im(z_{n-1}^H D (c_{n-1} + c_n)) + a Im(z_n^H D (c_n + c_{n+1})))/2
 *             - J_a,n c_n^H Mi c_n        (a = dt/2; missing terms at n = 0, N)
 *   dJdpsi0 = lambda_0.
 * J_nu,n, J_d,n, J_a,n = dJdobs[n*3 + 0..2] (columns whose bit is not in
 * `obs` are ignored).  psi0_packed: device complex128 initial states at
 * psi_off (natural order); E_packed/E_off, dt, nsteps as for
 * tdsez_propagate_batched; dJdobs_packed: device FP64 at obs_off;
 * dJdE_packed: device FP64 [nsteps+1] per system at E_off (overwritten);
 * dJdpsi0_packed: device complex128 at psi_off, or NULL.  The forward
 * states are recomputed from psi0 with a checkpoint every ckpt_stride steps
 * (0: ceil(sqrt(nsteps))); the recomputation of a segment keeps each
 * step's factorisation of A_n, which the adjoint step of that step reuses
 * (it only substitutes).  The cost is about two and a half propagations,
 * the memory (nsteps/ckpt_stride + ckpt_stride + 1) states and ckpt_stride
 * factorisations (each 16 (2p + 2) bytes per row and 16 (6p^2 + 4p) bytes
 * per chunk) per system
 * (device workspace owned by the batch, grown on demand; a smaller
 * ckpt_stride trades factorisation memory for checkpoint states, and a
 * failed allocation returns TDSEZ_EHIP).  FP64 only
 * (TDSEZ_FP32_REFINED: EUNSUPPORTED).  One workgroup per system, of the
 * waves its plan has (tdsez_batch_split: two, or four with cyclic reduction
 * of the separator system; the launches of the three wave counts run
 * concurrently, as for propagation).  Asynchronous on `stream`;
 * device failures are latched as for propagation.  Uses the batch's working
 * state, so it must not overlap a propagation of the same batch. */
tdsez_status tdsez_adjoint_batched(tdsez_batch b, const double* psi0_packed, const long* psi_off,
                                   const double* E_packed, const long* E_off, const double* dt,
                                   const int* nsteps, tdsez_precision prec, unsigned obs,
                                   const double* dJdobs_packed, const long* obs_off, double* dJdE_packed,
                                   double* dJdpsi0_packed, int ckpt_stride, void* stream);

/* ------------------------------------------------------------------ 2D
 * Tensor-product problem on [x breakpoints] x [y breakpoints] with the same
 * order on both axes, constant mass, x-polarised field (section II.C eq.
 * tensor3d with two factors; section V.B for the step).  Unknown (iy, ix)
 * is N_ix(x) N_iy(y) of the reduced 1D bases, row-major index iy*Nx + ix.
 * S2 = Sx(x)Sy, T2 = Tx(x)Sy + Sx(x)Ty, D2 = Dx(x)Sy, and the potential
 * matrix V2[(iy,ix),(jy,jx)] = sum_q wx wy V N_ix N_jx N_iy N_jy by the
 * tensor Gauss rule. */
typedef struct tdsez_system2d_s* tdsez_system2d;

/* Assemble a 2D problem on the device.  V_q: host FP64 samples of V at the
 * tensor grid of the per-axis quadrature points (tdsez_quad_points of each
 * axis), V_q[qy * nqx + qx], nqx = (nbx-1)*nq, nqy = (nby-1)*nq (copied).
 * dVx_q: samples of dV/dx at the same points, or NULL; with them the force
 * stencil G2[(iy,ix),(jy,jx)] = sum_q wx wy dV/dx N_ix N_jx N_iy N_jy is
 * assembled too, for the acceleration of section IV.A (eq.
 * pdm_acceleration with m = 1): a = -Re c^H G2 c - E c^H S2 c.
 * Also computes, once, the per-axis generalised eigendecompositions
 * T Q = S Q Lambda used by the preconditioner.  Needs at least 2p+1
 * unknowns per axis; order <= 8.  Synchronous.  EINVAL for a non-finite
 * sample. */
tdsez_status tdsez_assemble_2d(const double* breaks_x, int nbx, const double* breaks_y, int nby, int order, int nq,
                               const double* V_q, const double* dVx_q, tdsez_system2d* out);
tdsez_status tdsez_system2d_size(tdsez_system2d s, int* nx, int* ny, int* halfbw);
/* Potential matrix as a (2p+1)^2 stencil per row (host FP64, caller-owned):
 * out[row*(2p+1)^2 + (dy+p)*(2p+1) + (dx+p)] = V2[row][(iy+dy)*Nx + ix+dx]. */
tdsez_status tdsez_get_v2(tdsez_system2d s, double* host_out);
/* Crank-Nicolson propagation of psi (device complex128 [Ny][Nx], in/out)
 * over nsteps steps of dt with E (device FP64 [nsteps+1]).  Each step solves
 * A_n (c_{n+1} - c_n) = -i dt H_n c_n to relative residual tol, starting
 * from the previous step's increment, with the preconditioner P = exact
 * inverse of S2 + i dt/2 T2 (per-axis eigenvectors, GEMMs on the matrix
 * cores):
 *   TDSEZ_FP64: COCG in FP64, at most maxit iterations per step;
 *   TDSEZ_FP32_REFINED: iterative refinement, each sweep forms the FP64
 *     residual r = b - A x, solves A e = r by COCG in FP32 (FP32 copies of
 *     the operator and of P, made by the first such call) to a relative
 *     1e-5, and adds e to x in FP64; at most maxit sweeps per step.
 * Either way the result meets the same FP64 residual bound; ENOCONV when
 * the bound is not met.  obs: TDSEZ_OBS_NORM | TDSEZ_OBS_DIPOLE (x dipole)
 * | TDSEZ_OBS_ACCEL (x acceleration, for a system assembled with dVx_q;
 * EUNSUPPORTED otherwise); obs_out[n*3 + 0..2] = (nu_n, d_n, a_n) on the
 * device (0 for an unrequested column), always FP64.
 * Enqueued on `stream`, but the host waits for the iteration scalars, so
 * the call returns when done. */
tdsez_status tdsez_propagate_2d(tdsez_system2d s, double* psi, const double* E, double dt, int nsteps,
                                tdsez_precision prec, unsigned obs, double* obs_out, double tol, int maxit,
                                void* stream);
/* Steps, Krylov iterations (FP32 inner iterations for TDSEZ_FP32_REFINED),
 * the largest iteration count of one step and the refinement sweeps of the
 * 2D propagations since the last call (any pointer may be NULL); resets the
 * counters. */
tdsez_status tdsez_system2d_stats(tdsez_system2d s, long* steps, long* iterations, int* max_iterations,
                                  long* sweeps);
/* As tdsez_time_apply_3d, for the 2D operator kernel. */
tdsez_status tdsez_time_apply_2d(tdsez_system2d s, tdsez_precision prec, int reps, void* stream, double* ms_out);
void tdsez_system2d_destroy(tdsez_system2d s);

/* ------------------------------------------------------------------ 3D
 * Tensor-product problem on [x] x [y] x [z] breakpoints, same order on every
 * axis, constant mass, x-polarised field: the three-factor basis of section
 * II.C eq. tensor3d with the step of section V.B, as in the strong-scaling
 * study of section VI (Table II: hydrogen, 97 cubic B-splines per axis,
 * hydrogenic knots on [-25, 25]^3, 100 steps of 0.01).  Unknown (iz, iy, ix)
 * has the row-major index (iz*Ny + iy)*Nx + ix.  S3 = Sz(x)Sy(x)Sx,
 * T3 = Sz Sy Tx + Sz Ty Sx + Tz Sy Sx, D3 = Sz Sy Dx, and
 * V3[i][j] = sum_q wx wy wz V N_i N_j by the tensor Gauss rule: a
 * (2p+1)^3-point stencil per row (343 for cubic splines), of which the
 * device keeps the symmetric half. */
typedef struct tdsez_system3d_s* tdsez_system3d;

/* Assemble a 3D problem on the device.  V_q: host FP64 samples of V at the
 * tensor grid of the per-axis quadrature points, V_q[(qz*nqy + qy)*nqx + qx],
 * nq* = (nb*-1)*nq (copied).  Also computes, once, the three per-axis
 * generalised eigendecompositions of the preconditioner.  order <= 5; at
 * least 2p+1 unknowns per axis.  Device memory: (w^3+1)/2 * N doubles for
 * V3 (w = 2p+1; 1.26 GB at 97^3, p = 3), twice that while assembling, plus
 * 18 N doubles of work vectors.  Synchronous. */
tdsez_status tdsez_assemble_3d(const double* breaks_x, int nbx, const double* breaks_y, int nby,
                               const double* breaks_z, int nbz, int order, int nq, const double* V_q,
                               tdsez_system3d* out);
tdsez_status tdsez_system3d_size(tdsez_system3d s, int* nx, int* ny, int* nz, int* halfbw);
/* Lowest generalised eigenpair of (T3 + V3, S3) by inverse iteration with
 * the fixed shift sigma (section II.C eq. gen_ev; the paper's eigensolve
 * phase of the strong-scaling runs): each outer step solves
 * (H - sigma S) y = S x by conjugate gradients preconditioned with the
 * exact inverse of T3 - sigma S3 (the six per-axis contractions), then
 * x = y / |y|_S and E = x^T H x, until |E - E_prev| <= tol |E| and
 * |H x - E S x| / |S x| <= sqrt(tol).  sigma must lie below the lowest level
 * (EINVAL when H - sigma S is found not positive definite).  psi: device
 * complex128 [N] (out: the S-normalised real eigenvector, sign not fixed);
 * energy: host double (out).  ENOCONV after maxit outer steps.  Uses the
 * system's work vectors; synchronous. */
tdsez_status tdsez_ground_state_3d(tdsez_system3d s, double sigma, double tol, int maxit, double* psi,
                                   double* energy);
/* Rows of V3 as (2p+1)^3 stencils (host FP64, caller-owned, nrows*(2p+1)^3):
 * out[r*w^3 + ((dz+p)*w + (dy+p))*w + (dx+p)] = V3[rows[r]][neighbour], 0 for
 * a neighbour outside the grid.  EINVAL for a row outside 0..N-1. */
tdsez_status tdsez_get_v3_rows(tdsez_system3d s, const long* rows, int nrows, double* host_out);
/* out = a S3 c + b (T3 + V3 + Ebar D3) c for device complex128 c and out
 * (N entries each, distinct); a = are + i aim, b = bre + i bim.  Shares the
 * system's work vectors with tdsez_propagate_3d (do not overlap the two).
 * Asynchronous on `stream`. */
tdsez_status tdsez_apply_3d(tdsez_system3d s, const double* c, double* out, double are, double aim, double bre,
                            double bim, double Ebar, void* stream);
/* Crank-Nicolson propagation of psi (device complex128 [Nz][Ny][Nx], in/out);
 * arguments, precisions, observables, convergence control and ENOCONV as
 * for tdsez_propagate_2d, with the preconditioner the exact inverse of
 * S3 + i dt/2 T3 (six per-axis contractions on the matrix cores). */
tdsez_status tdsez_propagate_3d(tdsez_system3d s, double* psi, const double* E, double dt, int nsteps,
                                tdsez_precision prec, unsigned obs, double* obs_out, double tol, int maxit,
                                void* stream);
/* Average duration (ms, HIP events on `stream`) of `reps` back-to-back
 * launches of the operator kernel q = A p exactly as a Krylov iteration of
 * tdsez_propagate_3d launches it (FP64 or, for TDSEZ_FP32_REFINED, the FP32
 * operator); for roofline accounting.  Uses the work vectors; synchronises
 * `stream`. */
tdsez_status tdsez_time_apply_3d(tdsez_system3d s, tdsez_precision prec, int reps, void* stream, double* ms_out);
/* As tdsez_system2d_stats, for the 3D propagations since the last call. */
tdsez_status tdsez_system3d_stats(tdsez_system3d s, long* steps, long* iterations, int* max_iterations,
                                  long* sweeps);
void tdsez_system3d_destroy(tdsez_system3d s);

/* Phase profile of the last propagation of a profiled batch (see
 * tdsez_batch_set "profile").  Synchronises `stream`; out[10*s + 0..9] =
 * average shader-clock cycles per time step spent by system s in: the
 * right-hand-side/observables pass, the elimination pass (TDSEZ_FP32_REFINED
 * runs both as one sweep, counted in the first column), the fill pass, the
 * separator (reduced) solve, the back substitution, and summed over the
 * refinement sweeps their residual pass, separator solve and back
 * substitution; then the partition count; out[10*s + 9] is the largest
 * relative refinement residual of the run (see "refine_tol"; 0 for FP64
 * calls).  Profiling adds a barrier per
 * phase.  EINVAL when profiling is off. */
tdsez_status tdsez_batch_profile(tdsez_batch b, void* stream, double* out);

/* Synchronise `stream`, then return and clear the first device-side failure
 * latched by the batch (TDSEZ_OK if none); sys_out/step_out (may be NULL)
 * receive the system index and step. */
tdsez_status tdsez_batch_status(tdsez_batch b, void* stream, int* sys_out, int* step_out);

/* Same for the one-system plan of tdsez_propagate. */
tdsez_status tdsez_system_status(tdsez_system sys, void* stream, int* step_out);

/* Partition of tdsez_propagate's one-system plan for a long chain (the
 * Crank-Nicolson system of section V.B, eq. cn_system, on one N-row band).
 * By default a system whose four-wave plan would hold chunks of more than 48
 * rows (N above about 12 000 at order 8) is spread over G workgroups of four
 * waves on different compute units, launched cooperatively (all resident
 * at once): workgroup g owns Pl consecutive chunks (chunks of about 2p + 1
 * rows), reduces its part of the separator system by block cyclic reduction
 * down to its last separator block, and after a grid barrier every
 * workgroup solves the G-block system of those blocks itself (from both
 * ends at once, as far as its own two blocks); a second
 * grid barrier follows each back substitution (the next pass reads the
 * neighbouring workgroups' rows).  Observable sums are formed per
 * workgroup and added in workgroup order after the launch; a non-finite
 * series is latched after the launch (the workgroups cannot leave early)
 * and the refinement residual check of "refine_tol" applies per
 * workgroup.  Spanning calls run the plain kernels only: the extended
 * series, an absorber or the a_Q form return EUNSUPPORTED (set
 * "workgroups" to 1).  Keys: "workgroups" (0: automatic, 1: one workgroup,
 * 2..64: that many), "chunks_per_workgroup" (0: automatic = 64, else
 * 2..256).  Drops the one-system plan (rebuilt by the next call).  EINVAL
 * for an unknown key or a value out of range. */
tdsez_status tdsez_system_set(tdsez_system sys, const char* key, double value);

/* Workgroups and chunk count of tdsez_propagate's one-system plan (built
 * here if needed); either pointer may be NULL. */
tdsez_status tdsez_system_workgroups(tdsez_system sys, int* workgroups, int* chunks);

void tdsez_batch_destroy(tdsez_batch b);
void tdsez_system_destroy(tdsez_system sys);

#ifdef __cplusplus
}
#endif

#endif /* TDSEZ_H */
