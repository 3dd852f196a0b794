// Internal declarations shared by the HIP translation units of libtdsez.
// Not part of the public ABI (see include/tdsez.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "tdsez.h"

namespace tdsez {

// Largest supported half-bandwidth (order 8 B-splines).
constexpr int kMaxP = 7;
// Lanes of one wave64 (a propagation workgroup holds one, two or four waves).
constexpr int kWave = 64;
// Largest partition count of one system (one chunk per lane).
constexpr int kMaxChunks = 64;
// Largest partition count of a system run on two waves (tdsez_batch_split).
constexpr int kMaxChunks2 = 2 * kWave;
// Largest partition count of a system run on four waves (max_waves = 4).
constexpr int kMaxChunks4 = 4 * kWave;
// Most workgroups one spanning system may use.
constexpr int kMaxSpan = 64;
// Chunk-length rules L = sqrt(c N) of one, two and four waves per system.
constexpr double kRule1 = 0.6, kRule2 = 0.3, kRule4 = 0.15;
// Matrices stored per band row in the propagation layout, in this order:
// S, H0, D, G, Mi (propagation and the three main observables), W (weight of
// the complex absorbing potential), V, K (velocity), Q (a_Q form) for the
// extended per-step series.
constexpr int kNumMats = 9;
// The refinement residual reads S, H0 and D as their FP32 roundings hi with
// a signed 8-bit code q each: entry = hi (1 + q kLoScale), within
// |hi| kLoScale / 2 of the FP64 value (|FP64 - hi| <= 2^-24 |hi|, so
// |q| <= 128, clamped to 127).
constexpr double kLoScale = 0x1p-31;
enum { kMatS = 0, kMatH0 = 1, kMatD = 2, kMatG = 3, kMatMi = 4, kMatW = 5, kMatV = 6, kMatK = 7, kMatQ = 8 };
// Largest number of projection states of the population series.
constexpr int kMaxPop = 8;
// Columns of the extended series before the populations.
constexpr int kExtFixed = 10;

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
tdsez_status fail(tdsez_status st, const char* fmt, ...);

#define TDSEZ_HIP_TRY(expr)                                                                 \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::tdsez::fail(TDSEZ_EHIP, "%s failed: %s (%s:%d)", #expr,                \
                                 hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

// ---------------------------------------------------------------- complex
template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cplx<T> cmk(T r, T i) { return cplx<T>{r, i}; }
template <typename T>
__host__ __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ inline cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a - b*c
template <typename T>
__host__ __device__ inline cplx<T> cfms(cplx<T> a, cplx<T> b, cplx<T> c) {
    return {a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re};
}
// a + b*c
template <typename T>
__host__ __device__ inline cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> c) {
    return {a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re};
}
template <typename T>
__host__ __device__ inline cplx<T> cinv(cplx<T> a) {
    T s = T(1) / (a.re * a.re + a.im * a.im);
    return {a.re * s, -a.im * s};
}
template <typename T>
__host__ __device__ inline cplx<T> cscale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }

// ---------------------------------------------------------------- handles
// Assembled 1D system.  Device bands are FP64, lower half band by rows:
// band[m][j*(p+1) + d] = M[j][j-d] (0 when j-d < 0).
struct SystemData {
    int N = 0, p = 0, order = 0, nq = 0, nbreaks = 0;
    bool const_mass = true;
    std::vector<double> breaks;
    double minV = 0.0;               // min_q V(x_q), for the default eigen shift
    double* d_band[6] = {nullptr};   // S, T, V, D, G, Mi
    double* d_H0 = nullptr;          // T + V
    double* d_K = nullptr;           // velocity: K[j][j-d] (real antisymmetric part of eq. vel_elem)
    double* d_W = nullptr;           // absorbing-potential weight (nullptr: no absorber)
    double* d_Q = nullptr;           // a_Q form (nullptr: not given)
    int npop = 0;                    // projection states of the population series
    double* d_pops = nullptr;        // S phi_k, npop x N, natural order
    tdsez_batch solo = nullptr;      // one-system plan for tdsez_propagate
    int span_G = 0;                  // tdsez_system_set "workgroups" (0: automatic, 1: one workgroup)
    int span_Pl = 0;                 // tdsez_system_set "chunks_per_workgroup" (0: automatic)
};

// Per-system plan of the partitioned solve.
struct Plan {
    int N, p, P, L, m;   // rows, half-bandwidth, chunks, rows per chunk, interior rows
    int LS;              // interleave stride (P + 2: chunk k lives in column k + 1)
};

// Device descriptor of one system of a batch (read by the propagation kernel).
struct SysDesc {
    int N, p, P, L, m, LS;
    int nsteps;
    int mi_is_s;          // constant mass: Mi equals S bit for bit (m^-1 = 1 at every point)
    double dt;
    long long band_off;   // elements into the FP64/FP32 packed band buffers
    long long state_off;  // complex elements into the interleaved state buffer
    long long fac_off;    // complex elements into the factor workspace
    long long red_off;    // complex elements into the reduced-system workspace
    long long psi_off;    // complex elements into the caller's psi buffer
    long long E_off;      // doubles into the caller's E buffer
    long long obs_off;    // doubles into the caller's obs buffer
    // adjoint only: checkpoint stride and number of segments
    int ck, nseg;
    int cap;              // 1: absorbing potential present (W band)
    int aq;               // 1: a_Q form present (Q band)
    int npop;             // projection states
    long long proj_off;   // doubles into the packed projection states
    long long ext_off;    // doubles into the caller's extended-series buffer
    int G, Pl;            // workgroups of a spanning system (else 1) and chunks per workgroup
};

struct BatchData {
    std::vector<SystemData*> sys;
    std::vector<Plan> plan;
    std::vector<SysDesc> desc;       // host copy, offsets of the internal buffers
    int maxp = 0;
    int refine = 1;                  // refinement sweeps of TDSEZ_FP32_REFINED calls
    double refine_tol = 1e-2;        // ENOCONV when the last sweep's relative residual exceeds it
    double norm_tol = 0.0;
    int force_chunks = 0;
    long long band_elems = 0, state_elems = 0, fac_elems64 = 0, red_elems64 = 0;
    double* d_band64 = nullptr;
    float* d_band32 = nullptr;
    // 8-bit corrections of the FP32 S, H0, D bands (refinement residual):
    // per system 3 * state_off words in, [row][S, H0, D][column], byte d =
    // diagonal d
    unsigned long long* d_bandlo = nullptr;
    double* d_state = nullptr;       // interleaved complex128 states
    double* d_dtot = nullptr;        // increment of the current step (refinement sweeps)
    void* d_rhs = nullptr;           // right-hand side of the current step (FP64 or FP32)
    // adjoint workspaces (allocated by the first adjoint call, grown on demand)
    double* d_lam = nullptr;         // adjoint variable, state layout
    double* d_wsol = nullptr;        // solution of the conjugated solve, state layout
    double* d_ckpt = nullptr;        // checkpoint states
    double* d_seg = nullptr;         // states of the segment being reversed
    long long ckpt_elems = 0, seg_elems = 0;
    // the segment's factorisations (fac and red layouts, one slot per step)
    double* d_fac_seg = nullptr;
    double* d_red_seg = nullptr;
    long long fac_seg_elems = 0, red_seg_elems = 0;
    void* d_fac = nullptr;           // factor workspace (sized for FP64)
    void* d_red = nullptr;           // reduced-system workspace (sized for FP64)
    SysDesc* d_desc = nullptr;
    std::vector<SysDesc> desc_on_device;  // last uploaded descriptors (skip identical uploads)
    int* d_order = nullptr;          // workgroup -> system, longest first
    std::vector<int> order_host;     // host copy of d_order (pageable; uploaded asynchronously)
    std::vector<int> tuned_chunks;   // plan cache of tdsez_autotune (0 = rule), per system
    std::vector<char> two_wave_req;  // per system: may run on more than one wave (tdsez_batch_split)
    int max_waves = 2;               // waves a marked system may use (2 or 4; key max_waves)
    std::vector<char> waves;         // per system: waves of its plan (1; 2: 65..128 chunks; 4: 129..256)
    int nsplit = 0;                  // systems on more than one wave (first nsplit entries of d_order)
    int n4 = 0;                      // of those, systems on four waves (the first n4 entries)
    bool solo = false;               // the one-system plan of tdsez_propagate (may span workgroups)
    int span_G = 0;                  // > 1: the single system spans this many workgroups
    void* d_xch = nullptr;           // spanning launch: exchange buffers, super-block factors, step parts
    void* d_gfac = nullptr;
    double* d_obs_part = nullptr;
    long long obs_part_elems = 0;
    hipStream_t side = nullptr, side2 = nullptr;  // further streams of a split launch (default priority)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
    int* d_status = nullptr;         // [0] code, [1] system, [2] step
    unsigned long long* d_prof = nullptr;  // optional phase cycle counters, kProfSlots per system
    double* d_proj = nullptr;        // packed projection states S phi_k (interleaved layout)
    double* d_c0 = nullptr;          // initial states of the call (state layout), for the autocorrelation
    bool any_cap = false, any_aq = false;
    int nsys_alloc_desc = 0;
};

// Arguments of the persistent propagation kernels.
struct KernelArgs {
    const SysDesc* descs;
    const int* order;          // workgroup -> system index (longest first)
    int order_off;             // first entry of order read by this launch
    const void* band;          // FT bands (factorisation, solve, right-hand side)
    const double* band64;      // FP64 bands (S of the refinement residual)
    double* st;
    double* dtot;              // increment of the current step (refinement only)
    void* rhs;                 // right-hand side of the step (FT, state layout)
    void* fac;
    void* red;
    const double* E;
    double* obs;
    unsigned mask;
    int refine;
    double norm_tol;
    int* status;
    unsigned long long* prof;
    double refine_tol;         // ENOCONV threshold of the last sweep's relative residual
    // extended kernels only
    const double* c0;          // initial states (state layout), or nullptr: no autocorrelation
    const double* proj;        // packed projection states S phi_k
    double* ext;               // extended series (caller's buffer), or nullptr
    // spanning launch only (one system on several workgroups)
    void* xch;                 // exchanged super-block data, two buffers (FT)
    void* gfac;                // per workgroup: factors of the super-block system (FT)
    double* obs_part;          // per step and workgroup: norm, dipole, acceleration parts
    // refinement residual: corrections of the FP32 S, H0, D bands
    const unsigned long long* bandlo;
};

// ---------------------------------------------------------------- kernels
// Persistent propagation launchers, one translation unit each
// (tdsez_prop_*.hip): the four-wave kernel over order entries 0..n4-1 on
// stream s4, the two-wave kernel over the next n2 entries on s2 and the
// one-wave kernel over the n1 after them on s1.  probe selects the
// autotuner's separately named copies (plain kernels only).
hipError_t launch_prop_f64(const KernelArgs& ka, int n4, int n2, int n1, hipStream_t s4, hipStream_t s2,
                           hipStream_t s1, bool probe);
hipError_t launch_prop_f32(const KernelArgs& ka, int n4, int n2, int n1, hipStream_t s4, hipStream_t s2,
                           hipStream_t s1, bool probe);
// One system on G cooperative workgroups of four waves (sd.G = G).
hipError_t launch_prop_f64_span(const KernelArgs& ka, int G, hipStream_t s);
hipError_t launch_prop_f32_span(const KernelArgs& ka, int G, hipStream_t s);
// Extended kernels: absorbing potential, extended series, a_Q.
hipError_t launch_prop_xt64(const KernelArgs& ka, int n4, int n2, int n1, hipStream_t s4, hipStream_t s2,
                            hipStream_t s1);
hipError_t launch_prop_xt32(const KernelArgs& ka, int n4, int n2, int n1, hipStream_t s4, hipStream_t s2,
                            hipStream_t s1);
// Assembly (tdsez_assemble.hip)
tdsez_status assemble_device(const double* breaks, int nbreaks, int order, int nq,
                             const double* minv_q, const double* V_q, const double* dV_q,
                             SystemData* sys);
// W (which = 0, samples eta) or Q (which = 1, samples g and h) of an
// assembled system; replaces the previous band of that kind.
tdsez_status assemble_extra_device(SystemData* sys, int which, const double* a_q, const double* b_q);
// S phi_k of npop host vectors into sys->d_pops (replaces previous ones).
tdsez_status set_projectors_device(SystemData* sys, int npop, const double* phi);
// Host Gauss-Legendre (tdsez_assemble.hip)
int gauss_legendre_host(int nq, double* x, double* w);

// Propagation (tdsez_propagate.hip)
// rule c: chunk length L = sqrt(c N); max_chunks: kMaxChunks, kMaxChunks2 or kMaxChunks4
Plan make_plan(int N, int p, int force_chunks, int max_chunks = kMaxChunks, double rule = kRule1);
// Plan of a system that may use up to max_waves (1, 2 or 4) waves: the
// rule of the most waves whose plan needs more chunks than the next fewer
// waves hold.  force_chunks > 0 overrides the rule (capped by max_waves).
Plan multi_wave_plan(int N, int p, int force_chunks, int max_waves);
// Plan of one system spread over G workgroups of Pl chunks each (G Pl
// chunks in all); G = 0 or Pl = 0 pick them from N and p.  Returns G (1
// when the system does not need more than one workgroup).
int span_plan(int N, int p, int G, int Pl, Plan* out);
// Waves that a plan runs on.
inline int plan_waves(const Plan& pl) { return pl.P > kMaxChunks2 ? 4 : pl.P > kMaxChunks ? 2 : 1; }
tdsez_status pack_bands(BatchData* b);
// probe: launch the autotuner's separately named copy of the kernel
tdsez_status launch_propagate(BatchData* b, double* psi, const double* E, double* obs,
                              tdsez_precision prec, unsigned obs_mask, hipStream_t stream, bool probe = false,
                              double* ext = nullptr);
// Counters per system of the optional phase profile: 8 phases, the step
// count and the largest relative refinement residual (double bits).
constexpr int kProfSlots = 10;
// Adjoint (tdsez_adjoint.hip): descriptors already hold nsteps, dt and offsets
// Upload the batch descriptors, and the longest-first workgroup order derived
// from them, if they differ from the last upload (a repeated call with the
// same arguments then enqueues kernels only, so it can be captured into a
// graph after a warm-up call).
tdsez_status upload_descriptors(BatchData* b, hipStream_t stream);
tdsez_status launch_adjoint(BatchData* b, const double* psi0, const double* E, const double* dJdobs,
                            unsigned obs_mask, double* dJdE, double* dJdpsi0, int ckpt_stride,
                            hipStream_t stream);

// Eigen (tdsez_eigen.hip)
tdsez_status ground_state_device(SystemData* sys, int nev, double sigma, double tol, int maxit,
                                 double* eps_out, double* c_out);
tdsez_status ground_state_batched_device(BatchData* b, double sigma, double tol, int maxit, double* eps_out,
                                         double* psi, const long* psi_off);

}  // namespace tdsez

// The opaque handles of the ABI.
struct tdsez_system_s {
    tdsez::SystemData d;
};
struct tdsez_batch_s {
    tdsez::BatchData d;
};
