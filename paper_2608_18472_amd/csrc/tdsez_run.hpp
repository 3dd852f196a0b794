// Per-system driver of the persistent Crank-Nicolson kernels (the paper's
// section V.B, eq. cn_system) and the kernel templates; instantiated by the
// translation units tdsez_prop_*.hip, one precision and kernel family each,
// so that they compile in parallel.  The algorithm and the layouts are
// described at the top of tdsez_propagate.hip.
#pragma once

#include "tdsez_passes.hpp"

namespace tdsez {
namespace {

// Combine wave-uniform partial sums of the waves of a workgroup through
// LDS.  Every wave adds the parts in wave order, so all waves take the same
// decisions afterwards.  A no-op for one wave.
template <int NW, int CAP>
__device__ __forceinline__ void combine_waves(double (&v)[CAP], int cnt, int tid) {
    if constexpr (NW > 1) {
        __shared__ double buf[NW][CAP];
        if ((tid & (kWave - 1)) == 0)
            for (int i = 0; i < cnt; ++i) buf[tid / kWave][i] = v[i];
        __syncthreads();
        for (int i = 0; i < cnt; ++i) {
            double a = buf[0][i];
            for (int w = 1; w < NW; ++w) a += buf[w][i];
            v[i] = a;
        }
        __syncthreads();  // the slots are free again
    }
}

template <int PP, typename FT, int NW, bool SPAN>
__device__ __forceinline__ void reduced_solve(const SysDesc& sd, int tid, FT* red, bool factor, FT* zl,
                                              const SpanCtx<FT>& sc) {
    if constexpr (NW == 4) pass_reduced_cr<PP, FT, 4, SPAN>(sd, tid, red, factor, zl, sc);
    else if constexpr (NW == 2) pass_reduced2<PP, FT>(sd, tid, red, factor, zl);
    else pass_reduced<PP, FT>(sd, tid, red, factor, zl);
}

// NW = 1: one wave owns the system (P <= 64).  NW = 2: two waves (P in
// 65..128); thread t owns chunk t in the lane-serial passes, the separator
// system is solved from both ends (pass_reduced2) and the observable sums
// are combined across the waves through LDS.  NW = 4: four waves (P in
// 129..256), the separator system by block cyclic reduction
// (pass_reduced_cr).  XT: the extended kernels (an
// absorbing potential in A_n and B_n, the extended series of section V.D,
// the a_Q term of the acceleration).  SPAN: one system on sd.G workgroups of
// four waves (a cooperative launch): workgroup g owns chunks g Pl ..
// (g + 1) Pl - 1, the separator system is reduced per workgroup and the
// super blocks solved in every workgroup after a grid barrier, a second grid
// barrier follows every back substitution (the next pass reads the
// neighbouring workgroups' state rows), and the observable sums are written
// per workgroup (ka.obs_part) and added up after the launch.
template <int PP, typename FT, int NW, bool XT, bool SPAN = false>
__device__ __forceinline__ void run_system(const KernelArgs& ka, const SysDesc& sd, int sidx, FT* zl) {
    // optional phase profile: shader-clock cycles summed over the steps for
    // the passes H, A1 (FP32: one fused sweep counted under H), A2, R, B and,
    // per refinement sweep, C, R, B
    unsigned long long tp[kProfSlots - 2] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long t0 = 0;
    double worst_rel = 0.0;  // largest relative residual entering the last sweep
    const FT* band = (const FT*)ka.band;
    FT* fac = (FT*)ka.fac;
    FT* red = (FT*)ka.red;
    FT* rhs = (FT*)ka.rhs;
    double* st = ka.st;
    const int tid = threadIdx.x;
    const int wg = SPAN ? (int)blockIdx.x : 0;
    const int lane = SPAN ? wg * sd.Pl + tid : tid;  // chunk index
    const bool active = SPAN ? (tid < sd.Pl && lane < sd.P) : lane < sd.P;
    SpanCtx<FT> sc{0, sd.P, 0, 1, nullptr, nullptr};
    int phase = 0;  // reduced solves so far (SPAN: exchange buffer parity)
    if constexpr (SPAN) {
        sc.k0 = wg * sd.Pl;
        sc.Pl = sd.Pl;
        sc.g = wg;
        sc.G = sd.G;
        sc.gfac = (FT*)ka.gfac + 2 * (long long)wg * (sd.G + 1) * gfac_entry(PP);
    }
    auto span_ctx = [&]() {
        SpanCtx<FT> c = sc;
        if constexpr (SPAN) c.xch = (FT*)ka.xch + 2 * (long long)(phase & 1) * sd.G * xch_entry(PP);
        ++phase;
        return c;
    };
    const double alpha = 0.5 * sd.dt;
    const double* Es = ka.E + sd.E_off;
    double* os = ka.obs ? ka.obs + sd.obs_off : nullptr;
    const unsigned mask = ka.mask;
    const bool want_acc = (mask & TDSEZ_OBS_ACCEL) != 0;
    const int refine = ka.refine;
    double* dtot = refine > 0 ? ka.dtot : nullptr;
    const bool prof = ka.prof != nullptr;
    // extended pass: the extended series, or the a_Q part of the acceleration
    const bool want_ext = XT && (ka.ext != nullptr || (want_acc && sd.aq != 0));
    double* xo = (XT && ka.ext) ? ka.ext + sd.ext_off : nullptr;
    const int next = kExtFixed + sd.npop;
    // phase boundary: a barrier (so the clock covers the whole wave) when
    // profiling, then the cycles since the last boundary go to slot k
    auto mark = [&](int k) {
        if (prof) {
            __syncthreads();
            const unsigned long long t = clock64();
            tp[k] += t - t0;
            t0 = t;
        }
    };
    double nu0 = 0.0;
    for (int n = 0; n <= sd.nsteps; ++n) {
        const bool last = (n == sd.nsteps);
        const double En = Es[n];
        const double Ebar = last ? En : 0.5 * (En + Es[n + 1]);
        double part[3] = {0.0, 0.0, 0.0};
        double xs[XT ? kExtSums : 1];
        if constexpr (XT) {
            for (int i = 0; i < kExtSums; ++i) xs[i] = 0.0;
            if (want_ext && active) pass_extobs<PP>(sd, lane, ka.band64, st, ka.c0, ka.proj, xs);
        }
        if (prof) t0 = clock64();
        // FP32: right-hand side, observables and elimination in one sweep
        // (FP64 rows are twice the size and keep two passes); the last time
        // level needs the observables only
        constexpr bool kOneSweep = sizeof(FT) == 4;
        if (active) {
            if (kOneSweep && !last)
                pass_rhs_elim<PP, FT, XT>(sd, lane, band, st, fac, red, alpha, Ebar, En, want_acc, part);
            else
                pass_rhs<PP, FT, XT>(sd, lane, band, st, rhs, alpha, Ebar, En, want_acc, !last, part);
        }
        mark(0);
        if (!kOneSweep && active && !last)
            pass_elim<PP, FT, false, XT>(sd, lane, band, rhs, fac, red, alpha, Ebar);
        mark(1);
        if (active && !last) {
            constexpr bool kFused = sizeof(FT) == 4;
            pass_fill<PP, FT, kFused, XT>(sd, lane, band, fac, red, alpha, Ebar);
            if (!kFused) pass_schur<PP, FT>(sd, lane, fac, red);
        }
        double sums[3] = {wave_sum(part[0]), wave_sum(part[1]), wave_sum(part[2])};
        combine_waves<NW>(sums, 3, tid);
        double nu = sums[0], dip = sums[1], acc = sums[2];
        if constexpr (XT) {
            if (want_ext) {
                const int cnt = 8 + 2 * sd.npop;
                for (int i = 0; i < cnt; ++i) xs[i] = wave_sum(xs[i]);
                combine_waves<NW>(xs, cnt, tid);
                if (want_acc && sd.aq) acc += xs[4];
            }
        }
        if constexpr (SPAN) {
            // this workgroup's parts; the sums and the finiteness check follow
            // the launch (no workgroup may leave before the others)
            if (tid == 0 && ka.obs_part) {
                double* op = ka.obs_part + 3 * ((long long)n * sd.G + wg);
                op[0] = nu;
                op[1] = dip;
                op[2] = acc;
            }
        } else if (lane == 0 && os) {
            os[3 * n + 0] = (mask & TDSEZ_OBS_NORM) ? nu : 0.0;
            os[3 * n + 1] = (mask & TDSEZ_OBS_DIPOLE) ? dip : 0.0;
            os[3 * n + 2] = want_acc ? acc : 0.0;
        }
        if constexpr (XT) {
            if (lane == 0 && xo) {
                double* o = xo + (long long)next * n;
                o[0] = xs[0] - xs[1];          // kinetic
                o[1] = xs[1];                  // potential
                o[2] = En * dip;               // laser interaction
                o[3] = o[0] + o[1] + o[2];     // total
                o[4] = xs[2];                  // <m^-1>
                o[5] = xs[3];                  // velocity
                o[6] = xs[4];                  // a_Q
                o[7] = xs[5];                  // <W>
                o[8] = xs[6];                  // autocorrelation
                o[9] = xs[7];
                for (int q = 0; q < sd.npop; ++q)
                    o[kExtFixed + q] = xs[8 + 2 * q] * xs[8 + 2 * q] + xs[9 + 2 * q] * xs[9 + 2 * q];
            }
        }
        if (n == 0) nu0 = nu;
        if constexpr (!SPAN) {
            if (!isfinite(nu) || !isfinite(dip) || !isfinite(acc)) {
                if (lane == 0) latch(ka.status, TDSEZ_ENONFINITE, sidx, n);
                return;
            }
            if (ka.norm_tol > 0.0 && fabs(nu / nu0 - 1.0) > ka.norm_tol) {
                if (lane == 0) latch(ka.status, TDSEZ_ENORMDRIFT, sidx, n);
                return;
            }
        }
        if (last) break;
        __syncthreads();
        mark(2);
        reduced_solve<PP, FT, NW, SPAN>(sd, tid, red, true, zl, span_ctx());
        __syncthreads();
        mark(3);
        if (active) pass_backsub<PP, FT, XT>(sd, lane, band, st, dtot, true, fac, red, alpha, Ebar);
        if constexpr (SPAN) grid_barrier();
        __syncthreads();
        mark(4);
        // refinement sweeps exist for the FP32 factorisation only (FP64
        // launches pass refine = 0); FP64 code is built without them
        if constexpr (sizeof(FT) == 4) for (int sweep = 0; sweep < refine; ++sweep) {
            double nrm[2] = {0.0, 0.0};
            if (active)
                pass_residual<PP, FT, XT>(sd, lane, band, ka.band64, ka.bandlo, st, dtot, fac, red, alpha, Ebar,
                                          nrm);
            __syncthreads();
            mark(5);
            if (sweep + 1 == refine) {
                // the last sweep's starting residual measures the FP32
                // factorisation; beyond the batch tolerance the sweeps are
                // not converging (latched, the propagation goes on)
                // (SPAN: this workgroup's rows only)
                double rs[2] = {wave_sum(nrm[0]), wave_sum(nrm[1])};
                combine_waves<NW>(rs, 2, tid);
                const double rel = rs[1] > 0.0 ? sqrt(rs[0] / rs[1]) : 0.0;
                worst_rel = fmax(worst_rel, rel);
                if (!(rel <= ka.refine_tol) && tid == 0) latch(ka.status, TDSEZ_ENOCONV, sidx, n);
            }
            reduced_solve<PP, FT, NW, SPAN>(sd, tid, red, false, zl, span_ctx());
            __syncthreads();
            mark(6);
            if (active)
                pass_backsub<PP, FT, XT>(sd, lane, band, st, sweep + 1 < refine ? dtot : nullptr, false, fac,
                                         red, alpha, Ebar);
            if constexpr (SPAN) grid_barrier();
            __syncthreads();
            mark(7);
        }
    }
    if (prof && lane == 0 && tid == 0) {
        unsigned long long* pr = ka.prof + kProfSlots * sidx;
        for (int k = 0; k < kProfSlots - 2; ++k) pr[k] = tp[k];
        pr[kProfSlots - 2] = (unsigned long long)sd.nsteps;
        pr[kProfSlots - 1] = (unsigned long long)__double_as_longlong(worst_rel);
    }
}

// zl: the separator recurrence's right-hand-side vector, P * p complex in
// LDS, one array per kernel (shared by the p variants)
template <typename FT, int NW, bool XT, bool SPAN = false>
__device__ __forceinline__ void dispatch_system(const KernelArgs& ka) {
    // (four waves: the cyclic reduction's g vectors and block staging)
    __shared__ FT zl[NW == 4 ? CrLds<FT>::kTotal : 2 * kMaxP * kWave * NW];
    // a spanning launch holds one system (all its workgroups)
    const int sidx = ka.order[ka.order_off + (SPAN ? 0 : (int)blockIdx.x)];
    const SysDesc sd = ka.descs[sidx];
    switch (sd.p) {
        case 1: run_system<1, FT, NW, XT, SPAN>(ka, sd, sidx, zl); break;
        case 2: run_system<2, FT, NW, XT, SPAN>(ka, sd, sidx, zl); break;
        case 3: run_system<3, FT, NW, XT, SPAN>(ka, sd, sidx, zl); break;
        case 4: run_system<4, FT, NW, XT, SPAN>(ka, sd, sidx, zl); break;
        case 5: run_system<5, FT, NW, XT, SPAN>(ka, sd, sidx, zl); break;
        case 6: run_system<6, FT, NW, XT, SPAN>(ka, sd, sidx, zl); break;
        case 7: run_system<7, FT, NW, XT, SPAN>(ka, sd, sidx, zl); break;
        default: break;
    }
}

}  // namespace
}  // namespace tdsez

// Kernel names are per translation unit: the plain kernels keep the names
// propagate_kernel / propagate2_kernel / propagate4_kernel (one, two and four
// waves per system) and tune_probe*_kernel (the autotuner's probes), the
// extended ones propagate_xt_kernel / propagate2_xt_kernel /
// propagate4_xt_kernel.  Launch groups: entries 0..n4-1 of the order on s4,
// the next n2 on s2, the n1 after them on s1.
#define TDSEZ_LAUNCH_GROUP(KERNEL, T, NWAVES, COUNT, OFF, STREAM)                                           \
    if ((COUNT) > 0) {                                                                                     \
        k.order_off = (OFF);                                                                               \
        KERNEL<T><<<(COUNT), (NWAVES) * kWave, 0, (STREAM)>>>(k);                                         \
        hipError_t e = hipGetLastError();                                                                  \
        if (e != hipSuccess) return e;                                                                     \
    }

#define TDSEZ_DEFINE_PLAIN_LAUNCHER(FT, NAME)                                                               \
    namespace tdsez {                                                                                      \
    namespace {                                                                                            \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(kWave) void propagate_kernel(KernelArgs ka) { dispatch_system<T, 1, false>(ka); } \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(2 * kWave) void propagate2_kernel(KernelArgs ka) {                        \
        dispatch_system<T, 2, false>(ka);                                                                  \
    }                                                                                                      \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(4 * kWave) void propagate4_kernel(KernelArgs ka) {                        \
        dispatch_system<T, 4, false>(ka);                                                                  \
    }                                                                                                      \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(kWave) void tune_probe_kernel(KernelArgs ka) {                            \
        dispatch_system<T, 1, false>(ka);                                                                  \
    }                                                                                                      \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(2 * kWave) void tune_probe2_kernel(KernelArgs ka) {                       \
        dispatch_system<T, 2, false>(ka);                                                                  \
    }                                                                                                      \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(4 * kWave) void tune_probe4_kernel(KernelArgs ka) {                       \
        dispatch_system<T, 4, false>(ka);                                                                  \
    }                                                                                                      \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(4 * kWave) void propagate_span_kernel(KernelArgs ka) {                    \
        dispatch_system<T, 4, false, true>(ka);                                                            \
    }                                                                                                      \
    }                                                                                                      \
    hipError_t NAME##_span(const KernelArgs& ka, int G, hipStream_t s) {                                   \
        KernelArgs k = ka;                                                                                 \
        void* args[] = {&k};                                                                               \
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&propagate_span_kernel<FT>),       \
                                          dim3(G), dim3(4 * kWave), args, 0, s);                          \
    }                                                                                                      \
    hipError_t NAME(const KernelArgs& ka, int n4, int n2, int n1, hipStream_t s4, hipStream_t s2,         \
                    hipStream_t s1, bool probe) {                                                          \
        KernelArgs k = ka;                                                                                 \
        if (probe) {                                                                                       \
            TDSEZ_LAUNCH_GROUP(tune_probe4_kernel, FT, 4, n4, 0, s4)                                           \
            TDSEZ_LAUNCH_GROUP(tune_probe2_kernel, FT, 2, n2, n4, s2)                                          \
            TDSEZ_LAUNCH_GROUP(tune_probe_kernel, FT, 1, n1, n4 + n2, s1)                                      \
        } else {                                                                                           \
            TDSEZ_LAUNCH_GROUP(propagate4_kernel, FT, 4, n4, 0, s4)                                            \
            TDSEZ_LAUNCH_GROUP(propagate2_kernel, FT, 2, n2, n4, s2)                                           \
            TDSEZ_LAUNCH_GROUP(propagate_kernel, FT, 1, n1, n4 + n2, s1)                                       \
        }                                                                                                  \
        return hipSuccess;                                                                                 \
    }                                                                                                      \
    }

#define TDSEZ_DEFINE_XT_LAUNCHER(FT, NAME)                                                                  \
    namespace tdsez {                                                                                      \
    namespace {                                                                                            \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(kWave) void propagate_xt_kernel(KernelArgs ka) {                          \
        dispatch_system<T, 1, true>(ka);                                                                   \
    }                                                                                                      \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(2 * kWave) void propagate2_xt_kernel(KernelArgs ka) {                     \
        dispatch_system<T, 2, true>(ka);                                                                   \
    }                                                                                                      \
    template <typename T>                                                                                  \
    __global__ __launch_bounds__(4 * kWave) void propagate4_xt_kernel(KernelArgs ka) {                     \
        dispatch_system<T, 4, true>(ka);                                                                   \
    }                                                                                                      \
    }                                                                                                      \
    hipError_t NAME(const KernelArgs& ka, int n4, int n2, int n1, hipStream_t s4, hipStream_t s2,         \
                    hipStream_t s1) {                                                                      \
        KernelArgs k = ka;                                                                                 \
        TDSEZ_LAUNCH_GROUP(propagate4_xt_kernel, FT, 4, n4, 0, s4)                                             \
        TDSEZ_LAUNCH_GROUP(propagate2_xt_kernel, FT, 2, n2, n4, s2)                                            \
        TDSEZ_LAUNCH_GROUP(propagate_xt_kernel, FT, 1, n1, n4 + n2, s1)                                        \
        return hipSuccess;                                                                                 \
    }                                                                                                      \
    }
