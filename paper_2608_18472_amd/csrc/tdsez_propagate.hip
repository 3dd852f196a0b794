// Crank-Nicolson propagation kernels (the paper's section V.B, eq. cn_system).
//
// One workgroup per system (one wave64, or two or four for systems
// partitioned into more than 64 or 128 chunks); every system of a batch runs
// all its time steps inside one persistent launch (one launch per workgroup
// size).  Per step n, with
// H_n = H0 + Ebar_n D, Ebar_n = (E_n + E_{n+1})/2, A_n = S + i(dt/2) H_n:
//
//   A_n (c_{n+1} - c_n) = -i dt H_n c_n                               (1)
//
// which is eq. cn_system rewritten for the increment: the right-hand side
// is the residual (B_n - A_n) c_n of the initial guess c_n, so each step is
// one sweep of iterative refinement started from the previous state.  The
// residual, the state and every reduction are FP64; the factorisation and
// the banded solve run in FT (double, or float for the FP32 path).
//
// The banded solve of (1) is partitioned so that one long chain runs in
// parallel.  The N rows (padded with decoupled identity rows to P*L) are
// split into P chunks of L rows; the last p rows of every chunk form a
// separator.  Lane k owns chunk k and, in one top-down sweep:
//   - streams its band rows and state (a halo of p rows of the next chunk),
//   - forms (1)'s right-hand side and the FP64 observables of c_n,
//   - eliminates its m = L - p interior rows by right-looking complex
//     symmetric LDL^T (no pivoting: the Hermitian part S of A_n is positive
//     definite), carrying the coupling to the left separator as fill,
//   - leaves the 2p x 2p Schur complement on its two separators.
// The separators form a block tridiagonal system (p x p blocks) that the
// workgroup solves with entry-parallel block operations: by block LDL^T
// (one wave, or from both ends on two) or by block cyclic reduction (four).
// Two more lane-serial sweeps (forward correction for the separator values,
// then back substitution) recover the interior increments.
//
// Layouts (all "interleaved": lane k reads column k+1, so one wave load of a
// given local row is contiguous; columns 0 and P+1 are zero halos):
//   bands  [l][mat][d][col]  mat = S, H0, D, G, Mi; entry M[row][row-d],
//                           row = k*L + l
//   state  [l][col]          complex128
//   factor [j][item][k]      2p+2 items per interior pivot j (fac_items)
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "tdsez_passes.hpp"
// (the kernels themselves are instantiated in tdsez_prop_*.hip from tdsez_run.hpp)

namespace tdsez {

namespace {

// psi (natural order, complex128) <-> interleaved padded state
// (c0 != nullptr: also a copy of the initial state for the autocorrelation)
__global__ void pack_state_kernel(const SysDesc* __restrict__ descs, const double* __restrict__ psi,
                                  double* __restrict__ st, double* __restrict__ c0) {
    const SysDesc sd = descs[blockIdx.y];
    const long long total = (long long)sd.L * sd.LS;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int l = (int)(e / sd.LS), colx = (int)(e % sd.LS);
        int k = colx - 1;
        double re = 0.0, im = 0.0;
        if (k >= 0 && k < sd.P) {
            long long row = (long long)k * sd.L + l;
            if (row < sd.N) {
                re = psi[2 * (sd.psi_off + row)];
                im = psi[2 * (sd.psi_off + row) + 1];
            }
        }
        st[2 * (sd.state_off + e)] = re;
        st[2 * (sd.state_off + e) + 1] = im;
        if (c0) {
            c0[2 * (sd.state_off + e)] = re;
            c0[2 * (sd.state_off + e) + 1] = im;
        }
    }
}

// projection states S phi_k (natural order, npop x N) -> interleaved
// [k][l][column] layout of one system
__global__ void pack_proj_kernel(const double* __restrict__ src, int npop, int N, int P, int L, int LS,
                                 double* __restrict__ out) {
    const long long total = (long long)npop * L * LS;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int colx = (int)(e % LS);
        const long long r1 = e / LS;
        const int l = (int)(r1 % L), q = (int)(r1 / L);
        const int k = colx - 1;
        double v = 0.0;
        if (k >= 0 && k < P) {
            const long long row = (long long)k * L + l;
            if (row < N) v = src[(long long)q * N + row];
        }
        out[e] = v;
    }
}

__global__ void unpack_state_kernel(const SysDesc* __restrict__ descs, const double* __restrict__ st,
                                    double* __restrict__ psi) {
    const SysDesc sd = descs[blockIdx.y];
    for (long long row = blockIdx.x * (long long)blockDim.x + threadIdx.x; row < sd.N;
         row += (long long)gridDim.x * blockDim.x) {
        int k = (int)(row / sd.L), l = (int)(row % sd.L);
        long long e = (long long)l * sd.LS + k + 1;
        psi[2 * (sd.psi_off + row)] = st[2 * (sd.state_off + e)];
        psi[2 * (sd.psi_off + row) + 1] = st[2 * (sd.state_off + e) + 1];
    }
}

// FP64 master bands (lower half by rows) -> interleaved padded propagation
// layout in FP64 and FP32.  Padding rows are decoupled identity rows.
// Matrices in the kMat* order; a NULL source packs zeros.
struct BandSrc {
    const double* m[kNumMats];
};
__global__ void pack_band_kernel(BandSrc src, int N, int p, int P, int L, int LS,
                                 double* __restrict__ out64, float* __restrict__ out32) {
    const long long total = (long long)L * kNumMats * (p + 1) * LS;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int colx = (int)(e % LS);
        long long r1 = e / LS;
        int d = (int)(r1 % (p + 1));
        long long r2 = r1 / (p + 1);
        int mat = (int)(r2 % kNumMats);
        int l = (int)(r2 / kNumMats);
        int k = colx - 1;
        double v = 0.0;
        if (k >= 0 && k < P) {
            long long row = (long long)k * L + l;
            if (row < N) {
                const double* m = src.m[mat];
                v = m ? m[row * (p + 1) + d] : 0.0;
            } else if (mat == kMatS && d == 0) {
                v = 1.0;
            }
        }
        out64[e] = v;
        out32[e] = (float)v;
    }
}

// Signed 8-bit code of an FP64 band entry v against its FP32 rounding hi:
// the q for which hi (1 + q kLoScale) is nearest to v.
__device__ __forceinline__ int band_code(double v) {
    const float hi = (float)v;
    if (hi == 0.0f) return 0;
    const double t = rint((v - (double)hi) / ((double)hi * kLoScale));
    return (int)fmin(127.0, fmax(-127.0, t));
}

// Corrections of the FP32 S, H0, D bands for the refinement residual, from
// the packed FP64 bands of one system: word (l, m, c) holds the codes of the
// p + 1 diagonals of matrix m at row l, column c (byte d = diagonal d).
__global__ void pack_lo_kernel(const double* __restrict__ b64, int p, int L, int LS,
                               unsigned long long* __restrict__ lo) {
    const long long total = (long long)L * 3 * LS;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int col = (int)(e % LS);
        const long long r = e / LS;
        const int m = (int)(r % 3);  // kMatS, kMatH0, kMatD
        const long long l = r / 3;
        unsigned long long w = 0;
        for (int d = 0; d <= p; ++d) {
            const double v = b64[((l * kNumMats + m) * (p + 1) + d) * LS + col];
            w |= (unsigned long long)(unsigned char)(signed char)band_code(v) << (8 * d);
        }
        lo[e] = w;
    }
}

}  // namespace

// Observables of a spanning system: the per-workgroup parts of every step
// added in workgroup order; the earliest non-finite step is latched as in
// the one-workgroup kernels.  One workgroup of 256 threads.
__global__ void span_sum_kernel(const double* __restrict__ part, int G, int nsteps, double* __restrict__ obs,
                                unsigned mask, int* __restrict__ status) {
    __shared__ int first[256];
    int bad = nsteps + 1;
    for (int n = threadIdx.x; n <= nsteps; n += blockDim.x) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int g = 0; g < G; ++g)
            for (int c = 0; c < 3; ++c) v[c] += part[3 * ((long long)n * G + g) + c];
        if (obs) {
            obs[3 * n + 0] = (mask & TDSEZ_OBS_NORM) ? v[0] : 0.0;
            obs[3 * n + 1] = (mask & TDSEZ_OBS_DIPOLE) ? v[1] : 0.0;
            obs[3 * n + 2] = (mask & TDSEZ_OBS_ACCEL) ? v[2] : 0.0;
        }
        if ((!isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2])) && n < bad) bad = n;
    }
    first[threadIdx.x] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = nsteps + 1;
        for (int t = 0; t < (int)blockDim.x; ++t) m = first[t] < m ? first[t] : m;
        if (m <= nsteps) latch(status, TDSEZ_ENONFINITE, 0, m);
    }
}

Plan make_plan(int N, int p, int force_chunks, int max_chunks, double rule) {
    Plan pl;
    pl.N = N;
    pl.p = p;
    int P;
    if (force_chunks > 0) {
        P = force_chunks;
    } else {
        // balance the lane-serial sweep (~L rows) against the serial block
        // chain of the reduced system (~P blocks; P/2 on two waves, hence
        // half the rule constant there)
        double Lopt = std::sqrt(rule * N);
        if (Lopt < 2.0 * p + 2) Lopt = 2.0 * p + 2;
        P = (int)std::lround(N / Lopt);
    }
    if (P < 1) P = 1;
    if (P > max_chunks) P = max_chunks;
    for (;;) {
        int L = (N + P - 1) / P;
        if (L < 2 * p) L = 2 * p;
        if (L - p >= p || P == 1) {
            pl.P = P;
            pl.L = L;
            pl.m = L - p;
            break;
        }
        --P;
    }
    pl.LS = pl.P + 2;
    return pl;
}

Plan multi_wave_plan(int N, int p, int force_chunks, int max_waves) {
    const int cap = max_waves >= 4 ? kMaxChunks4 : max_waves == 2 ? kMaxChunks2 : kMaxChunks;
    if (force_chunks > 0) return make_plan(N, p, force_chunks, cap);
    if (max_waves >= 4) {
        Plan p4 = make_plan(N, p, 0, kMaxChunks4, kRule4);
        if (p4.P > kMaxChunks2) return p4;
    }
    if (max_waves >= 2) {
        Plan p2 = make_plan(N, p, 0, kMaxChunks2, kRule2);
        if (p2.P > kMaxChunks) return p2;
    }
    return make_plan(N, p, 0);
}

int span_plan(int N, int p, int G, int Pl, Plan* out) {
    if (Pl <= 0) Pl = 64;
    if (Pl > kMaxChunks4) Pl = kMaxChunks4;
    if (G <= 0) {
        // chunks of about 2p + 1 rows (measured on the 30 007-row H2+ chain:
        // 64 chunks per workgroup and 15- to 16-row chunks beat 32, 48, 96,
        // 128 or 256 chunks per workgroup and 17- to 21-row chunks)
        const double Lt = 2.0 * p + 1.0;
        G = (int)std::lround(N / (Lt * Pl));
        if (G > kMaxSpan) G = kMaxSpan;
    }
    // every chunk needs at least 2p rows
    while (G > 1 && (long long)G * Pl * 2 * p > N) --G;
    if (G < 2) return 1;
    *out = make_plan(N, p, G * Pl, G * Pl);
    return out->P == G * Pl ? G : 1;
}

// The one-workgroup plan of a lone system (tdsez_propagate and the
// allocation-free call): the multi-wave plan, but on two waves as soon as 65
// chunks of at least 2p rows fit.  A lone system is latency-bound, so the
// shorter chunks and the two-ended separator chain pay where the batch rule
// (which weighs the waves against the other systems) keeps one wave.
static Plan lone_plan(int N, int p) {
    Plan pl = multi_wave_plan(N, p, 0, 4);
    if (plan_waves(pl) == 1 && (N + kMaxChunks) / (kMaxChunks + 1) >= 2 * p) {
        const Plan p2 = make_plan(N, p, kMaxChunks + 1, kMaxChunks2);
        if (p2.P == kMaxChunks + 1) pl = p2;
    }
    return pl;
}

tdsez_status pack_bands(BatchData* b) {
    const int nsys = (int)b->sys.size();
    b->plan.resize(nsys);
    b->desc.resize(nsys);
    long long boff = 0, soff = 0, foff = 0, roff = 0, poff = 0;
    b->maxp = 0;
    b->any_cap = b->any_aq = false;
    b->waves.assign(nsys, 1);
    b->nsplit = 0;
    b->n4 = 0;
    b->span_G = 1;
    for (int s = 0; s < nsys; ++s) {
        SystemData* sy = b->sys[s];
        const int tuned = s < (int)b->tuned_chunks.size() ? b->tuned_chunks[s] : 0;
        const bool req = s < (int)b->two_wave_req.size() && b->two_wave_req[s];
        const int force = b->force_chunks > 0 ? b->force_chunks : tuned;
        // a marked system runs on the most waves whose rule needs them (a
        // system whose two-wave rule gives at most 64 chunks stays on one
        // wave, with the one-wave rule); an unmarked one on one wave
        Plan pl = multi_wave_plan(sy->N, sy->p, force, req ? b->max_waves : 1);
        if (b->solo && nsys == 1 && force == 0 && req && b->max_waves >= 4) pl = lone_plan(sy->N, sy->p);
        // the one-system plan of tdsez_propagate spreads a long chain over
        // several workgroups: automatically once the four-wave plan holds
        // chunks of more than 48 rows, or as set by tdsez_system_set
        if (b->solo && nsys == 1 && force == 0 && sy->span_G != 1) {
            const bool want = sy->span_G > 1 || (pl.P == kMaxChunks4 && pl.L > 48);
            Plan sp;
            if (want) {
                const int G = span_plan(sy->N, sy->p, sy->span_G, sy->span_Pl, &sp);
                if (G > 1) {
                    pl = sp;
                    b->span_G = G;
                }
            }
        }
        b->plan[s] = pl;
        b->waves[s] = (char)plan_waves(pl);
        if (b->waves[s] > 1) ++b->nsplit;
        if (b->waves[s] == 4) ++b->n4;
        SysDesc& d = b->desc[s];
        d = SysDesc{};
        d.N = pl.N; d.p = pl.p; d.P = pl.P; d.L = pl.L; d.m = pl.m; d.LS = pl.LS;
        d.G = b->span_G;
        d.Pl = pl.P / b->span_G;
        d.mi_is_s = sy->const_mass ? 1 : 0;
        d.cap = sy->d_W ? 1 : 0;
        d.aq = sy->d_Q ? 1 : 0;
        d.npop = sy->npop;
        d.proj_off = poff;
        poff += (long long)sy->npop * pl.L * pl.LS;
        b->any_cap = b->any_cap || d.cap;
        b->any_aq = b->any_aq || d.aq;
        d.band_off = boff;
        d.state_off = soff;
        d.fac_off = foff;
        d.red_off = roff;
        boff += (long long)pl.L * kNumMats * (pl.p + 1) * pl.LS;
        soff += (long long)pl.L * pl.LS;
        foff += (long long)pl.m * fac_items(pl.p) * pl.P;
        roff += RedLayout<double>::total(pl.p, pl.P);
        if (pl.p > b->maxp) b->maxp = pl.p;
    }
    b->band_elems = boff;
    b->state_elems = soff;
    b->fac_elems64 = foff;
    b->red_elems64 = roff;
    TDSEZ_HIP_TRY(hipMalloc(&b->d_band64, sizeof(double) * (size_t)boff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_band32, sizeof(float) * (size_t)boff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_bandlo, sizeof(unsigned long long) * 3 * (size_t)soff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_state, 2 * sizeof(double) * (size_t)soff));
    // increments of the refinement sweeps; the halo columns stay zero
    TDSEZ_HIP_TRY(hipMalloc(&b->d_dtot, 2 * sizeof(double) * (size_t)soff));
    TDSEZ_HIP_TRY(hipMemset(b->d_dtot, 0, 2 * sizeof(double) * (size_t)soff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_rhs, 2 * sizeof(double) * (size_t)soff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_fac, 2 * sizeof(double) * (size_t)(foff > 0 ? foff : 1)));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_red, 2 * sizeof(double) * (size_t)roff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_desc, sizeof(SysDesc) * nsys));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_order, sizeof(int) * nsys));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_status, sizeof(int) * 4));
    if (poff > 0) TDSEZ_HIP_TRY(hipMalloc(&b->d_proj, sizeof(double) * (size_t)poff));
    TDSEZ_HIP_TRY(hipMemset(b->d_status, 0, sizeof(int) * 4));
    b->nsys_alloc_desc = nsys;
    b->desc_on_device.clear();
    if (b->nsplit > 0 && !b->side) {
        TDSEZ_HIP_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
        TDSEZ_HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        TDSEZ_HIP_TRY(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    }
    if (b->n4 > 0 && b->nsplit > b->n4 && !b->side2) {
        TDSEZ_HIP_TRY(hipStreamCreateWithFlags(&b->side2, hipStreamNonBlocking));
        TDSEZ_HIP_TRY(hipEventCreateWithFlags(&b->ev_join2, hipEventDisableTiming));
    }
    for (int s = 0; s < nsys; ++s) {
        SystemData* sy = b->sys[s];
        const Plan& pl = b->plan[s];
        long long total = (long long)pl.L * kNumMats * (pl.p + 1) * pl.LS;
        int th = 256;
        int nb = (int)std::min<long long>((total + th - 1) / th, 4096);
        BandSrc src;
        src.m[kMatS] = sy->d_band[0];
        src.m[kMatH0] = sy->d_H0;
        src.m[kMatD] = sy->d_band[3];
        src.m[kMatG] = sy->d_band[4];
        src.m[kMatMi] = sy->d_band[5];
        src.m[kMatW] = sy->d_W;
        src.m[kMatV] = sy->d_band[2];
        src.m[kMatK] = sy->d_K;
        src.m[kMatQ] = sy->d_Q;
        pack_band_kernel<<<nb, th>>>(src, pl.N, pl.p, pl.P, pl.L, pl.LS, b->d_band64 + b->desc[s].band_off,
                                     b->d_band32 + b->desc[s].band_off);
        TDSEZ_HIP_TRY(hipGetLastError());
        {
            const long long nlo = 3LL * pl.L * pl.LS;
            pack_lo_kernel<<<(int)std::min<long long>((nlo + th - 1) / th, 4096), th>>>(
                b->d_band64 + b->desc[s].band_off, pl.p, pl.L, pl.LS, b->d_bandlo + 3 * b->desc[s].state_off);
            TDSEZ_HIP_TRY(hipGetLastError());
        }
        if (sy->npop > 0) {
            long long tp = (long long)sy->npop * pl.L * pl.LS;
            pack_proj_kernel<<<(int)std::min<long long>((tp + 255) / 256, 4096), 256>>>(
                sy->d_pops, sy->npop, pl.N, pl.P, pl.L, pl.LS, b->d_proj + b->desc[s].proj_off);
            TDSEZ_HIP_TRY(hipGetLastError());
        }
    }
    TDSEZ_HIP_TRY(hipDeviceSynchronize());
    return TDSEZ_OK;
}

tdsez_status upload_descriptors(BatchData* b, hipStream_t stream) {
    const size_t n = b->desc.size();
    if (b->desc_on_device.size() == n &&
        std::memcmp(b->desc_on_device.data(), b->desc.data(), sizeof(SysDesc) * n) == 0)
        return TDSEZ_OK;
    // an upload is a copy from pageable host memory, which a stream capture
    // cannot hold: a captured call must repeat the previous call's arguments
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    TDSEZ_HIP_TRY(hipStreamIsCapturing(stream, &cap));
    if (cap != hipStreamCaptureStatusNone) {
        size_t at = 0;
        if (b->desc_on_device.size() == n) {
            const unsigned char* x = reinterpret_cast<const unsigned char*>(b->desc_on_device.data());
            const unsigned char* y = reinterpret_cast<const unsigned char*>(b->desc.data());
            while (at < sizeof(SysDesc) * n && x[at] == y[at]) ++at;
        }
        return fail(TDSEZ_EINVAL,
                    "captured propagation call with arguments that differ from the previous call (descriptor byte "
                    "%zu of %zu): run the call once eagerly with the same arguments first",
                    at, sizeof(SysDesc) * n);
    }
    // Workgroups are dispatched in index order, so when the batch holds more
    // systems than the device has wave slots the costliest ones (cost
    // N (p + 1) nsteps) start first and the short ones fill in behind them.
    // Four-wave systems come first, then two-wave systems (each launch reads
    // its own range of entries), each group longest first.
    b->order_host.resize(n);
    for (size_t s = 0; s < n; ++s) b->order_host[s] = (int)s;
    auto cost = [&](int s) {
        const SysDesc& d = b->desc[s];
        return (double)d.N * (d.p + 1) * (double)d.nsteps;
    };
    auto waves = [&](int s) { return s < (int)b->waves.size() ? (int)b->waves[s] : 1; };
    std::stable_sort(b->order_host.begin(), b->order_host.end(), [&](int x, int y) {
        if (waves(x) != waves(y)) return waves(x) > waves(y);
        return cost(x) > cost(y);
    });
    TDSEZ_HIP_TRY(hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(SysDesc) * n, hipMemcpyHostToDevice, stream));
    TDSEZ_HIP_TRY(hipMemcpyAsync(b->d_order, b->order_host.data(), sizeof(int) * n, hipMemcpyHostToDevice,
                                 stream));
    b->desc_on_device = b->desc;
    return TDSEZ_OK;
}

tdsez_status launch_propagate(BatchData* b, double* psi, const double* E, double* obs,
                              tdsez_precision prec, unsigned obs_mask, hipStream_t stream, bool probe,
                              double* ext) {
    const int nsys = (int)b->sys.size();
    if (tdsez_status st = upload_descriptors(b, stream)) return st;
    long long maxL = 1, maxN = 1;
    for (const auto& pl : b->plan) {
        maxL = std::max<long long>(maxL, (long long)pl.L * pl.LS);
        maxN = std::max<long long>(maxN, pl.N);
    }
    {
        dim3 grid((unsigned)std::min<long long>((maxL + 255) / 256, 1024), nsys);
        if (ext && !b->d_c0) TDSEZ_HIP_TRY(hipMalloc(&b->d_c0, 2 * sizeof(double) * (size_t)b->state_elems));
        pack_state_kernel<<<grid, 256, 0, stream>>>(b->d_desc, psi, b->d_state, ext ? b->d_c0 : nullptr);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    KernelArgs ka{};
    ka.descs = b->d_desc;
    ka.order = b->d_order;
    ka.order_off = 0;
    ka.band64 = b->d_band64;
    ka.bandlo = b->d_bandlo;
    ka.st = b->d_state;
    ka.dtot = b->d_dtot;
    ka.rhs = b->d_rhs;
    ka.fac = b->d_fac;
    ka.red = b->d_red;
    ka.E = E;
    ka.obs = obs;
    ka.mask = obs_mask;
    ka.norm_tol = b->norm_tol;
    ka.status = b->d_status;
    ka.prof = b->d_prof;
    ka.refine_tol = b->refine_tol;
    ka.c0 = ext ? b->d_c0 : nullptr;
    ka.proj = b->d_proj;
    ka.ext = ext;
    // the extended kernels: an absorber in some system, the extended series,
    // or the a_Q part of a requested acceleration
    const bool xt = b->any_cap || ext != nullptr || (b->any_aq && (obs_mask & TDSEZ_OBS_ACCEL));
    const bool fp64 = prec == TDSEZ_FP64;
    ka.band = fp64 ? (const void*)b->d_band64 : (const void*)b->d_band32;
    ka.refine = fp64 ? 0 : b->refine;
    if (b->span_G > 1) {
        // one system on span_G cooperative workgroups
        if (xt) return fail(TDSEZ_EUNSUPPORTED,
                            "the extended kernels run on one workgroup: tdsez_system_set(sys, \"workgroups\", 1)");
        const int G = b->span_G, p = b->plan[0].p, ns = b->desc[0].nsteps;
        const size_t xch_b = 2 * sizeof(double) * (size_t)(2 * G * xch_entry(p));
        const size_t gfac_b = 2 * sizeof(double) * (size_t)((long long)G * (G + 1) * gfac_entry(p));
        if (!b->d_xch) {
            TDSEZ_HIP_TRY(hipMalloc(&b->d_xch, xch_b));
            TDSEZ_HIP_TRY(hipMalloc(&b->d_gfac, gfac_b));
        }
        const long long need = 3LL * (ns + 1) * G;
        if (need > b->obs_part_elems) {
            (void)hipFree(b->d_obs_part);
            b->d_obs_part = nullptr;
            b->obs_part_elems = 0;
            TDSEZ_HIP_TRY(hipMalloc(&b->d_obs_part, sizeof(double) * (size_t)need));
            b->obs_part_elems = need;
        }
        ka.xch = b->d_xch;
        ka.gfac = b->d_gfac;
        ka.obs_part = b->d_obs_part;
        TDSEZ_HIP_TRY(fp64 ? launch_prop_f64_span(ka, G, stream) : launch_prop_f32_span(ka, G, stream));
        span_sum_kernel<<<1, 256, 0, stream>>>(b->d_obs_part, G, ns, obs, obs_mask, b->d_status);
        TDSEZ_HIP_TRY(hipGetLastError());
        dim3 grid((unsigned)std::min<long long>((maxN + 255) / 256, 1024), nsys);
        unpack_state_kernel<<<grid, 256, 0, stream>>>(b->d_desc, b->d_state, psi);
        TDSEZ_HIP_TRY(hipGetLastError());
        return TDSEZ_OK;
    }
    // Multi-wave systems (the costliest of the batch) are launched first,
    // the first group on the caller's stream; the other groups run
    // concurrently on side streams forked from and joined back into the
    // caller's stream (all streams at the default priority).
    const int n4 = b->n4, n2 = b->nsplit - b->n4, n1 = nsys - b->nsplit;
    hipStream_t grp[3] = {stream, stream, stream};  // streams of the 4-, 2- and 1-wave launches
    hipStream_t sides[2] = {b->side, b->side2};
    hipEvent_t joins[2] = {b->ev_join, b->ev_join2};
    int nside = 0;
    {
        const int cnt[3] = {n4, n2, n1};
        bool first = true;
        for (int g = 0; g < 3; ++g) {
            if (cnt[g] == 0) continue;
            if (first) {
                first = false;
                continue;
            }
            if (nside == 0) TDSEZ_HIP_TRY(hipEventRecord(b->ev_fork, stream));
            TDSEZ_HIP_TRY(hipStreamWaitEvent(sides[nside], b->ev_fork, 0));
            grp[g] = sides[nside++];
        }
    }
    hipError_t le;
    if (xt) le = fp64 ? launch_prop_xt64(ka, n4, n2, n1, grp[0], grp[1], grp[2])
                      : launch_prop_xt32(ka, n4, n2, n1, grp[0], grp[1], grp[2]);
    else le = fp64 ? launch_prop_f64(ka, n4, n2, n1, grp[0], grp[1], grp[2], probe)
                   : launch_prop_f32(ka, n4, n2, n1, grp[0], grp[1], grp[2], probe);
    TDSEZ_HIP_TRY(le);
    for (int k = 0; k < nside; ++k) {
        TDSEZ_HIP_TRY(hipEventRecord(joins[k], sides[k]));
        TDSEZ_HIP_TRY(hipStreamWaitEvent(stream, joins[k], 0));
    }
    {
        dim3 grid((unsigned)std::min<long long>((maxN + 255) / 256, 1024), nsys);
        unpack_state_kernel<<<grid, 256, 0, stream>>>(b->d_desc, b->d_state, psi);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    return TDSEZ_OK;
}

}  // namespace tdsez

// ---------------------------------------------------------------- no-alloc
// tdsez_propagate_noalloc: the single-system propagation with every working
// buffer in one file-scope device array, for callers that cannot allocate.
namespace tdsez {
namespace {

constexpr size_t kNoallocBytes = size_t(64) << 20;
// The array's name is a host-side stand-in in host code: kernels get the
// per-device address from hipGetSymbolAddress (g_noalloc_ptr), never the name.
__device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {nullptr};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// descriptor, workgroup order and cleared status, from kernel arguments (no
// host buffer outlives the call)
__global__ void noalloc_setup_kernel(SysDesc d, SysDesc* __restrict__ desc, int* __restrict__ order,
                                     int* __restrict__ status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *desc = d;
        order[0] = 0;
        for (int i = 0; i < 4; ++i) status[i] = 0;
    }
}

}  // namespace
}  // namespace tdsez

extern "C" tdsez_status tdsez_propagate_noalloc(tdsez_system sys_h, double* psi, const double* E, double dt,
                                                int nsteps, tdsez_precision prec, unsigned obs, double* obs_out,
                                                int* dev_status, void* stream_v) {
    using namespace tdsez;
    if (!sys_h || !psi || !E) return fail(TDSEZ_EINVAL, "NULL argument");
    SystemData* sy = &sys_h->d;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TDSEZ_EINVAL, "dt must be > 0");
    if (nsteps < 0) return fail(TDSEZ_EINVAL, "nsteps < 0");
    if (prec != TDSEZ_FP64 && prec != TDSEZ_FP32_REFINED) return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    if (obs & ~7u) return fail(TDSEZ_EINVAL, "unknown observable bits 0x%x", obs);
    if (obs && !obs_out) return fail(TDSEZ_EINVAL, "obs requested but obs_out is NULL");
    if (sy->d_W || sy->d_Q) return fail(TDSEZ_EUNSUPPORTED, "no-alloc propagation: no absorber or a_Q form");
    if ((obs & TDSEZ_OBS_ACCEL) && !sy->const_mass)
        return fail(TDSEZ_EUNSUPPORTED, "position-dependent mass: the acceleration needs the a_Q form");
    // the one-workgroup plan of tdsez_propagate (up to four waves; no spanning)
    const Plan pl = lone_plan(sy->N, sy->p);
    const int nw = plan_waves(pl);
    // scratch layout
    const long long nband = (long long)pl.L * kNumMats * (pl.p + 1) * pl.LS;
    const long long nstate = (long long)pl.L * pl.LS;
    const long long nfac = (long long)pl.m * fac_items(pl.p) * pl.P;
    const long long nred = RedLayout<double>::total(pl.p, pl.P);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    const size_t o_desc = take(sizeof(SysDesc)), o_order = take(sizeof(int)), o_status = take(4 * sizeof(int));
    const size_t o_b64 = take(sizeof(double) * nband), o_b32 = take(sizeof(float) * nband);
    const size_t o_st = take(2 * sizeof(double) * nstate), o_dtot = take(2 * sizeof(double) * nstate);
    const size_t o_rhs = take(2 * sizeof(double) * nstate), o_fac = take(2 * sizeof(double) * (nfac > 0 ? nfac : 1));
    const size_t o_red = take(2 * sizeof(double) * nred);
    const size_t o_lo = take(sizeof(unsigned long long) * 3 * nstate);
    if (off > kNoallocBytes)
        return fail(TDSEZ_EINVAL, "no-alloc propagation: N = %d needs %zu bytes of scratch, the limit is %zu", sy->N,
                    off, kNoallocBytes);
    int dev = 0;
    TDSEZ_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TDSEZ_EUNSUPPORTED, "device index %d", dev);
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            void* p = nullptr;
            TDSEZ_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            g_noalloc_ptr[dev] = p;
        }
        base = static_cast<unsigned char*>(g_noalloc_ptr[dev]);
    }
    hipStream_t stream = (hipStream_t)stream_v;
    SysDesc d{};
    d.N = pl.N; d.p = pl.p; d.P = pl.P; d.L = pl.L; d.m = pl.m; d.LS = pl.LS;
    d.nsteps = nsteps;
    d.dt = dt;
    d.mi_is_s = sy->const_mass ? 1 : 0;
    SysDesc* ddesc = reinterpret_cast<SysDesc*>(base + o_desc);
    int* dorder = reinterpret_cast<int*>(base + o_order);
    int* dstatus = dev_status ? dev_status : reinterpret_cast<int*>(base + o_status);
    double* b64 = reinterpret_cast<double*>(base + o_b64);
    float* b32 = reinterpret_cast<float*>(base + o_b32);
    unsigned long long* lo = reinterpret_cast<unsigned long long*>(base + o_lo);
    double* st = reinterpret_cast<double*>(base + o_st);
    noalloc_setup_kernel<<<1, 64, 0, stream>>>(d, ddesc, dorder, dstatus);
    TDSEZ_HIP_TRY(hipGetLastError());
    {
        BandSrc src;
        src.m[kMatS] = sy->d_band[0];
        src.m[kMatH0] = sy->d_H0;
        src.m[kMatD] = sy->d_band[3];
        src.m[kMatG] = sy->d_band[4];
        src.m[kMatMi] = sy->d_band[5];
        src.m[kMatW] = nullptr;
        src.m[kMatV] = sy->d_band[2];
        src.m[kMatK] = sy->d_K;
        src.m[kMatQ] = nullptr;
        const int nb = (int)std::min<long long>((nband + 255) / 256, 4096);
        pack_band_kernel<<<nb, 256, 0, stream>>>(src, pl.N, pl.p, pl.P, pl.L, pl.LS, b64, b32);
        TDSEZ_HIP_TRY(hipGetLastError());
        pack_lo_kernel<<<(int)std::min<long long>((3 * nstate + 255) / 256, 4096), 256, 0, stream>>>(
            b64, pl.p, pl.L, pl.LS, lo);
        TDSEZ_HIP_TRY(hipGetLastError());
        dim3 grid((unsigned)std::min<long long>((nstate + 255) / 256, 1024), 1);
        pack_state_kernel<<<grid, 256, 0, stream>>>(ddesc, psi, st, nullptr);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    KernelArgs ka{};
    ka.descs = ddesc;
    ka.order = dorder;
    ka.order_off = 0;
    ka.band64 = b64;
    ka.bandlo = lo;
    ka.st = st;
    ka.dtot = reinterpret_cast<double*>(base + o_dtot);
    ka.rhs = base + o_rhs;
    ka.fac = base + o_fac;
    ka.red = base + o_red;
    ka.E = E;
    ka.obs = obs ? obs_out : nullptr;
    ka.mask = obs;
    ka.norm_tol = 0.0;
    ka.status = dstatus;
    ka.prof = nullptr;
    ka.refine_tol = 1e-2;
    ka.c0 = nullptr;
    ka.proj = nullptr;
    ka.ext = nullptr;
    const bool fp64 = prec == TDSEZ_FP64;
    ka.band = fp64 ? (const void*)b64 : (const void*)b32;
    ka.refine = fp64 ? 0 : 1;
    const int n4 = nw == 4 ? 1 : 0, n2 = nw == 2 ? 1 : 0, n1 = nw == 1 ? 1 : 0;
    TDSEZ_HIP_TRY(fp64 ? launch_prop_f64(ka, n4, n2, n1, stream, stream, stream, false)
                       : launch_prop_f32(ka, n4, n2, n1, stream, stream, stream, false));
    {
        dim3 grid((unsigned)std::min<long long>(((long long)pl.N + 255) / 256, 1024), 1);
        unpack_state_kernel<<<grid, 256, 0, stream>>>(ddesc, st, psi);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    return TDSEZ_OK;
}
