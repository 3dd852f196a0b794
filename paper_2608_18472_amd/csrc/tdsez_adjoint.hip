// Discrete adjoint of the batched Crank-Nicolson propagation (gradients of a
// function J of the observable series with respect to the field samples and
// the initial state).
//
// The forward recursion is A_n c_{n+1} = B_n c_n with A_n = S + i a H_n,
// B_n = S - i a H_n = conj(A_n), H_n = H0 + Ebar_n D, a = dt/2,
// Ebar_n = (E_n + E_{n+1})/2 (section V.B).  For J(nu, d, a-series) the
// adjoint recursion, run backwards from lambda_N = g_N, is
//   z_n = B_n^-1 lambda_{n+1} = conj(A_n^-1 conj(lambda_{n+1}))
//   lambda_n = g_n + A_n z_n
//   dJ/dEbar_n = a Im(z_n^H D (c_n + c_{n+1}))
//   g_n = 2 dJ/dnu_n S c_n + 2 dJ/dd_n D c_n - 2 dJ/da_n (G c_n + E_n Mi c_n)
//   dJ/dE_n = (dJ/dEbar_{n-1} + dJ/dEbar_n)/2 - dJ/da_n c_n^H Mi c_n
// and dJ/dpsi0 = lambda_0.  The solve with B_n reuses the partitioned
// factorisation of A_n on the conjugated right-hand side.
//
// States are not stored for every step: a first forward sweep keeps every
// ck-th state (ck ~ sqrt(nsteps)); each segment between two checkpoints is
// recomputed into a segment buffer before its adjoint steps run.  The
// recomputation keeps every step's factorisation of A_n (factor rows and
// separator factors, one slot per step of the segment), so an adjoint step
// only substitutes: forward with the stored rows, the separator solve, back
// substitution.  The cost is about two forward propagations and a half; the
// memory (nsteps/ck + ck + 1) states and ck factorisations per system (each
// 16 (2p + 2) bytes per row of factor rows and 16 (6p^2 + 4p) bytes per
// chunk of separator data).  Everything
// runs in FP64, one
// wave per system, or two or four for the systems marked by
// tdsez_batch_split (their separator system solved from both ends, or by
// block cyclic reduction), all systems of one workgroup size in one launch.
#include <algorithm>
#include <cmath>

#include "tdsez_passes.hpp"

namespace tdsez {

namespace {

struct AdjArgs {
    const SysDesc* descs;
    const int* order;     // workgroup -> system index (longest first)
    const double* band;   // FP64 bands
    double* st;           // working state (interleaved)
    double* rhs;          // right-hand side of the forward steps
    double* fac;
    double* red;
    double* lam;          // lambda_{n+1} / lambda_n (interleaved)
    double* wsol;         // A_n^-1 conj(lambda_{n+1}) (interleaved, zero halos)
    double* ckpt;
    double* seg;
    const double* psi0;   // caller's initial states (natural order)
    const double* E;
    const double* dJdobs; // [n*3 + 0..2] per system, at obs_off
    unsigned mask;
    double* dJdE;         // per system at E_off
    double* dJdpsi0;      // per system at psi_off, or nullptr
    int* status;
    long long state_total;  // complex elements of one whole-batch state
    int order_off;          // first entry of order read by this launch
    long long fac_total;    // complex elements of one slot of fac (whole batch)
    long long red_total;    // complex elements of one slot of red (whole batch)
};

// copy the system's interleaved state (L x LS complex, at state_off of a
// batch-layout buffer) with lane k owning column k+1 and the first/last lane
// also copying the zero halo columns
__device__ __forceinline__ void copy_state(const SysDesc& sd, int lane, const double* src, double* dst) {
    if (lane >= sd.P) return;
    const int LS = sd.LS;
    // the lane's own column, eight rows in flight at a time (the stores of a
    // row would otherwise wait for its loads one row after the other)
    constexpr int kRows = 8;
    for (int l0 = 0; l0 < sd.L; l0 += kRows) {
        double re[kRows], im[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int l = l0 + u < sd.L ? l0 + u : sd.L - 1;
            const long long at = sd.state_off + (long long)l * LS + lane + 1;
            re[u] = src[2 * at];
            im[u] = src[2 * at + 1];
        }
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            if (l0 + u < sd.L) {
                const long long at = sd.state_off + (long long)(l0 + u) * LS + lane + 1;
                dst[2 * at] = re[u];
                dst[2 * at + 1] = im[u];
            }
        }
    }
    // the zero halo columns 0 (first lane) and P + 1 (last lane; one lane
    // copies both when P = 1)
    for (int h = 0; h < 2; ++h) {
        if (!(h == 0 ? lane == 0 : lane == sd.P - 1)) continue;
        const int hc = h == 0 ? 0 : sd.P + 1;
        for (int l = 0; l < sd.L; ++l) {
            const long long at = sd.state_off + (long long)l * LS + hc;
            dst[2 * at] = src[2 * at];
            dst[2 * at + 1] = src[2 * at + 1];
        }
    }
}

// Update pass of adjoint step n (lane-serial over chunk k, rows 0..L-1 and a
// halo of p rows of the next chunk):
//   lambda_n = A_n z + g_n         (z = conj(wsol); z = 0 when !has_z)
//   part[0] = sum Im(conj(z_r) (D v)_r), v = c_n + c_{n+1}
//   part[1] = c_n^H Mi c_n
// Band products use the scatter/gather split of the right-hand-side pass;
// pairs (r, r-d) of the two reductions are counted by the owner of row r.
template <int PP>
__device__ __forceinline__ void pass_adjoint_update(const SysDesc& sd, int k, const double* __restrict__ band,
                                    const double* __restrict__ wsol, const double* __restrict__ cn,
                                    const double* __restrict__ cn1, double* __restrict__ lam,
                                    bool has_z, double alpha, double Ebar, double En, double jn,
                                    double jd, double ja, double part[2]) {
    constexpr int NM = kNumMats;
    const int L = sd.L, LS = sd.LS;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const double* __restrict__ bnd = band + sd.band_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
    const double* __restrict__ ws = wsol + 2 * sd.state_off;
    const double* __restrict__ c0 = cn + 2 * sd.state_off;
    const double* __restrict__ c1 = has_z ? cn1 + 2 * sd.state_off : nullptr;
    double* __restrict__ lm = lam + 2 * sd.state_off;

    cplx<double> zw[PP + 1], cw[PP + 1], vw[PP + 1];  // rows r-p..r, slot PP newest
    cplx<double> az[PP + 1], kc[PP + 1];               // pending (A z), (K c) of rows r-p..r
    auto load3 = [&](unsigned at, cplx<double>& z, cplx<double>& c, cplx<double>& v) {
        c = cmk<double>(c0[2 * at], c0[2 * at + 1]);
        z = cmk<double>(0, 0);
        v = c;
        if (has_z) {
            z = cmk<double>(ws[2 * at], -ws[2 * at + 1]);
            v = cmk<double>(c.re + c1[2 * at], c.im + c1[2 * at + 1]);
        }
    };
#pragma unroll
    for (int i = 0; i <= PP; ++i) {
        az[i] = cmk<double>(0, 0);
        kc[i] = cmk<double>(0, 0);
    }
    zw[0] = cw[0] = vw[0] = cmk<double>(0, 0);
#pragma unroll
    for (int d = 0; d < PP; ++d) {
        const unsigned at = (unsigned)(L - PP + d) * (unsigned)LS + (unsigned)(col - 1);
        load3(at, zw[d + 1], cw[d + 1], vw[d + 1]);
    }
    double dimag = 0.0, mexp = 0.0;
    // band and state rows, loaded one row ahead of their use
    struct RowIn {
        double s[PP + 1], h[PP + 1], d[PP + 1], g[PP + 1], m[PP + 1];
        cplx<double> z, c, v;
    };
    auto load_row = [&](int r) {
        if (r >= L + PP) r = L + PP - 1;  // past the end: reload the last row (unused)
        const bool own = r < L;
        const int lr = own ? r : r - L;
        const unsigned cc = (unsigned)(own ? col : col + 1);
        const unsigned rb = (unsigned)lr * rowstride + cc;
        RowIn in;
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            in.s[d] = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
            in.h[d] = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
            in.d[d] = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
            in.g[d] = bnd[rb + (unsigned)((3 * (PP + 1) + d) * LS)];
            in.m[d] = bnd[rb + (unsigned)((4 * (PP + 1) + d) * LS)];
        }
        load3((unsigned)lr * (unsigned)LS + cc, in.z, in.c, in.v);
        return in;
    };
    auto stream_row = [&](const RowIn& in, int r, bool own) {
        cplx<double> a[PP + 1];
        double kk[PP + 1], dd[PP + 1], mi[PP + 1];
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            const double s = in.s[d];
            const double h = in.h[d];
            dd[d] = in.d[d];
            const double g = in.g[d];
            mi[d] = in.m[d];
            a[d] = cmk<double>(s, alpha * (h + Ebar * dd[d]));
            kk[d] = 2.0 * jn * s + 2.0 * jd * dd[d] - 2.0 * ja * (g + En * mi[d]);
        }
        const cplx<double> zr = in.z, cr = in.c, vr = in.v;
#pragma unroll
        for (int d = 0; d < PP; ++d) {
            zw[d] = zw[d + 1];
            cw[d] = cw[d + 1];
            vw[d] = vw[d + 1];
            az[d] = az[d + 1];
            kc[d] = kc[d + 1];
        }
        zw[PP] = zr;
        cw[PP] = cr;
        vw[PP] = vr;
        cplx<double> sa = cmk<double>(0, 0), sk = cmk<double>(0, 0);
        if (own) {
#pragma unroll
            for (int d = 0; d <= PP; ++d) {
                sa = cfma(sa, a[d], zw[PP - d]);
                sk.re += kk[d] * cw[PP - d].re;
                sk.im += kk[d] * cw[PP - d].im;
            }
            // reductions over the pairs (r, r - d)
            double di = dd[0] * (zr.re * vr.im - zr.im * vr.re);
            double me = mi[0] * (cr.re * cr.re + cr.im * cr.im);
#pragma unroll
            for (int d = 1; d <= PP; ++d) {
                // Im(conj(z_r) v_{r-d} + conj(z_{r-d}) v_r)
                di += dd[d] * (zr.re * vw[PP - d].im - zr.im * vw[PP - d].re + zw[PP - d].re * vr.im -
                               zw[PP - d].im * vr.re);
                me += 2.0 * mi[d] * (cr.re * cw[PP - d].re + cr.im * cw[PP - d].im);
            }
            dimag += di;
            mexp += me;
        }
        az[PP] = sa;
        kc[PP] = sk;
#pragma unroll
        for (int d = 1; d <= PP; ++d) {
            az[PP - d] = cfma(az[PP - d], a[d], zr);
            kc[PP - d].re += kk[d] * cr.re;
            kc[PP - d].im += kk[d] * cr.im;
        }
        if (r >= PP) {
            const unsigned o = (unsigned)(r - PP) * (unsigned)LS + (unsigned)col;
            lm[2 * o] = az[0].re + kc[0].re;
            lm[2 * o + 1] = az[0].im + kc[0].im;
        }
    };
    RowIn cur = load_row(0);
    for (int r = 0; r < L; ++r) {
        const RowIn nxt = load_row(r + 1);
        stream_row(cur, r, true);
        cur = nxt;
    }
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        const RowIn nxt = load_row(L + t + 1);
        stream_row(cur, L + t, false);
        cur = nxt;
    }
    part[0] = dimag;
    part[1] = mexp;
}

// Forward substitution of conj(b) (b in state layout) with the factor rows
// stored by the factorisation of A_n (passes A1/A2 of the segment's forward
// step): yhat_j of every interior pivot, and the separator rows' right-hand
// side yR and the left separator's Schur right-hand side gT of the chunk, as
// passes A1 and A2 form them for a new right-hand side.
template <int PP>
__device__ __forceinline__ void pass_fwdsub_conj(const SysDesc& sd, int k, const double* __restrict__ rhs,
                                                 double* __restrict__ fac, double* __restrict__ red) {
    constexpr int IT = 2 * PP + 2;
    const int L = sd.L, LS = sd.LS, P = sd.P, m = sd.m;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const int kk = col - 1;
    const double* __restrict__ rs = rhs + 2 * sd.state_off;
    double* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned fstride = (unsigned)(IT * P);
    auto fitem = [&](int j, int item) {
        return ld_c(fc, (unsigned)j * fstride + (unsigned)(item * P) + (unsigned)kk);
    };
    auto b_of = [&](int r) {
        const cplx<double> v = ld_c(rs, (unsigned)r * (unsigned)LS + (unsigned)col);
        return cmk<double>(v.re, -v.im);
    };
    struct FRow {
        cplx<double> l[PP], dinv, f[PP];
    };
    auto load_frow = [&](int j) {
        if (j > m - 1) j = m - 1;
        FRow fr;
#pragma unroll
        for (int i = 0; i < PP; ++i) fr.l[i] = fitem(j, i);
        fr.dinv = fitem(j, PP);
#pragma unroll
        for (int t = 0; t < PP; ++t) fr.f[t] = fitem(j, PP + 2 + t);
        return fr;
    };
    cplx<double> y[PP + 1], gT[PP];
#pragma unroll
    for (int i = 0; i <= PP; ++i) y[i] = cmk<double>(0, 0);
#pragma unroll
    for (int t = 0; t < PP; ++t) gT[t] = cmk<double>(0, 0);
    FRow fcur = load_frow(0);
    cplx<double> bcur = b_of(0);
    for (int j = 0; j < m; ++j) {
        const FRow fnxt = load_frow(j + 1);
        const cplx<double> bnxt = b_of(j + 1 < L ? j + 1 : L - 1);
        const cplx<double> yj = cadd(y[0], bcur);
        st_c(fc, (unsigned)j * fstride + (unsigned)((PP + 1) * P) + (unsigned)kk, yj);
#pragma unroll
        for (int i = 1; i <= PP; ++i) y[i] = cfms(y[i], fcur.l[i - 1], yj);
#pragma unroll
        for (int t = 0; t < PP; ++t) gT[t] = cfms(gT[t], cmul(fcur.f[t], fcur.dinv), yj);
#pragma unroll
        for (int i = 1; i <= PP; ++i) y[i - 1] = y[i];
        y[PP] = cmk<double>(0, 0);
        fcur = fnxt;
        bcur = bnxt;
    }
    // the separator rows m .. L-1 of the chunk
#pragma unroll
    for (int t = 0; t < PP; ++t) y[t] = cadd(y[t], b_of(m + t));
    double* rb = red + 2 * (sd.red_off + (long long)k * RedLayout<double>::chunk_block(PP));
    constexpr int pp = PP * PP;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        st_c(rb, (unsigned)(3 * pp + i), y[i]);
        st_c(rb, (unsigned)(3 * pp + PP + i), gT[i]);
    }
}

template <int PP, int NW>
__device__ __forceinline__ void adj_reduced(const SysDesc& sd, int tid, double* red, double* zl, bool factor) {
    if constexpr (NW == 4) {
        const SpanCtx<double> one{0, sd.P, 0, 1, nullptr, nullptr};  // one workgroup
        pass_reduced_cr<PP, double, 4, false>(sd, tid, red, factor, zl, one);
    } else if constexpr (NW == 2) {
        pass_reduced2<PP, double>(sd, tid, red, factor, zl);
    } else {
        pass_reduced<PP, double>(sd, tid, red, factor, zl);
    }
}

// sum over the workgroup of wave-uniform values (wave order, so every wave
// gets the same bits)
template <int NW>
__device__ __forceinline__ double wg_sum(double v, int tid) {
    v = wave_sum(v);
    if constexpr (NW > 1) {
        __shared__ double buf[NW];
        if ((tid & (kWave - 1)) == 0) buf[tid / kWave] = v;
        __syncthreads();
        v = buf[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) v += buf[w];
        __syncthreads();
    }
    return v;
}

// one forward step n -> n+1 in place on st (FP64, no refinement); the
// factorisation of A_n is left in the factor slot (fac, red)
template <int PP, int NW>
__device__ __forceinline__ void forward_step(const AdjArgs& ka, const SysDesc& sd, int lane, double alpha, double Ebar,
                                             double* zl, double* fac, double* red) {
    const bool active = lane < sd.P;
    double part[3];
    if (active) {
        pass_rhs<PP, double>(sd, lane, ka.band, ka.st, ka.rhs, alpha, Ebar, Ebar, false, true, part);
        pass_elim<PP, double>(sd, lane, ka.band, ka.rhs, fac, red, alpha, Ebar);
        pass_fill<PP, double, false>(sd, lane, ka.band, fac, red, alpha, Ebar);
        pass_schur<PP, double>(sd, lane, fac, red);
    }
    __syncthreads();
    adj_reduced<PP, NW>(sd, lane, red, zl, true);
    __syncthreads();
    if (active) pass_backsub<PP, double>(sd, lane, ka.band, ka.st, nullptr, true, fac, red, alpha, Ebar);
    __syncthreads();
}

template <int PP, int NW>
__device__ __forceinline__ void run_adjoint(const AdjArgs& ka, const SysDesc& sd, int sidx, double* zl) {
    const int lane = threadIdx.x;
    const bool active = lane < sd.P;
    const int N = sd.N, L = sd.L, LS = sd.LS, ns = sd.nsteps, ck = sd.ck;
    const double alpha = 0.5 * sd.dt;
    const double* Es = ka.E + sd.E_off;
    const double* jo = ka.dJdobs + sd.obs_off;
    double* gE = ka.dJdE + sd.E_off;
    double* ckpt = ka.ckpt;
    double* seg = ka.seg;
    const bool use_n = (ka.mask & TDSEZ_OBS_NORM) != 0;
    const bool use_d = (ka.mask & TDSEZ_OBS_DIPOLE) != 0;
    const bool use_a = (ka.mask & TDSEZ_OBS_ACCEL) != 0;
    auto jn = [&](int n) { return use_n ? jo[3 * n + 0] : 0.0; };
    auto jd = [&](int n) { return use_d ? jo[3 * n + 1] : 0.0; };
    auto ja = [&](int n) { return use_a ? jo[3 * n + 2] : 0.0; };
    auto ebar = [&](int n) { return 0.5 * (Es[n] + Es[n + 1]); };
    // checkpoint and segment buffers hold whole-batch states (the system's
    // part at state_off, like the working state)
    auto state_at = [&](double* base, long long idx) { return base + 2 * (idx * ka.state_total); };
    // factor slot of step n0 + t of the segment being reversed (whole-batch
    // fac and red layouts, the system's part at fac_off / red_off)
    auto fac_slot = [&](int t) { return ka.fac + 2 * ((long long)t * ka.fac_total); };
    auto red_slot = [&](int t) { return ka.red + 2 * ((long long)t * ka.red_total); };

    // initial state: natural order -> interleaved, zero halos and padding
    if (active) {
        for (int l = 0; l < L; ++l) {
            const long long row = (long long)lane * L + l;
            const long long at = sd.state_off + (long long)l * LS + lane + 1;
            double re = 0.0, im = 0.0;
            if (row < N) {
                re = ka.psi0[2 * (sd.psi_off + row)];
                im = ka.psi0[2 * (sd.psi_off + row) + 1];
            }
            ka.st[2 * at] = re;
            ka.st[2 * at + 1] = im;
            if (lane == 0) {
                const long long h = sd.state_off + (long long)l * LS;
                ka.st[2 * h] = ka.st[2 * h + 1] = 0.0;
            }
            if (lane == sd.P - 1) {
                const long long h = sd.state_off + (long long)l * LS + sd.P + 1;
                ka.st[2 * h] = ka.st[2 * h + 1] = 0.0;
            }
        }
    }
    for (int n = lane; n <= ns; n += NW * kWave) gE[n] = 0.0;
    __syncthreads();
    // forward sweep keeping checkpoints 0, ck, 2 ck, ...
    copy_state(sd, lane, ka.st, state_at(ckpt, 0));
    __syncthreads();
    for (int n = 0; n < ns; ++n) {
        forward_step<PP, NW>(ka, sd, lane, alpha, ebar(n), zl, fac_slot(0), red_slot(0));
        if ((n + 1) % ck == 0 && n + 1 < ns) {
            copy_state(sd, lane, ka.st, state_at(ckpt, (n + 1) / ck));
            __syncthreads();
        }
    }
    // lambda_N = g_N and the direct field term of step N
    {
        double part[2] = {0.0, 0.0};
        if (active)
            pass_adjoint_update<PP>(sd, lane, ka.band, ka.wsol, ka.st, nullptr, ka.lam, false, alpha, Es[ns],
                                    Es[ns], jn(ns), jd(ns), ja(ns), part);
        const double me = wg_sum<NW>(part[1], lane);
        if (lane == 0) gE[ns] -= ja(ns) * me;
        __syncthreads();
    }
    for (int sgi = sd.nseg - 1; sgi >= 0; --sgi) {
        const int n0 = sgi * ck;
        const int n1 = n0 + ck < ns ? n0 + ck : ns;
        // recompute c_{n0} .. c_{n1} into the segment buffer
        copy_state(sd, lane, state_at(ckpt, sgi), ka.st);
        copy_state(sd, lane, state_at(ckpt, sgi), state_at(seg, 0));
        __syncthreads();
        for (int n = n0; n < n1; ++n) {
            forward_step<PP, NW>(ka, sd, lane, alpha, ebar(n), zl, fac_slot(n - n0), red_slot(n - n0));
            copy_state(sd, lane, ka.st, state_at(seg, n - n0 + 1));
            __syncthreads();
        }
        for (int n = n1 - 1; n >= n0; --n) {
            const double Eb = ebar(n);
            // w = A_n^-1 conj(lambda_{n+1}) with the factorisation of A_n kept
            // by the recomputation of step n
            double* fs = fac_slot(n - n0);
            double* rs = red_slot(n - n0);
            if (active) pass_fwdsub_conj<PP>(sd, lane, ka.lam, fs, rs);
            __syncthreads();
            adj_reduced<PP, NW>(sd, lane, rs, zl, false);
            __syncthreads();
            if (active) pass_backsub<PP, double>(sd, lane, ka.band, ka.wsol, nullptr, true, fs, rs, alpha, Eb, true);
            __syncthreads();
            // lambda_n = g_n + A_n z, z = conj(w)
            double part[2] = {0.0, 0.0};
            if (active)
                pass_adjoint_update<PP>(sd, lane, ka.band, ka.wsol, state_at(seg, n - n0),
                                        state_at(seg, n - n0 + 1), ka.lam, true, alpha, Eb, Es[n], jn(n),
                                        jd(n), ja(n), part);
            const double di = wg_sum<NW>(part[0], lane);
            const double me = wg_sum<NW>(part[1], lane);
            if (!isfinite(di) || !isfinite(me)) {
                if (lane == 0) latch(ka.status, TDSEZ_ENONFINITE, sidx, n);
                return;
            }
            if (lane == 0) {
                const double dEb = alpha * di;
                gE[n] += 0.5 * dEb - ja(n) * me;
                gE[n + 1] += 0.5 * dEb;
            }
            __syncthreads();
        }
    }
    // dJ/dpsi0 = lambda_0
    if (ka.dJdpsi0 && active) {
        const double* lm = ka.lam + 2 * sd.state_off;
        for (int l = 0; l < L; ++l) {
            const long long row = (long long)lane * L + l;
            if (row >= N) break;
            const long long at = (long long)l * LS + lane + 1;
            ka.dJdpsi0[2 * (sd.psi_off + row)] = lm[2 * at];
            ka.dJdpsi0[2 * (sd.psi_off + row) + 1] = lm[2 * at + 1];
        }
    }
}

template <int NW>
__device__ __forceinline__ void dispatch_adjoint(const AdjArgs& ka) {
    // the separator recurrence's right-hand-side vector (P * p complex)
    // (four waves: the cyclic reduction's g vectors and block staging)
    __shared__ double zl[NW == 4 ? CrLds<double>::kTotal : 2 * kMaxP * kWave * NW];
    const int sidx = ka.order[ka.order_off + blockIdx.x];
    const SysDesc sd = ka.descs[sidx];
    switch (sd.p) {
        case 1: run_adjoint<1, NW>(ka, sd, sidx, zl); break;
        case 2: run_adjoint<2, NW>(ka, sd, sidx, zl); break;
        case 3: run_adjoint<3, NW>(ka, sd, sidx, zl); break;
        case 4: run_adjoint<4, NW>(ka, sd, sidx, zl); break;
        case 5: run_adjoint<5, NW>(ka, sd, sidx, zl); break;
        case 6: run_adjoint<6, NW>(ka, sd, sidx, zl); break;
        case 7: run_adjoint<7, NW>(ka, sd, sidx, zl); break;
        default: break;
    }
}

__global__ __launch_bounds__(kWave) void adjoint_kernel(AdjArgs ka) { dispatch_adjoint<1>(ka); }
__global__ __launch_bounds__(2 * kWave) void adjoint2_kernel(AdjArgs ka) { dispatch_adjoint<2>(ka); }
__global__ __launch_bounds__(4 * kWave) void adjoint4_kernel(AdjArgs ka) { dispatch_adjoint<4>(ka); }

}  // namespace

tdsez_status launch_adjoint(BatchData* b, const double* psi0, const double* E, const double* dJdobs,
                            unsigned obs_mask, double* dJdE, double* dJdpsi0, int ckpt_stride,
                            hipStream_t stream) {
    const int nsys = (int)b->sys.size();
    const long long state_total = b->state_elems;
    int max_nseg = 1, max_ck = 1;
    for (int s = 0; s < nsys; ++s) {
        SysDesc& d = b->desc[s];
        const int ns = d.nsteps;
        int ck = ckpt_stride > 0 ? ckpt_stride : (int)std::ceil(std::sqrt((double)(ns > 0 ? ns : 1)));
        if (ck > ns) ck = ns > 0 ? ns : 1;
        if (ck < 1) ck = 1;
        d.ck = ck;
        d.nseg = ns > 0 ? (ns + ck - 1) / ck : 0;
        max_nseg = std::max(max_nseg, d.nseg);
        max_ck = std::max(max_ck, ck);
    }
    const long long ck_total = (long long)max_nseg * state_total;
    const long long seg_total = (long long)(max_ck + 1) * state_total;
    // one factor slot per step of a segment
    const long long facs_total = (long long)max_ck * b->fac_elems64;
    const long long reds_total = (long long)max_ck * b->red_elems64;
    if (!b->d_lam) {
        TDSEZ_HIP_TRY(hipMalloc(&b->d_lam, 2 * sizeof(double) * (size_t)state_total));
        TDSEZ_HIP_TRY(hipMalloc(&b->d_wsol, 2 * sizeof(double) * (size_t)state_total));
        // halo columns of the solution buffer are read and never written
        TDSEZ_HIP_TRY(hipMemset(b->d_wsol, 0, 2 * sizeof(double) * (size_t)state_total));
    }
    if (ck_total > b->ckpt_elems) {
        (void)hipFree(b->d_ckpt);
        b->d_ckpt = nullptr;
        b->ckpt_elems = 0;
        TDSEZ_HIP_TRY(hipMalloc(&b->d_ckpt, 2 * sizeof(double) * (size_t)ck_total));
        b->ckpt_elems = ck_total;
    }
    if (seg_total > b->seg_elems) {
        (void)hipFree(b->d_seg);
        b->d_seg = nullptr;
        b->seg_elems = 0;
        TDSEZ_HIP_TRY(hipMalloc(&b->d_seg, 2 * sizeof(double) * (size_t)seg_total));
        b->seg_elems = seg_total;
    }
    if (facs_total > b->fac_seg_elems) {
        (void)hipFree(b->d_fac_seg);
        b->d_fac_seg = nullptr;
        b->fac_seg_elems = 0;
        TDSEZ_HIP_TRY(hipMalloc(&b->d_fac_seg, 2 * sizeof(double) * (size_t)facs_total));
        b->fac_seg_elems = facs_total;
    }
    if (reds_total > b->red_seg_elems) {
        (void)hipFree(b->d_red_seg);
        b->d_red_seg = nullptr;
        b->red_seg_elems = 0;
        TDSEZ_HIP_TRY(hipMalloc(&b->d_red_seg, 2 * sizeof(double) * (size_t)reds_total));
        b->red_seg_elems = reds_total;
    }
    if (tdsez_status st = upload_descriptors(b, stream)) return st;
    AdjArgs ka{};
    ka.descs = b->d_desc;
    ka.order = b->d_order;
    ka.band = b->d_band64;
    ka.st = b->d_state;
    ka.rhs = (double*)b->d_rhs;
    ka.fac = b->d_fac_seg;
    ka.red = b->d_red_seg;
    ka.fac_total = b->fac_elems64;
    ka.red_total = b->red_elems64;
    ka.lam = b->d_lam;
    ka.wsol = b->d_wsol;
    ka.ckpt = b->d_ckpt;
    ka.seg = b->d_seg;
    ka.psi0 = psi0;
    ka.E = E;
    ka.dJdobs = dJdobs;
    ka.mask = obs_mask;
    ka.dJdE = dJdE;
    ka.dJdpsi0 = dJdpsi0;
    ka.status = b->d_status;
    ka.state_total = state_total;
    // four-wave systems first (entries 0..n4-1 of the order), then the
    // two-wave and the one-wave systems; the first non-empty group runs on
    // the caller's stream, the others concurrently on the batch's side
    // streams forked from and joined back into it
    const int n4 = b->n4, n2 = b->nsplit - b->n4, n1 = nsys - b->nsplit;
    hipStream_t grp[3] = {stream, stream, stream};
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
    if (n4 > 0) {
        ka.order_off = 0;
        adjoint4_kernel<<<n4, 4 * kWave, 0, grp[0]>>>(ka);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    if (n2 > 0) {
        ka.order_off = n4;
        adjoint2_kernel<<<n2, 2 * kWave, 0, grp[1]>>>(ka);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    if (n1 > 0) {
        ka.order_off = n4 + n2;
        adjoint_kernel<<<n1, kWave, 0, grp[2]>>>(ka);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    for (int k = 0; k < nside; ++k) {
        TDSEZ_HIP_TRY(hipEventRecord(joins[k], sides[k]));
        TDSEZ_HIP_TRY(hipStreamWaitEvent(stream, joins[k], 0));
    }
    return TDSEZ_OK;
}

}  // namespace tdsez
