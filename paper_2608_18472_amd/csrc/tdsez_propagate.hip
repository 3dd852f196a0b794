// Crank-Nicolson propagation kernels (the paper's section V.B, eq. cn_system).
//
// One workgroup (one wave64) per system; every system of a batch runs all
// its time steps inside one persistent launch.  Per step n, with
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
// whole wave solves by block LDL^T with entry-parallel block operations.
// Two more lane-serial sweeps (forward correction for the separator values,
// then back substitution) recover the interior increments.
//
// Layouts (all "interleaved": lane k reads column k+1, so one wave load of a
// given local row is contiguous; columns 0 and P+1 are zero halos):
//   bands  [l][mat][d][col]  mat = S, H0, D, G, Mi; entry M[row][row-d],
//                           row = k*L + l
//   state  [l][col]          complex128
//   factor [j][item][k]      item 0..p-1: L[j+1+i][j], p: 1/D_j, p+1: yhat_j
#include <cmath>

#include "tdsez_internal.hpp"

namespace tdsez {

namespace {

template <typename FT>
struct ReducedIdx {
    // per chunk block: W (p*p), F (p*p), TL (p*p), yR (p), gT (p)
    __host__ __device__ static long long chunk_block(int p) { return 3LL * p * p + 2LL * p; }
    __host__ __device__ static long long total(int p, int P) {
        return (long long)P * (chunk_block(p) + (long long)p * p + 2LL * p);
    }
};

// compile-time switches of one streamed row: insert with left-separator
// fill, shift the window, eliminate a pivot
struct TagFillShift { static constexpr bool fill = true, shift = true; };
struct TagShift { static constexpr bool fill = false, shift = true; };
struct TagNone { static constexpr bool fill = false, shift = false; };
struct NoElim { static constexpr bool elim = false; };
struct Elim { static constexpr bool elim = true; };

__device__ inline double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// complex element idx of an interleaved (re, im) array; per-system indices
// fit in 32 bits, which lets the compiler use SGPR-base + 32-bit offsets
template <typename FT>
__device__ inline cplx<FT> ld_c(const FT* base, unsigned idx) {
    return cplx<FT>{base[2u * idx], base[2u * idx + 1u]};
}
template <typename FT>
__device__ inline void st_c(FT* base, unsigned idx, cplx<FT> v) {
    base[2u * idx] = v.re;
    base[2u * idx + 1u] = v.im;
}

// Pass A: observables of c_n, right-hand side of (1), interior elimination
// and the chunk's Schur contribution.  Lane-serial over the chunk.
template <int PP, typename FT>
__device__ void pass_factor(const SysDesc& sd, int k, const FT* __restrict__ band,
                            const double* __restrict__ st, FT* __restrict__ fac,
                            FT* __restrict__ red, double alpha, double Ebar, double En,
                            bool want_acc, bool do_factor, double obs_part[3]) {
    constexpr int NM = kNumMats;
    const int L = sd.L, m = sd.m, LS = sd.LS, P = sd.P;
    int col = k + 1;
    // Per-lane addresses are rebuilt every step instead of being hoisted out
    // of the time loop (that would keep hundreds of them live in registers).
    asm volatile("" : "+v"(col));
    const FT* __restrict__ bnd = band + sd.band_off;
    const double* __restrict__ cst = st + 2 * sd.state_off;
    FT* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
    const FT a_f = (FT)alpha;
    const FT eb_f = (FT)Ebar;

    cplx<FT> W[PP + 1][PP + 1];
    cplx<FT> F[PP + 1][PP];
    cplx<FT> y[PP + 1];
    cplx<FT> TL[PP][PP];
    cplx<FT> gT[PP];
    cplx<double> cw[PP + 1];
    cplx<double> hacc[PP + 1];
#pragma unroll
    for (int i = 0; i <= PP; ++i) {
#pragma unroll
        for (int j = 0; j <= PP; ++j) W[i][j] = cmk<FT>(0, 0);
#pragma unroll
        for (int t = 0; t < PP; ++t) F[i][t] = cmk<FT>(0, 0);
        y[i] = cmk<FT>(0, 0);
        hacc[i] = cmk<double>(0, 0);
    }
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        gT[t] = cmk<FT>(0, 0);
#pragma unroll
        for (int u = 0; u < PP; ++u) TL[t][u] = cmk<FT>(0, 0);
    }
    // c rows -p..-1 come from the previous chunk (column k; zero for k = 0).
    // The window is shifted before each streamed row, so row -p+d starts in
    // slot d+1 (after the first shift cw[p - d] holds row -d, d = 1..p).
    cw[0] = cmk<double>(0, 0);
#pragma unroll
    for (int d = 0; d < PP; ++d) {
        unsigned at = (unsigned)(L - PP + d) * (unsigned)LS + (unsigned)(col - 1);
        cw[d + 1] = cmk<double>(cst[2 * at], cst[2 * at + 1]);
    }
    double nu = 0.0, dip = 0.0, acc = 0.0;

    // one streamed row: r is the chunk-local row (0 <= r < L + p)
    auto stream_row = [&](int r, bool own, auto insert_tag, auto elim_tag) {
        constexpr bool kInsertFill = decltype(insert_tag)::fill;
        const int lr = own ? r : r - L;
        const unsigned cc = (unsigned)(own ? col : col + 1);
        const unsigned rb = (unsigned)lr * rowstride + cc;
        FT bS[PP + 1], bH[PP + 1], bD[PP + 1];
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            bS[d] = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
            bH[d] = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
            bD[d] = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
        }
        const unsigned sat = (unsigned)lr * (unsigned)LS + cc;
        cplx<double> cr = cmk<double>(cst[2 * sat], cst[2 * sat + 1]);
#pragma unroll
        for (int d = 0; d < PP; ++d) cw[d] = cw[d + 1];
        cw[PP] = cr;
        // H_n row entries in FP64 from the stored band values
        double h[PP + 1];
#pragma unroll
        for (int d = 0; d <= PP; ++d) h[d] = (double)bH[d] + Ebar * (double)bD[d];
        // pending (H_n c) accumulators: hacc[PP - d] is row r - d
#pragma unroll
        for (int d = 0; d < PP; ++d) hacc[d] = hacc[d + 1];
        {
            cplx<double> s = cmk<double>(0, 0);
            if (own) {
#pragma unroll
                for (int d = 0; d <= PP; ++d) {
                    s.re += h[d] * cw[PP - d].re;
                    s.im += h[d] * cw[PP - d].im;
                }
            }
            hacc[PP] = s;
        }
#pragma unroll
        for (int d = 1; d <= PP; ++d) {
            hacc[PP - d].re += h[d] * cr.re;
            hacc[PP - d].im += h[d] * cr.im;
        }
        if (own) {
            // observables: pairs (r, r-d), counted by the owner of the larger row
            double o[PP + 1];
#pragma unroll
            for (int d = 0; d <= PP; ++d) o[d] = cr.re * cw[PP - d].re + cr.im * cw[PP - d].im;
            double sn = (double)bS[0] * o[0], sd_ = (double)bD[0] * o[0];
#pragma unroll
            for (int d = 1; d <= PP; ++d) {
                sn += 2.0 * (double)bS[d] * o[d];
                sd_ += 2.0 * (double)bD[d] * o[d];
            }
            nu += sn;
            dip += sd_;
            if (want_acc) {
                double sg = 0.0, sm = 0.0;
#pragma unroll
                for (int d = 0; d <= PP; ++d) {
                    FT bG = bnd[rb + (unsigned)((3 * (PP + 1) + d) * LS)];
                    FT bM = bnd[rb + (unsigned)((4 * (PP + 1) + d) * LS)];
                    double w = d == 0 ? 1.0 : 2.0;
                    sg += w * (double)bG * o[d];
                    sm += w * (double)bM * o[d];
                }
                acc -= sg + En * sm;
            }
        }
        if (!do_factor) return;
        // complete right-hand side of row r - p: -i dt H_n c = (2a Im, -2a Re)
        cplx<FT> rhs = cmk<FT>((FT)(2.0 * alpha * hacc[0].im), (FT)(-2.0 * alpha * hacc[0].re));
        if (own) {
            // insert row r as window slot PP: A[r][r-d] = S + i a (H0 + Ebar D)
#pragma unroll
            for (int d = 0; d <= PP; ++d) {
                cplx<FT> a = cmk<FT>(bS[d], a_f * (bH[d] + eb_f * bD[d]));
                if (kInsertFill) {
                    if (r - d >= 0) W[PP][PP - d] = a;
                    else F[PP][r - d + PP] = a;  // coupling to the left separator
                } else {
                    W[PP][PP - d] = a;
                }
            }
        }
        if (decltype(elim_tag)::elim) {
            const int j = r - PP;
            y[0] = cadd(y[0], rhs);
            cplx<FT> dinv = cinv(W[0][0]);
            cplx<FT> l[PP + 1];
#pragma unroll
            for (int i = 1; i <= PP; ++i) l[i] = cmul(W[i][0], dinv);
            cplx<FT> f[PP], g[PP];
#pragma unroll
            for (int t = 0; t < PP; ++t) {
                f[t] = F[0][t];
                g[t] = cmul(f[t], dinv);
            }
#pragma unroll
            for (int i = 1; i <= PP; ++i)
#pragma unroll
                for (int i2 = 1; i2 <= i; ++i2) W[i][i2] = cfms(W[i][i2], l[i], W[i2][0]);
#pragma unroll
            for (int i = 1; i <= PP; ++i)
#pragma unroll
                for (int t = 0; t < PP; ++t) F[i][t] = cfms(F[i][t], l[i], f[t]);
#pragma unroll
            for (int t = 0; t < PP; ++t)
#pragma unroll
                for (int u = t; u < PP; ++u) TL[t][u] = cfms(TL[t][u], f[t], g[u]);
            cplx<FT> yj = y[0];
#pragma unroll
            for (int i = 1; i <= PP; ++i) y[i] = cfms(y[i], l[i], yj);
#pragma unroll
            for (int t = 0; t < PP; ++t) gT[t] = cfms(gT[t], g[t], yj);
            // store the factor row of pivot j
            const unsigned fb = (unsigned)j * (unsigned)((PP + 2) * P) + (unsigned)(col - 1);
#pragma unroll
            for (int i = 1; i <= PP; ++i) st_c(fc, fb + (unsigned)((i - 1) * P), l[i]);
            st_c(fc, fb + (unsigned)(PP * P), dinv);
            st_c(fc, fb + (unsigned)((PP + 1) * P), yj);
        }
        if (decltype(insert_tag)::shift) {
#pragma unroll
            for (int i = 1; i <= PP; ++i) {
#pragma unroll
                for (int i2 = 1; i2 <= i; ++i2) W[i - 1][i2 - 1] = W[i][i2];
#pragma unroll
                for (int t = 0; t < PP; ++t) F[i - 1][t] = F[i][t];
                y[i - 1] = y[i];
            }
#pragma unroll
            for (int i2 = 0; i2 <= PP; ++i2) W[PP][i2] = cmk<FT>(0, 0);
#pragma unroll
            for (int t = 0; t < PP; ++t) F[PP][t] = cmk<FT>(0, 0);
            y[PP] = cmk<FT>(0, 0);
        } else {
            // halo rows: right-hand side of separator row r - p -> slot r - L
            // (added by the caller with a compile-time slot)
            (void)rhs;
        }
    };

    // rows 0..p-1: insert (with left-separator fill), no pivot yet
#pragma unroll
    for (int r = 0; r < PP; ++r) stream_row(r, true, TagFillShift{}, NoElim{});
    // rows p..L-1: insert, eliminate pivot r - p, shift
    for (int r = PP; r < L; ++r) stream_row(r, true, TagShift{}, Elim{});
    // halo rows L..L+p-1 of the next chunk complete the separator rows
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        stream_row(L + t, false, TagNone{}, NoElim{});
        if (do_factor) {
            cplx<FT> rhs = cmk<FT>((FT)(2.0 * alpha * hacc[0].im), (FT)(-2.0 * alpha * hacc[0].re));
            y[t] = cadd(y[t], rhs);
        }
    }
    obs_part[0] = nu;
    obs_part[1] = dip;
    obs_part[2] = acc;
    if (!do_factor) return;
    (void)m;
    // Schur contribution of this chunk
    FT* rb = red + 2 * (sd.red_off + (long long)k * ReducedIdx<FT>::chunk_block(PP));
    const int pp = PP * PP;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
#pragma unroll
        for (int i2 = 0; i2 <= i; ++i2) {
            st_c(rb, i * PP + i2, W[i][i2]);
            st_c(rb, i2 * PP + i, W[i][i2]);
        }
#pragma unroll
        for (int t = 0; t < PP; ++t) st_c(rb, pp + i * PP + t, F[i][t]);
#pragma unroll
        for (int u = i; u < PP; ++u) {
            st_c(rb, 2 * pp + i * PP + u, TL[i][u]);
            st_c(rb, 2 * pp + u * PP + i, TL[i][u]);
        }
        st_c(rb, 3 * pp + i, y[i]);
        st_c(rb, 3 * pp + PP + i, gT[i]);
    }
}

// Pass R: block tridiagonal solve over the P separators (block size p).
//   Sigma_s = W_s + TL_{s+1},  coupling T[s][s-1] = F_s,  g_s = yR_s + gT_{s+1}
//   Delta_0 = Sigma_0; Delta_s = Sigma_s - F_s Delta_{s-1}^-1 F_s^T
//   z_s = g_s - F_s Delta_{s-1}^-1 z_{s-1}
//   x_{P-1} = Delta^-1 z; x_s = Delta_s^-1 (z_s - F_{s+1}^T x_{s+1})
// Entry-parallel: lane (i, j) = (lane / 8, lane % 8) holds one entry of an
// 8 x 8 block (p <= 7, the rest is identity padding).
template <typename FT>
__device__ void pass_reduced(const SysDesc& sd, int lane, FT* __restrict__ red) {
    const int p = sd.p, P = sd.P;
    const long long cb = ReducedIdx<FT>::chunk_block(p);
    FT* rbase = red + 2 * sd.red_off;
    FT* dinv_base = rbase + 2 * ((long long)P * cb);            // P blocks of p*p
    FT* z_base = dinv_base + 2 * ((long long)P * p * p);         // P vectors of p
    FT* x_base = z_base + 2 * ((long long)P * p);                // P vectors of p
    __shared__ cplx<FT> sA[64], sPrev[64], sF[64], sM[64];
    __shared__ cplx<FT> sz[8], szp[8], sx[8], sw[8];
    const int i = lane >> 3, j = lane & 7;
    const bool valid = (i < p) && (j < p);
    const int pp = p * p;
    for (int s = 0; s < P; ++s) {
        const FT* rs = rbase + 2 * ((long long)s * cb);
        cplx<FT> v = cmk<FT>(i == j ? (FT)1 : (FT)0, 0);
        cplx<FT> fv = cmk<FT>(0, 0);
        if (valid) {
            v = ld_c(rs, i * p + j);
            fv = ld_c(rs, pp + i * p + j);
            if (s + 1 < P) v = cadd(v, ld_c(rs + 2 * cb, 2 * pp + i * p + j));
        }
        if (lane < 8) {
            cplx<FT> g = cmk<FT>(0, 0);
            if (lane < p) {
                g = ld_c(rs, 3 * pp + lane);
                if (s + 1 < P) g = cadd(g, ld_c(rs + 2 * cb, 3 * pp + p + lane));
            }
            sz[lane] = g;
        }
        sF[lane] = fv;
        __syncthreads();
        if (s >= 1) {
            // M = F_s Delta_{s-1}^-1
            cplx<FT> mm = cmk<FT>(0, 0);
            for (int l = 0; l < p; ++l) mm = cfma(mm, sF[i * 8 + l], sPrev[l * 8 + j]);
            sM[lane] = valid ? mm : cmk<FT>(0, 0);
            __syncthreads();
            if (valid)
                for (int l = 0; l < p; ++l) v = cfms(v, sM[i * 8 + l], sF[j * 8 + l]);
            if (lane < p) {
                cplx<FT> g = sz[lane];
                for (int l = 0; l < p; ++l) g = cfms(g, sM[lane * 8 + l], szp[l]);
                sz[lane] = g;
            }
        }
        sA[lane] = v;
        __syncthreads();
        // in-place Gauss-Jordan inverse (no pivoting)
        for (int q = 0; q < p; ++q) {
            cplx<FT> aqq = sA[q * 8 + q], aiq = sA[i * 8 + q], aqj = sA[q * 8 + j], aij = sA[lane];
            cplx<FT> piv = cinv(aqq);
            cplx<FT> nv;
            if (i == q && j == q) nv = piv;
            else if (i == q) nv = cmul(aqj, piv);
            else if (j == q) nv = cscale(cmul(aiq, piv), (FT)-1);
            else nv = cfms(aij, cmul(aiq, piv), aqj);
            __syncthreads();
            sA[lane] = nv;
            __syncthreads();
        }
        cplx<FT> dv = sA[lane];
        sPrev[lane] = dv;
        if (valid) st_c(dinv_base, (long long)s * pp + i * p + j, dv);
        if (lane < 8) {
            szp[lane] = sz[lane];
            if (lane < p) st_c(z_base, (long long)s * p + lane, sz[lane]);
        }
        __syncthreads();
    }
    // backward substitution
    for (int s = P - 1; s >= 0; --s) {
        if (lane < 8) {
            cplx<FT> w = cmk<FT>(0, 0);
            if (lane < p) {
                w = ld_c(z_base, (long long)s * p + lane);
                if (s + 1 < P) {
                    const FT* rn = rbase + 2 * ((long long)(s + 1) * cb);
                    for (int t = 0; t < p; ++t) w = cfms(w, ld_c(rn, pp + t * p + lane), sx[t]);
                }
            }
            sw[lane] = w;
        }
        __syncthreads();
        if (lane < p) {
            cplx<FT> xv = cmk<FT>(0, 0);
            for (int l = 0; l < p; ++l) xv = cfma(xv, ld_c(dinv_base, (long long)s * pp + lane * p + l), sw[l]);
            sx[lane] = xv;
            st_c(x_base, (long long)s * p + lane, xv);
        }
        __syncthreads();
    }
}

// Passes U and C: forward correction of yhat for the separator values, then
// back substitution; adds the increment to the FP64 state.
template <int PP, typename FT>
__device__ void pass_backsub(const SysDesc& sd, int k, const FT* __restrict__ band,
                             double* __restrict__ st, FT* __restrict__ fac,
                             const FT* __restrict__ red, double alpha, double Ebar) {
    constexpr int NM = kNumMats;
    const int m = sd.m, LS = sd.LS, P = sd.P;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const int kk = col - 1;
    const FT* __restrict__ bnd = band + sd.band_off;
    double* __restrict__ cst = st + 2 * sd.state_off;
    FT* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
    const long long cb = ReducedIdx<FT>::chunk_block(PP);
    const FT* x_base = red + 2 * (sd.red_off + (long long)P * cb + (long long)P * PP * PP +
                                  (long long)P * PP);
    const FT a_f = (FT)alpha;
    const FT eb_f = (FT)Ebar;
    cplx<FT> xl[PP], xr[PP];
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        xl[t] = kk >= 1 ? ld_c(x_base, (long long)(kk - 1) * PP + t) : cmk<FT>(0, 0);
        xr[t] = ld_c(x_base, (long long)kk * PP + t);
    }
    auto Aentry = [&](int lrow, int d) {
        const unsigned rb = (unsigned)lrow * rowstride + (unsigned)col;
        FT s = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
        FT h = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
        FT dd = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
        return cmk<FT>(s, a_f * (h + eb_f * dd));
    };
    // u = L^-1 delta, delta = E x_left (rows 0..p-1) + F x_right (rows m-p..m-1)
    cplx<FT> pu[PP + 1];
#pragma unroll
    for (int jj = 0; jj <= PP; ++jj) pu[jj] = cmk<FT>(0, 0);
#pragma unroll
    for (int jj = 0; jj < PP; ++jj) {
        // A[jj][-p+t] is band row jj, diagonal jj + p - t, for t >= jj
#pragma unroll
        for (int t = jj; t < PP; ++t) pu[jj] = cfma(pu[jj], Aentry(jj, jj + PP - t), xl[t]);
    }
    for (int j = 0; j < m; ++j) {
        const unsigned fb = (unsigned)j * (unsigned)((PP + 2) * P) + (unsigned)kk;
        cplx<FT> u = pu[0];
        if (j >= m - PP) {
            // A[m+t][j] is band row m+t, diagonal m+t-j (when <= p)
#pragma unroll
            for (int t = 0; t < PP; ++t) {
                int d = m + t - j;
                if (d <= PP) u = cfma(u, Aentry(m + t, d), xr[t]);
            }
        }
        cplx<FT> yh = ld_c(fc, fb + (unsigned)((PP + 1) * P));
        st_c(fc, fb + (unsigned)((PP + 1) * P), csub(yh, u));
#pragma unroll
        for (int i = 1; i <= PP; ++i) {
            cplx<FT> li = ld_c(fc, fb + (unsigned)((i - 1) * P));
            pu[i - 1] = cfms(pu[i], li, u);
        }
        pu[PP] = cmk<FT>(0, 0);
    }
    // back substitution of the interior system, x_j = dinv_j yhat'_j -
    // sum_i L[j+i][j] x_{j+i} over interior rows only (the separator coupling
    // is already in yhat' through u, so the window starts at zero)
    cplx<FT> xw[PP + 1];
#pragma unroll
    for (int t = 0; t <= PP; ++t) xw[t] = cmk<FT>(0, 0);
    for (int j = m - 1; j >= 0; --j) {
        const unsigned fb = (unsigned)j * (unsigned)((PP + 2) * P) + (unsigned)kk;
        cplx<FT> xj = cmul(ld_c(fc, fb + (unsigned)(PP * P)), ld_c(fc, fb + (unsigned)((PP + 1) * P)));
#pragma unroll
        for (int i = 1; i <= PP; ++i) xj = cfms(xj, ld_c(fc, fb + (unsigned)((i - 1) * P)), xw[i]);
#pragma unroll
        for (int i = PP; i >= 2; --i) xw[i] = xw[i - 1];
        xw[1] = xj;
        unsigned at = (unsigned)j * (unsigned)LS + (unsigned)col;
        cst[2 * at] += (double)xj.re;
        cst[2 * at + 1] += (double)xj.im;
    }
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        unsigned at = (unsigned)(m + t) * (unsigned)LS + (unsigned)col;
        cst[2 * at] += (double)xr[t].re;
        cst[2 * at + 1] += (double)xr[t].im;
    }
}

__device__ inline void latch(int* status, int code, int sys, int step) {
    if (atomicCAS(&status[0], 0, code) == 0) {
        status[1] = sys;
        status[2] = step;
    }
}

template <int PP, typename FT>
__device__ void run_system(const SysDesc& sd, int sidx, const FT* __restrict__ band,
                           double* __restrict__ st, FT* __restrict__ fac, FT* __restrict__ red,
                           const double* __restrict__ E, double* __restrict__ obs, unsigned mask,
                           double norm_tol, int* status, unsigned long long* __restrict__ prof) {
    // optional phase profile: shader-clock cycles spent in the factor sweep,
    // the reduced solve and the back-substitution sweeps, summed over steps
    unsigned long long t_fac = 0, t_red = 0, t_back = 0, t0 = 0;
    const int lane = threadIdx.x;
    const bool active = lane < sd.P;
    const double alpha = 0.5 * sd.dt;
    const double* Es = E + sd.E_off;
    double* os = obs ? obs + sd.obs_off : nullptr;
    const bool want_acc = (mask & TDSEZ_OBS_ACCEL) != 0;
    double nu0 = 0.0;
    for (int n = 0; n <= sd.nsteps; ++n) {
        const bool last = (n == sd.nsteps);
        const double En = Es[n];
        const double Ebar = last ? En : 0.5 * (En + Es[n + 1]);
        double part[3] = {0.0, 0.0, 0.0};
        if (prof) t0 = clock64();
        if (active)
            pass_factor<PP, FT>(sd, lane, band, st, fac, red, alpha, Ebar, En, want_acc, !last, part);
        double nu = wave_sum(part[0]);
        double dip = wave_sum(part[1]);
        double acc = wave_sum(part[2]);
        if (lane == 0 && os) {
            os[3 * n + 0] = (mask & TDSEZ_OBS_NORM) ? nu : 0.0;
            os[3 * n + 1] = (mask & TDSEZ_OBS_DIPOLE) ? dip : 0.0;
            os[3 * n + 2] = want_acc ? acc : 0.0;
        }
        if (n == 0) nu0 = nu;
        if (!isfinite(nu) || !isfinite(dip) || !isfinite(acc)) {
            if (lane == 0) latch(status, TDSEZ_ENONFINITE, sidx, n);
            return;
        }
        if (norm_tol > 0.0 && fabs(nu / nu0 - 1.0) > norm_tol) {
            if (lane == 0) latch(status, TDSEZ_ENORMDRIFT, sidx, n);
            return;
        }
        if (last) break;
        __syncthreads();
        if (prof) { unsigned long long t = clock64(); t_fac += t - t0; t0 = t; }
        pass_reduced<FT>(sd, lane, red);
        __syncthreads();
        if (prof) { unsigned long long t = clock64(); t_red += t - t0; t0 = t; }
        if (active) pass_backsub<PP, FT>(sd, lane, band, st, fac, red, alpha, Ebar);
        __syncthreads();
        if (prof) { unsigned long long t = clock64(); t_back += t - t0; }
    }
    if (prof && lane == 0) {
        prof[4 * sidx + 0] = t_fac;
        prof[4 * sidx + 1] = t_red;
        prof[4 * sidx + 2] = t_back;
        prof[4 * sidx + 3] = (unsigned long long)sd.nsteps;
    }
}

template <typename FT>
__global__ __launch_bounds__(kWave) void propagate_kernel(const SysDesc* __restrict__ descs,
                                                          const FT* __restrict__ band,
                                                          double* __restrict__ st,
                                                          FT* __restrict__ fac,
                                                          FT* __restrict__ red,
                                                          const double* __restrict__ E,
                                                          double* __restrict__ obs, unsigned mask,
                                                          double norm_tol, int* status,
                                                          unsigned long long* __restrict__ prof) {
    const int sidx = blockIdx.x;
    const SysDesc sd = descs[sidx];
    switch (sd.p) {
        case 1: run_system<1, FT>(sd, sidx, band, st, fac, red, E, obs, mask, norm_tol, status, prof); break;
        case 2: run_system<2, FT>(sd, sidx, band, st, fac, red, E, obs, mask, norm_tol, status, prof); break;
        case 3: run_system<3, FT>(sd, sidx, band, st, fac, red, E, obs, mask, norm_tol, status, prof); break;
        case 4: run_system<4, FT>(sd, sidx, band, st, fac, red, E, obs, mask, norm_tol, status, prof); break;
        case 5: run_system<5, FT>(sd, sidx, band, st, fac, red, E, obs, mask, norm_tol, status, prof); break;
        case 6: run_system<6, FT>(sd, sidx, band, st, fac, red, E, obs, mask, norm_tol, status, prof); break;
        case 7: run_system<7, FT>(sd, sidx, band, st, fac, red, E, obs, mask, norm_tol, status, prof); break;
        default: break;
    }
}

// psi (natural order, complex128) <-> interleaved padded state
__global__ void pack_state_kernel(const SysDesc* __restrict__ descs, const double* __restrict__ psi,
                                  double* __restrict__ st) {
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
__global__ void pack_band_kernel(const double* __restrict__ S, const double* __restrict__ H0,
                                 const double* __restrict__ D, const double* __restrict__ G,
                                 const double* __restrict__ Mi, int N, int p, int P, int L, int LS,
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
                const double* src = mat == 0 ? S : mat == 1 ? H0 : mat == 2 ? D : mat == 3 ? G : Mi;
                v = src[row * (p + 1) + d];
            } else if (mat == 0 && d == 0) {
                v = 1.0;
            }
        }
        out64[e] = v;
        out32[e] = (float)v;
    }
}

}  // namespace

Plan make_plan(int N, int p, int force_chunks) {
    Plan pl;
    pl.N = N;
    pl.p = p;
    int P;
    if (force_chunks > 0) {
        P = force_chunks;
    } else {
        // balance the lane-serial sweep (~L rows) against the serial block
        // chain of the reduced system (~P blocks)
        double Lopt = std::sqrt(0.6 * N);
        if (Lopt < 2.0 * p + 2) Lopt = 2.0 * p + 2;
        P = (int)std::lround(N / Lopt);
    }
    if (P < 1) P = 1;
    if (P > kMaxChunks) P = kMaxChunks;
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

tdsez_status pack_bands(BatchData* b) {
    const int nsys = (int)b->sys.size();
    b->plan.resize(nsys);
    b->desc.resize(nsys);
    long long boff = 0, soff = 0, foff = 0, roff = 0;
    b->maxp = 0;
    for (int s = 0; s < nsys; ++s) {
        SystemData* sy = b->sys[s];
        Plan pl = make_plan(sy->N, sy->p, b->force_chunks);
        b->plan[s] = pl;
        SysDesc& d = b->desc[s];
        d = SysDesc{};
        d.N = pl.N; d.p = pl.p; d.P = pl.P; d.L = pl.L; d.m = pl.m; d.LS = pl.LS;
        d.band_off = boff;
        d.state_off = soff;
        d.fac_off = foff;
        d.red_off = roff;
        boff += (long long)pl.L * kNumMats * (pl.p + 1) * pl.LS;
        soff += (long long)pl.L * pl.LS;
        foff += (long long)pl.m * (pl.p + 2) * pl.P;
        roff += ReducedIdx<double>::total(pl.p, pl.P);
        if (pl.p > b->maxp) b->maxp = pl.p;
    }
    b->band_elems = boff;
    b->state_elems = soff;
    b->fac_elems64 = foff;
    b->red_elems64 = roff;
    TDSEZ_HIP_TRY(hipMalloc(&b->d_band64, sizeof(double) * (size_t)boff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_band32, sizeof(float) * (size_t)boff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_state, 2 * sizeof(double) * (size_t)soff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_fac, 2 * sizeof(double) * (size_t)(foff > 0 ? foff : 1)));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_red, 2 * sizeof(double) * (size_t)roff));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_desc, sizeof(SysDesc) * nsys));
    TDSEZ_HIP_TRY(hipMalloc(&b->d_status, sizeof(int) * 4));
    TDSEZ_HIP_TRY(hipMemset(b->d_status, 0, sizeof(int) * 4));
    b->nsys_alloc_desc = nsys;
    for (int s = 0; s < nsys; ++s) {
        SystemData* sy = b->sys[s];
        const Plan& pl = b->plan[s];
        long long total = (long long)pl.L * kNumMats * (pl.p + 1) * pl.LS;
        int th = 256;
        int nb = (int)std::min<long long>((total + th - 1) / th, 4096);
        pack_band_kernel<<<nb, th>>>(sy->d_band[0], sy->d_H0, sy->d_band[3], sy->d_band[4],
                                     sy->d_band[5], pl.N, pl.p, pl.P, pl.L, pl.LS,
                                     b->d_band64 + b->desc[s].band_off,
                                     b->d_band32 + b->desc[s].band_off);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    TDSEZ_HIP_TRY(hipDeviceSynchronize());
    return TDSEZ_OK;
}

tdsez_status launch_propagate(BatchData* b, double* psi, const double* E, double* obs,
                              tdsez_precision prec, unsigned obs_mask, hipStream_t stream) {
    const int nsys = (int)b->sys.size();
    TDSEZ_HIP_TRY(hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(SysDesc) * nsys,
                                 hipMemcpyHostToDevice, stream));
    long long maxL = 1, maxN = 1;
    for (const auto& pl : b->plan) {
        maxL = std::max<long long>(maxL, (long long)pl.L * pl.LS);
        maxN = std::max<long long>(maxN, pl.N);
    }
    {
        dim3 grid((unsigned)std::min<long long>((maxL + 255) / 256, 1024), nsys);
        pack_state_kernel<<<grid, 256, 0, stream>>>(b->d_desc, psi, b->d_state);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    if (prec == TDSEZ_FP64) {
        propagate_kernel<double><<<nsys, kWave, 0, stream>>>(
            b->d_desc, b->d_band64, b->d_state, (double*)b->d_fac, (double*)b->d_red, E, obs,
            obs_mask, b->norm_tol, b->d_status, b->d_prof);
    } else {
        propagate_kernel<float><<<nsys, kWave, 0, stream>>>(
            b->d_desc, b->d_band32, b->d_state, (float*)b->d_fac, (float*)b->d_red, E, obs,
            obs_mask, b->norm_tol, b->d_status, b->d_prof);
    }
    TDSEZ_HIP_TRY(hipGetLastError());
    {
        dim3 grid((unsigned)std::min<long long>((maxN + 255) / 256, 1024), nsys);
        unpack_state_kernel<<<grid, 256, 0, stream>>>(b->d_desc, b->d_state, psi);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    return TDSEZ_OK;
}

}  // namespace tdsez
