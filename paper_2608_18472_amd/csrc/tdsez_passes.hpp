// Device passes of the partitioned Crank-Nicolson solve, shared by the
// propagation and adjoint kernels (internal header, not part of the ABI).
// The algorithm and the data layouts are described at the top of
// tdsez_propagate.hip.
#pragma once

#include <hip/hip_cooperative_groups.h>

#include <cmath>

#include "tdsez_internal.hpp"

namespace tdsez {
namespace {

// Reduced-system workspace of one system (complex elements of FT).
template <typename FT>
struct RedLayout {
    // per separator block: W (p*p), F (p*p), TL (p*p), yR (p), gT (p)
    __host__ __device__ static long long chunk_block(int p) { return 3LL * p * p + 2LL * p; }
    __host__ __device__ static long long dinv(int p, int P) { return (long long)P * chunk_block(p); }
    __host__ __device__ static long long mblk(int p, int P) { return dinv(p, P) + (long long)P * p * p; }
    __host__ __device__ static long long zvec(int p, int P) { return mblk(p, P) + (long long)P * p * p; }
    __host__ __device__ static long long xvec(int p, int P) { return zvec(p, P) + (long long)P * p; }
    // third block factor per separator, used by the cyclic reduction of
    // four-wave systems (the Dinv and M slots hold the other two)
    __host__ __device__ static long long vblk(int p, int P) { return xvec(p, P) + (long long)P * p; }
    __host__ __device__ static long long total(int p, int P) { return vblk(p, P) + (long long)P * p * p; }
};

// Factor rows: pivot j of chunk k stores, at fb = j * IT * P + item * P + k
// (IT = 2p + 2 complex items): items 0..p-1 the multipliers L[j+1+i][j],
// item p 1/D_j, item p+1 yhat_j = (L^-1 b)_j, items p+2..2p+1 the fill row
// f_j = (L^-1 A_{I,left})_j (coupling of pivot j to the left separator).
__host__ __device__ inline int fac_items(int p) { return 2 * p + 2; }



// 1/z with the hardware reciprocal: one v_rcp_f32 (about 1 ulp) for FP32,
// v_rcp_f64 refined by two Newton steps for FP64.  Used for pivots, which
// are never zero (the Hermitian part of A_n is positive definite).
__device__ inline float rcp_dev(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ inline double rcp_dev(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}
template <typename FT>
__device__ inline cplx<FT> cinv_dev(cplx<FT> a) {
    FT s = rcp_dev(a.re * a.re + a.im * a.im);
    return {a.re * s, -a.im * s};
}
template <typename FT>
__device__ inline cplx<FT> csel(bool c, cplx<FT> x, cplx<FT> y) {
    return {c ? x.re : y.re, c ? x.im : y.im};
}
// value of lane `src` (wave-uniform) in every lane, without LDS
__device__ inline float bcast_lane(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double bcast_lane(double v, int src) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}
template <typename FT>
__device__ inline cplx<FT> bcast_c(cplx<FT> v, int src) {
    return {bcast_lane(v.re, src), bcast_lane(v.im, src)};
}

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

// Pass H: FP64 observables of c_n and the right-hand side of (1),
//   rhs_r = -i dt (H0 + Ebar D) c_n,   r = 0..L-1 of chunk k,
// stored (in FT) for the elimination.  Lane-serial over the chunk's rows
// plus a halo of p rows of the next chunk; each pair of rows (r, r-d) of an
// observable is counted by the owner of the larger row.
template <int PP, typename FT, bool XT = false>
__device__ __forceinline__ void pass_rhs(const SysDesc& sd, int k, const FT* __restrict__ band,
                         const double* __restrict__ st, FT* __restrict__ rhs, double alpha,
                         double Ebar, double En, bool want_acc, bool want_rhs, double obs_part[3]) {
    constexpr int NM = kNumMats;
    const int L = sd.L, LS = sd.LS;
    const bool mi_is_s = sd.mi_is_s != 0;
    // with an absorber (extended kernels only) the Hamiltonian is H - i W
    const bool cap = XT && sd.cap != 0;
    int col = k + 1;
    // Per-lane addresses are rebuilt every step instead of being hoisted out
    // of the time loop (that would keep hundreds of them live in registers).
    asm volatile("" : "+v"(col));
    const FT* __restrict__ bnd = band + sd.band_off;
    const double* __restrict__ cst = st + 2 * sd.state_off;
    FT* __restrict__ rs = rhs + 2 * sd.state_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);

    cplx<double> cw[PP + 1];    // c rows r-p..r (slot PP newest)
    cplx<double> hacc[PP + 1];  // pending (H c) of rows r-p..r
    cplx<double> wacc[XT ? PP + 1 : 1];  // pending (W c) (absorber)
#pragma unroll
    for (int i = 0; i <= PP; ++i) hacc[i] = cmk<double>(0, 0);
#pragma unroll
    for (int i = 0; i < (XT ? PP + 1 : 1); ++i) wacc[i] = cmk<double>(0, 0);
    // c rows -p..-1 come from the previous chunk (column k; zero for k = 0)
    cw[0] = cmk<double>(0, 0);
#pragma unroll
    for (int d = 0; d < PP; ++d) {
        unsigned at = (unsigned)(L - PP + d) * (unsigned)LS + (unsigned)(col - 1);
        cw[d + 1] = cmk<double>(cst[2 * at], cst[2 * at + 1]);
    }
    double nu = 0.0, dip = 0.0, acc = 0.0;

    struct RowIn {
        FT bS[PP + 1], bH[PP + 1], bD[PP + 1], bG[PP + 1], bM[PP + 1];
        FT bW[XT ? PP + 1 : 1];
        cplx<double> cr;
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
            in.bS[d] = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
            in.bH[d] = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
            in.bD[d] = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
            in.bG[d] = (FT)0;
            in.bM[d] = (FT)0;
        }
        if constexpr (XT) {
#pragma unroll
            for (int d = 0; d <= PP; ++d)
                in.bW[d] = cap ? bnd[rb + (unsigned)((kMatW * (PP + 1) + d) * LS)] : (FT)0;
        }
        if (want_acc && own) {
#pragma unroll
            for (int d = 0; d <= PP; ++d) in.bG[d] = bnd[rb + (unsigned)((3 * (PP + 1) + d) * LS)];
            // with constant mass Mi is S, whose row is already loaded
            if (!mi_is_s) {
#pragma unroll
                for (int d = 0; d <= PP; ++d) in.bM[d] = bnd[rb + (unsigned)((4 * (PP + 1) + d) * LS)];
            }
        }
        const unsigned sat = (unsigned)lr * (unsigned)LS + cc;
        in.cr = cmk<double>(cst[2 * sat], cst[2 * sat + 1]);
        return in;
    };
    auto stream_row = [&](const RowIn& in, int r, bool own) {
        const cplx<double> cr = in.cr;
#pragma unroll
        for (int d = 0; d < PP; ++d) cw[d] = cw[d + 1];
        cw[PP] = cr;
        double h[PP + 1];
#pragma unroll
        for (int d = 0; d <= PP; ++d) h[d] = (double)in.bH[d] + Ebar * (double)in.bD[d];
#pragma unroll
        for (int d = 0; d < PP; ++d) hacc[d] = hacc[d + 1];
        {
            cplx<double> sum = cmk<double>(0, 0);
            if (own) {
#pragma unroll
                for (int d = 0; d <= PP; ++d) {
                    sum.re += h[d] * cw[PP - d].re;
                    sum.im += h[d] * cw[PP - d].im;
                }
            }
            hacc[PP] = sum;
        }
#pragma unroll
        for (int d = 1; d <= PP; ++d) {
            hacc[PP - d].re += h[d] * cr.re;
            hacc[PP - d].im += h[d] * cr.im;
        }
        if constexpr (XT) {
#pragma unroll
            for (int d = 0; d < PP; ++d) wacc[d] = wacc[d + 1];
            cplx<double> sum = cmk<double>(0, 0);
            if (own) {
#pragma unroll
                for (int d = 0; d <= PP; ++d) {
                    sum.re += (double)in.bW[d] * cw[PP - d].re;
                    sum.im += (double)in.bW[d] * cw[PP - d].im;
                }
            }
            wacc[PP] = sum;
#pragma unroll
            for (int d = 1; d <= PP; ++d) {
                wacc[PP - d].re += (double)in.bW[d] * cr.re;
                wacc[PP - d].im += (double)in.bW[d] * cr.im;
            }
        }
        if (own) {
            double o[PP + 1];
#pragma unroll
            for (int d = 0; d <= PP; ++d) o[d] = cr.re * cw[PP - d].re + cr.im * cw[PP - d].im;
            double sn = (double)in.bS[0] * o[0], sdp = (double)in.bD[0] * o[0];
#pragma unroll
            for (int d = 1; d <= PP; ++d) {
                sn += 2.0 * (double)in.bS[d] * o[d];
                sdp += 2.0 * (double)in.bD[d] * o[d];
            }
            nu += sn;
            dip += sdp;
            if (want_acc) {
                double sg = 0.0, sm = 0.0;
#pragma unroll
                for (int d = 0; d <= PP; ++d) {
                    double w = d == 0 ? 1.0 : 2.0;
                    sg += w * (double)in.bG[d] * o[d];
                    if (!mi_is_s) sm += w * (double)in.bM[d] * o[d];
                }
                acc -= sg + En * (mi_is_s ? sn : sm);
            }
        }
        // row r - p is complete: -i dt H c = (2a Im, -2a Re); an absorber
        // adds -dt W c
        if (want_rhs && r >= PP) {
            const unsigned at = (unsigned)(r - PP) * (unsigned)LS + (unsigned)col;
            double zr = 2.0 * alpha * hacc[0].im, zi = -2.0 * alpha * hacc[0].re;
            if constexpr (XT) {
                zr -= 2.0 * alpha * wacc[0].re;
                zi -= 2.0 * alpha * wacc[0].im;
            }
            st_c(rs, at, cmk<FT>((FT)zr, (FT)zi));
        }
    };
    // rows are loaded two ahead of their use
    RowIn cur = load_row(0);
    RowIn nx1 = load_row(1);
    for (int r = 0; r < L; ++r) {
        RowIn nx2 = load_row(r + 2);
        stream_row(cur, r, true);
        cur = nx1;
        nx1 = nx2;
    }
    if (want_rhs) {
#pragma unroll
        for (int t = 0; t < PP; ++t) {
            RowIn nx2 = load_row(L + t + 2);
            stream_row(cur, L + t, false);
            cur = nx1;
            nx1 = nx2;
        }
    }
    obs_part[0] = nu;
    obs_part[1] = dip;
    obs_part[2] = acc;
}

// Pass A1: complex symmetric LDL^T of the chunk's rows in order (no
// pivoting: the Hermitian part S of A_n is positive definite) with forward
// substitution of the right-hand side.  Row r of A_n = S + i a (H0 + Ebar D)
// enters a (p+1)-row window; pivot j = r - p leaves it.  Entries coupling
// rows 0..p-1 to the left separator are the fill of pass A2.  Stores the
// multipliers, 1/D_j and yhat_j of every interior pivot, and the Schur block
// W and right-hand side yR of the chunk's separator rows.  With kConj the
// right-hand side is the complex conjugate of `rhs` (adjoint solves).
template <int PP, typename FT, bool kConj = false, bool XT = false>
__device__ __forceinline__ void pass_elim(const SysDesc& sd, int k, const FT* __restrict__ band,
                          const FT* __restrict__ rhs, FT* __restrict__ fac, FT* __restrict__ red,
                          double alpha, double Ebar) {
    const bool cap = XT && sd.cap != 0;
    constexpr int NM = kNumMats;
    constexpr int IT = 2 * PP + 2;
    const int L = sd.L, LS = sd.LS, P = sd.P;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const int kk = col - 1;
    const FT* __restrict__ bnd = band + sd.band_off;
    const FT* __restrict__ rs = rhs + 2 * sd.state_off;
    FT* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
    const unsigned fstride = (unsigned)(IT * P);
    const FT a_f = (FT)alpha;
    const FT eb_f = (FT)Ebar;

    cplx<FT> W[PP + 1][PP + 1];  // lower triangle used: W[i][i2], i2 <= i
    cplx<FT> y[PP + 1];
#pragma unroll
    for (int i = 0; i <= PP; ++i) {
#pragma unroll
        for (int i2 = 0; i2 <= PP; ++i2) W[i][i2] = cmk<FT>(0, 0);
        y[i] = cmk<FT>(0, 0);
    }
    struct RowIn {
        FT bS[PP + 1], bH[PP + 1], bD[PP + 1];
        cplx<FT> b;
    };
    auto load_row = [&](int r) {
        if (r >= L) r = L - 1;
        const unsigned rb = (unsigned)r * rowstride + (unsigned)col;
        RowIn in;
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            in.bS[d] = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
            in.bH[d] = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
            in.bD[d] = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
            // absorber: real part S + a W
            if (cap) in.bS[d] += a_f * bnd[rb + (unsigned)((kMatW * (PP + 1) + d) * LS)];
        }
        in.b = ld_c(rs, (unsigned)r * (unsigned)LS + (unsigned)col);
        return in;
    };
    auto row = [&](const RowIn& in, int r, bool first_rows, bool elim) {
        // insert row r as window slot PP: A[r][r-d] = S + i a (H0 + Ebar D)
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            const cplx<FT> a = cmk<FT>(in.bS[d], a_f * (in.bH[d] + eb_f * in.bD[d]));
            if (!first_rows || r - d >= 0) W[PP][PP - d] = a;
        }
        y[PP] = kConj ? cmk<FT>(in.b.re, -in.b.im) : in.b;
        if (elim) {
            const int j = r - PP;
            const cplx<FT> dinv = cinv_dev(W[0][0]);
            cplx<FT> l[PP + 1];
#pragma unroll
            for (int i = 1; i <= PP; ++i) l[i] = cmul(W[i][0], dinv);
#pragma unroll
            for (int i = 1; i <= PP; ++i)
#pragma unroll
                for (int i2 = 1; i2 <= i; ++i2) W[i][i2] = cfms(W[i][i2], l[i], W[i2][0]);
            const cplx<FT> yj = y[0];
#pragma unroll
            for (int i = 1; i <= PP; ++i) y[i] = cfms(y[i], l[i], yj);
            const unsigned fb = (unsigned)j * fstride + (unsigned)kk;
#pragma unroll
            for (int i = 1; i <= PP; ++i) st_c(fc, fb + (unsigned)((i - 1) * P), l[i]);
            st_c(fc, fb + (unsigned)(PP * P), dinv);
            st_c(fc, fb + (unsigned)((PP + 1) * P), yj);
        }
        // shift the window by one row
#pragma unroll
        for (int i = 1; i <= PP; ++i) {
#pragma unroll
            for (int i2 = 1; i2 <= i; ++i2) W[i - 1][i2 - 1] = W[i][i2];
            y[i - 1] = y[i];
        }
#pragma unroll
        for (int i2 = 0; i2 <= PP; ++i2) W[PP][i2] = cmk<FT>(0, 0);
        y[PP] = cmk<FT>(0, 0);
    };
    // rows are loaded two ahead of their use
    RowIn cur = load_row(0);
    RowIn nx1 = load_row(1);
#pragma unroll
    for (int r = 0; r < PP; ++r) {
        RowIn nx2 = load_row(r + 2);
        row(cur, r, true, false);
        cur = nx1;
        nx1 = nx2;
    }
    for (int r = PP; r < L; ++r) {
        RowIn nx2 = load_row(r + 2);
        row(cur, r, false, true);
        cur = nx1;
        nx1 = nx2;
    }
    // the window now holds the chunk's separator rows m..L-1
    FT* rb = red + 2 * (sd.red_off + (long long)k * RedLayout<FT>::chunk_block(PP));
    const int pp = PP * PP;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
#pragma unroll
        for (int i2 = 0; i2 <= i; ++i2) {
            st_c(rb, (unsigned)(i * PP + i2), W[i][i2]);
            st_c(rb, (unsigned)(i2 * PP + i), W[i][i2]);
        }
        st_c(rb, (unsigned)(3 * pp + i), y[i]);
    }
}

// Passes H and A1 in one sweep (propagation steps that continue): each band
// row and state row of the chunk (and of a p-row halo of the next chunk) is
// read once to
//  - accumulate the FP64 observables of c_n, as pass_rhs;
//  - build the right-hand side -i dt (H0 + Ebar D) c_n inside the
//    elimination window instead of storing it: row r receives the part from
//    c_{r-p..r} when it enters the window and the parts from c_{r+1..r+p} in
//    the next p steps, all before it leaves the window as pivot r; the
//    elimination updates of earlier pivots arrive in between, which is
//    harmless since both are additive;
//  - eliminate as pass_elim (multipliers, 1/D_j, yhat_j; Schur block W and
//    right-hand side yR of the separator rows).
template <int PP, typename FT, bool XT = false>
__device__ __forceinline__ void pass_rhs_elim(const SysDesc& sd, int k, const FT* __restrict__ band,
                                              const double* __restrict__ st, FT* __restrict__ fac,
                                              FT* __restrict__ red, double alpha, double Ebar, double En,
                                              bool want_acc, double obs_part[3]) {
    constexpr int NM = kNumMats;
    constexpr int IT = 2 * PP + 2;
    const int L = sd.L, LS = sd.LS, P = sd.P;
    const bool mi_is_s = sd.mi_is_s != 0;
    const bool cap = XT && sd.cap != 0;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const int kk = col - 1;
    const FT* __restrict__ bnd = band + sd.band_off;
    const double* __restrict__ cst = st + 2 * sd.state_off;
    FT* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
    const unsigned fstride = (unsigned)(IT * P);
    const FT a_f = (FT)alpha;
    const FT eb_f = (FT)Ebar;
    const double twoa = 2.0 * alpha;
    // -i 2a z, rounded to the factor precision
    auto rhs_of = [&](double zr, double zi) { return cmk<FT>((FT)(twoa * zi), (FT)(-twoa * zr)); };
    // -2a (h - i w) c for an absorber row entry pair (h, w) and state c
    auto rhs_cap = [&](double h, double w, cplx<double> c) {
        return cmk<FT>((FT)(twoa * (h * c.im - w * c.re)), (FT)(-twoa * (h * c.re + w * c.im)));
    };

    cplx<double> cw[PP + 1];     // c rows r-p..r (slot PP newest)
    cplx<FT> W[PP + 1][PP + 1];  // lower triangle used: rows r-p..r in slots 0..PP
    cplx<FT> y[PP + 1];
#pragma unroll
    for (int i = 0; i <= PP; ++i) {
#pragma unroll
        for (int i2 = 0; i2 <= PP; ++i2) W[i][i2] = cmk<FT>(0, 0);
        y[i] = cmk<FT>(0, 0);
    }
    // c rows -p..-1 come from the previous chunk (column k; zero for k = 0)
    cw[0] = cmk<double>(0, 0);
#pragma unroll
    for (int d = 0; d < PP; ++d) {
        unsigned at = (unsigned)(L - PP + d) * (unsigned)LS + (unsigned)(col - 1);
        cw[d + 1] = cmk<double>(cst[2 * at], cst[2 * at + 1]);
    }
    double nu = 0.0, dip = 0.0, acc = 0.0;

    struct RowIn {
        FT bS[PP + 1], bH[PP + 1], bD[PP + 1], bG[PP + 1], bM[PP + 1];
        FT bW[XT ? PP + 1 : 1];
        cplx<double> cr;
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
            in.bS[d] = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
            in.bH[d] = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
            in.bD[d] = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
            in.bG[d] = (FT)0;
            in.bM[d] = (FT)0;
        }
        if constexpr (XT) {
#pragma unroll
            for (int d = 0; d <= PP; ++d)
                in.bW[d] = cap ? bnd[rb + (unsigned)((kMatW * (PP + 1) + d) * LS)] : (FT)0;
        }
        if (want_acc && own) {
#pragma unroll
            for (int d = 0; d <= PP; ++d) in.bG[d] = bnd[rb + (unsigned)((3 * (PP + 1) + d) * LS)];
            if (!mi_is_s) {
#pragma unroll
                for (int d = 0; d <= PP; ++d) in.bM[d] = bnd[rb + (unsigned)((4 * (PP + 1) + d) * LS)];
            }
        }
        const unsigned sat = (unsigned)lr * (unsigned)LS + cc;
        in.cr = cmk<double>(cst[2 * sat], cst[2 * sat + 1]);
        return in;
    };
    // own row r: observables, right-hand-side parts, insertion, elimination
    // of pivot r - p, shift
    auto own_row = [&](const RowIn& in, int r, bool first_rows, bool elim) {
        const cplx<double> cr = in.cr;
#pragma unroll
        for (int d = 0; d < PP; ++d) cw[d] = cw[d + 1];
        cw[PP] = cr;
        double h[PP + 1];
#pragma unroll
        for (int d = 0; d <= PP; ++d) h[d] = (double)in.bH[d] + Ebar * (double)in.bD[d];
        if constexpr (!XT) {
            {
                // row r: sum_d M[r][r-d] c_{r-d}
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int d = 0; d <= PP; ++d) {
                    sr += h[d] * cw[PP - d].re;
                    si += h[d] * cw[PP - d].im;
                }
                y[PP] = cadd(y[PP], rhs_of(sr, si));
            }
            // rows r-d receive M[r-d][r] c_r = M[r][r-d] c_r
#pragma unroll
            for (int d = 1; d <= PP; ++d) y[PP - d] = cadd(y[PP - d], rhs_of(h[d] * cr.re, h[d] * cr.im));
        } else {
            // the same with the absorber: H - i W
#pragma unroll
            for (int d = 0; d <= PP; ++d) y[PP] = cadd(y[PP], rhs_cap(h[d], (double)in.bW[d], cw[PP - d]));
#pragma unroll
            for (int d = 1; d <= PP; ++d) y[PP - d] = cadd(y[PP - d], rhs_cap(h[d], (double)in.bW[d], cr));
        }
        {
            double o[PP + 1];
#pragma unroll
            for (int d = 0; d <= PP; ++d) o[d] = cr.re * cw[PP - d].re + cr.im * cw[PP - d].im;
            double sn = (double)in.bS[0] * o[0], sdp = (double)in.bD[0] * o[0];
#pragma unroll
            for (int d = 1; d <= PP; ++d) {
                sn += 2.0 * (double)in.bS[d] * o[d];
                sdp += 2.0 * (double)in.bD[d] * o[d];
            }
            nu += sn;
            dip += sdp;
            if (want_acc) {
                double sg = 0.0, sm = 0.0;
#pragma unroll
                for (int d = 0; d <= PP; ++d) {
                    double w = d == 0 ? 1.0 : 2.0;
                    sg += w * (double)in.bG[d] * o[d];
                    if (!mi_is_s) sm += w * (double)in.bM[d] * o[d];
                }
                acc -= sg + En * (mi_is_s ? sn : sm);
            }
        }
        // insert row r of A_n = S + i a (H0 + Ebar D) (+ a W with an absorber)
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            FT re = in.bS[d];
            if constexpr (XT) re += a_f * in.bW[d];
            const cplx<FT> a = cmk<FT>(re, a_f * (in.bH[d] + eb_f * in.bD[d]));
            if (!first_rows || r - d >= 0) W[PP][PP - d] = a;
        }
        if (elim) {
            const int j = r - PP;
            const cplx<FT> dinv = cinv_dev(W[0][0]);
            cplx<FT> l[PP + 1];
#pragma unroll
            for (int i = 1; i <= PP; ++i) l[i] = cmul(W[i][0], dinv);
#pragma unroll
            for (int i = 1; i <= PP; ++i)
#pragma unroll
                for (int i2 = 1; i2 <= i; ++i2) W[i][i2] = cfms(W[i][i2], l[i], W[i2][0]);
            const cplx<FT> yj = y[0];
#pragma unroll
            for (int i = 1; i <= PP; ++i) y[i] = cfms(y[i], l[i], yj);
            const unsigned fb = (unsigned)j * fstride + (unsigned)kk;
#pragma unroll
            for (int i = 1; i <= PP; ++i) st_c(fc, fb + (unsigned)((i - 1) * P), l[i]);
            st_c(fc, fb + (unsigned)(PP * P), dinv);
            st_c(fc, fb + (unsigned)((PP + 1) * P), yj);
        }
        // shift the window by one row
#pragma unroll
        for (int i = 1; i <= PP; ++i) {
#pragma unroll
            for (int i2 = 1; i2 <= i; ++i2) W[i - 1][i2 - 1] = W[i][i2];
            y[i - 1] = y[i];
        }
#pragma unroll
        for (int i2 = 0; i2 <= PP; ++i2) W[PP][i2] = cmk<FT>(0, 0);
        y[PP] = cmk<FT>(0, 0);
    };
    // rows are loaded one ahead of their use (the work per row covers the
    // latency; a deeper prefetch does not fit the register file)
    RowIn cur = load_row(0);
#pragma unroll
    for (int r = 0; r < PP; ++r) {
        RowIn nxt = load_row(r + 1);
        own_row(cur, r, true, false);
        cur = nxt;
    }
    for (int r = PP; r < L; ++r) {
        RowIn nxt = load_row(r + 1);
        own_row(cur, r, false, true);
        cur = nxt;
    }
    // halo rows L + t of the next chunk: their c reaches the separator rows
    // L - p .. L - 1, which now sit in window slots 0 .. p-1
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        RowIn nxt = load_row(L + t + 1);
        const cplx<double> cr = cur.cr;
#pragma unroll
        for (int d = t + 1; d <= PP; ++d) {
            const double hd = (double)cur.bH[d] + Ebar * (double)cur.bD[d];
            if constexpr (XT) y[PP + t - d] = cadd(y[PP + t - d], rhs_cap(hd, (double)cur.bW[d], cr));
            else y[PP + t - d] = cadd(y[PP + t - d], rhs_of(hd * cr.re, hd * cr.im));
        }
        cur = nxt;
    }
    FT* rb = red + 2 * (sd.red_off + (long long)k * RedLayout<FT>::chunk_block(PP));
    const int pp = PP * PP;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
#pragma unroll
        for (int i2 = 0; i2 <= i; ++i2) {
            st_c(rb, (unsigned)(i * PP + i2), W[i][i2]);
            st_c(rb, (unsigned)(i2 * PP + i), W[i][i2]);
        }
        st_c(rb, (unsigned)(3 * pp + i), y[i]);
    }
    obs_part[0] = nu;
    obs_part[1] = dip;
    obs_part[2] = acc;
}

// Pass A2: the fill of the chunk's rows towards the left separator,
//   F = L^-1 A_{I,left}  (row j of F is stored with pivot j as f_j),
// the separator rows' part of it (block F of the reduced system) and the
// Schur update of the left separator,
//   TL = -sum_j f_j^T (1/D_j) f_j,   gT = -sum_j f_j^T (1/D_j) yhat_j.
// Only rows 0..p-1 couple to the left separator directly; the multipliers of
// pass A1 carry the fill down the chunk.  With kTL == false the Schur update
// is left to pass_schur (fewer live registers for FP64).
template <int PP, typename FT, bool kTL, bool XT = false>
__device__ __forceinline__ void pass_fill(const SysDesc& sd, int k, const FT* __restrict__ band, FT* __restrict__ fac,
                          FT* __restrict__ red, double alpha, double Ebar) {
    const bool cap = XT && sd.cap != 0;
    constexpr int NM = kNumMats;
    constexpr int IT = 2 * PP + 2;
    const int L = sd.L, LS = sd.LS, P = sd.P, m = sd.m;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const int kk = col - 1;
    const FT* __restrict__ bnd = band + sd.band_off;
    FT* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
    const unsigned fstride = (unsigned)(IT * P);
    const FT a_f = (FT)alpha;
    const FT eb_f = (FT)Ebar;
    auto fitem = [&](int j, int item) {
        return ld_c(fc, (unsigned)j * fstride + (unsigned)(item * P) + (unsigned)kk);
    };
    cplx<FT> F[PP + 1][PP];
    cplx<FT> TL[PP][PP];  // upper triangle used
    cplx<FT> gT[PP];
#pragma unroll
    for (int i = 0; i <= PP; ++i)
#pragma unroll
        for (int t = 0; t < PP; ++t) F[i][t] = cmk<FT>(0, 0);
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        gT[t] = cmk<FT>(0, 0);
#pragma unroll
        for (int u = 0; u < PP; ++u) TL[t][u] = cmk<FT>(0, 0);
    }
    // rows 0..p-1: A[r][r-d] for r - d < 0 couples to left separator row
    // t = r - d + p; after the r-th shift, row r sits in window slot r
#pragma unroll
    for (int r = 0; r < PP; ++r) {
        const unsigned rb = (unsigned)r * rowstride + (unsigned)col;
#pragma unroll
        for (int d = r + 1; d <= PP; ++d) {
            FT sv = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
            FT hv = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
            FT dv = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
            if (cap) sv += a_f * bnd[rb + (unsigned)((kMatW * (PP + 1) + d) * LS)];
            F[r][r - d + PP] = cmk<FT>(sv, a_f * (hv + eb_f * dv));
        }
    }
    // pivots j = 0..m-1 leave the window from slot 0 (slot i is row j + i)
    struct FRow {
        cplx<FT> l[PP], dinv, yh;
    };
    auto load_frow = [&](int j) {
        if (j > m - 1) j = m - 1;
        FRow fr;
#pragma unroll
        for (int i = 0; i < PP; ++i) fr.l[i] = fitem(j, i);
        if (kTL) {
            fr.dinv = fitem(j, PP);
            fr.yh = fitem(j, PP + 1);
        }
        return fr;
    };
    FRow cur = load_frow(0);
    FRow nx1 = load_frow(1);
    for (int j = 0; j < m; ++j) {
        FRow nx2 = load_frow(j + 2);
        cplx<FT> f[PP];
#pragma unroll
        for (int t = 0; t < PP; ++t) f[t] = F[0][t];
        const unsigned fb = (unsigned)j * fstride + (unsigned)kk;
#pragma unroll
        for (int t = 0; t < PP; ++t) st_c(fc, fb + (unsigned)((PP + 2 + t) * P), f[t]);
#pragma unroll
        for (int i = 1; i <= PP; ++i)
#pragma unroll
            for (int t = 0; t < PP; ++t) F[i][t] = cfms(F[i][t], cur.l[i - 1], f[t]);
        if (kTL) {
            cplx<FT> g[PP];
#pragma unroll
            for (int t = 0; t < PP; ++t) g[t] = cmul(f[t], cur.dinv);
#pragma unroll
            for (int t = 0; t < PP; ++t)
#pragma unroll
                for (int u = t; u < PP; ++u) TL[t][u] = cfms(TL[t][u], f[t], g[u]);
#pragma unroll
            for (int t = 0; t < PP; ++t) gT[t] = cfms(gT[t], g[t], cur.yh);
        }
        // shift the window by one row
#pragma unroll
        for (int i = 1; i <= PP; ++i)
#pragma unroll
            for (int t = 0; t < PP; ++t) F[i - 1][t] = F[i][t];
#pragma unroll
        for (int t = 0; t < PP; ++t) F[PP][t] = cmk<FT>(0, 0);
        cur = nx1;
        nx1 = nx2;
    }
    FT* rb = red + 2 * (sd.red_off + (long long)k * RedLayout<FT>::chunk_block(PP));
    const int pp = PP * PP;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
#pragma unroll
        for (int t = 0; t < PP; ++t) st_c(rb, (unsigned)(pp + i * PP + t), F[i][t]);
        if (kTL) {
#pragma unroll
            for (int u = i; u < PP; ++u) {
                st_c(rb, (unsigned)(2 * pp + i * PP + u), TL[i][u]);
                st_c(rb, (unsigned)(2 * pp + u * PP + i), TL[i][u]);
            }
            st_c(rb, (unsigned)(3 * pp + PP + i), gT[i]);
        }
    }
}

// Pass A3 (used when pass_fill runs without the Schur update): TL and gT of
// the left separator from the stored fill rows.
template <int PP, typename FT>
__device__ __forceinline__ void pass_schur(const SysDesc& sd, int k, const FT* __restrict__ fac, FT* __restrict__ red) {
    constexpr int IT = 2 * PP + 2;
    const int P = sd.P, m = sd.m;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const int kk = col - 1;
    const FT* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned fstride = (unsigned)(IT * P);
    auto fitem = [&](int j, int item) {
        return ld_c(fc, (unsigned)j * fstride + (unsigned)(item * P) + (unsigned)kk);
    };
    cplx<FT> TL[PP][PP];
    cplx<FT> gT[PP];
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        gT[t] = cmk<FT>(0, 0);
#pragma unroll
        for (int u = 0; u < PP; ++u) TL[t][u] = cmk<FT>(0, 0);
    }
    struct FRow {
        cplx<FT> f[PP], dinv, yh;
    };
    auto load_frow = [&](int j) {
        if (j > m - 1) j = m - 1;
        FRow fr;
#pragma unroll
        for (int t = 0; t < PP; ++t) fr.f[t] = fitem(j, PP + 2 + t);
        fr.dinv = fitem(j, PP);
        fr.yh = fitem(j, PP + 1);
        return fr;
    };
    FRow cur = load_frow(0);
    for (int j = 0; j < m; ++j) {
        FRow nxt = load_frow(j + 1);
        cplx<FT> g[PP];
#pragma unroll
        for (int t = 0; t < PP; ++t) g[t] = cmul(cur.f[t], cur.dinv);
#pragma unroll
        for (int t = 0; t < PP; ++t)
#pragma unroll
            for (int u = t; u < PP; ++u) TL[t][u] = cfms(TL[t][u], cur.f[t], g[u]);
#pragma unroll
        for (int t = 0; t < PP; ++t) gT[t] = cfms(gT[t], g[t], cur.yh);
        cur = nxt;
    }
    FT* rb = red + 2 * (sd.red_off + (long long)k * RedLayout<FT>::chunk_block(PP));
    const int pp = PP * PP;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
#pragma unroll
        for (int u = i; u < PP; ++u) {
            st_c(rb, (unsigned)(2 * pp + i * PP + u), TL[i][u]);
            st_c(rb, (unsigned)(2 * pp + u * PP + i), TL[i][u]);
        }
        st_c(rb, (unsigned)(3 * pp + PP + i), gT[i]);
    }
}

// orders one wave's LDS accesses (written entries become visible to the
// wave's other lanes; later writes wait for earlier reads)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pass R: block tridiagonal solve over the P separators (block size p).
//   Sigma_s = W_s + TL_{s+1},  coupling T[s][s-1] = F_s,  g_s = yR_s + gT_{s+1}
//   Delta_0 = Sigma_0,  M_s = F_s Delta_{s-1}^-1,  Delta_s = Sigma_s - M_s F_s^T
//   z_0 = g_0,  z_s = g_s - M_s z_{s-1}
//   x_{P-1} = Delta_{P-1}^-1 z_{P-1},  x_s = Delta_s^-1 (z_s - F_{s+1}^T x_{s+1})
// Entry-parallel over one wave: lane 8i + j holds entry (i, j) of an 8 x 8
// block (p <= 7; padding rows and columns are identity / zero).  Products
// and the Gauss-Jordan inverse exchange entries with wave shuffles, so the
// chain has no LDS round trips or barriers.  Vectors are held either in row
// layout (lane (i, j) holds v[i]) or in column layout (lane (i, j) holds
// v[j]).  With factor == false the block factors Delta_s^-1 and M_s stored by
// an earlier call are reused (a further solve with the same matrix).

// compile-time flag argument of the generic chain lambdas below
template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

template <typename FT>
__device__ inline cplx<FT> shfl_c(cplx<FT> v, int src) {
    return cplx<FT>{__shfl(v.re, src, 64), __shfl(v.im, src, 64)};
}
// Data-parallel-primitive lane permutes (VALU latency, no LDS round trip):
// quad_perm [1,0,3,2] and [2,3,0,1] pair lanes within a quad, row_half_mirror
// reverses each group of 8 lanes (pairing its two quads).
template <int CTRL>
__device__ inline float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
constexpr int kDppQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;
template <int CTRL, typename FT>
__device__ inline cplx<FT> dpp_c(cplx<FT> v) {
    return {dpp<CTRL>(v.re), dpp<CTRL>(v.im)};
}
// sum over the 8 lanes of a row group (lane = 8i + j, summed over j); every
// lane of the group receives the sum.  Needs all 64 lanes active.
template <typename FT>
__device__ inline cplx<FT> row_sum(cplx<FT> v) {
    v = cadd(v, dpp_c<kDppQuadXor1>(v));
    v = cadd(v, dpp_c<kDppQuadXor2>(v));
    return cadd(v, dpp_c<kDppRowHalfMirror>(v));
}

// Pass R over one or two waves.  One wave (NW = 1): the recurrence above
// over blocks 0..P-1, then the backward sweep.  Two waves (NW = 2, systems
// with more than 64 chunks): the separator system is eliminated from both
// ends at once.  Wave 0 runs the recurrence over blocks 0..h-1 (h = P/2);
// wave 1 runs it backwards over blocks P-1..h, where the coupling of block s
// to the block eliminated before it is F_{s+1}^T (the system is symmetric,
// so the step is the same with the coupling transposed):
//   G_{P-1} = Sigma_{P-1},  N_s = F_{s+1}^T G_{s+1}^-1,
//   G_s = Sigma_s - N_s F_{s+1},  w_s = g_s - N_s w_{s+1}.
// Wave 1 then joins the halves at block h:
//   M_h = F_h Delta_{h-1}^-1,  Delta'_h = G_h - M_h F_h^T,
//   z'_h = w_h - M_h z_{h-1},  x_h = Delta'_h^-1 z'_h,
// and the waves back-substitute outwards:
//   x_s = Delta_s^-1 (z_s - F_{s+1}^T x_{s+1}),  s = h-1 .. 0     (wave 0)
//   x_s = G_s^-1 (w_s - F_s x_{s-1}),            s = h+1 .. P-1   (wave 1).
// Storage: Delta_s^-1 and G_s^-1 in the Dinv slots (Delta'_h^-1 at h), M_s
// and N_s in the M slots (M_h in the otherwise unused slot P-1), z_s and w_s
// in z (z'_h at h).  Both waves reach the same two barriers.  z lives in
// LDS (zl: P * p complex, declared once per kernel): it is written and read
// back within the pass, and LDS traffic does not queue behind the streaming
// passes of the other waves of the CU.  The back substitution writes x_s
// over z_s in LDS and copies each wave's x to the workspace after its loop.
template <int PP, typename FT, int NW>
__device__ __forceinline__ void pass_reduced_w(const SysDesc& sd, int tid, FT* __restrict__ red, bool factor,
                                               FT* __restrict__ zl) {
    constexpr int p = PP;
    const int P = sd.P, h = NW == 2 ? P / 2 : P;
    const int wv = NW == 2 ? tid >> 6 : 0, lane = tid & 63;
    const long long cb = RedLayout<FT>::chunk_block(p);
    FT* rbase = red + 2 * sd.red_off;
    FT* dinv_base = rbase + 2 * RedLayout<FT>::dinv(p, P);
    FT* m_base = rbase + 2 * RedLayout<FT>::mblk(p, P);
    FT* z_base = zl;
    FT* x_base = rbase + 2 * RedLayout<FT>::xvec(p, P);
    const int i = lane >> 3, j = lane & 7;
    const bool valid = (i < p) && (j < p);
    constexpr unsigned pp = (unsigned)(p * p);
    const unsigned eij = (unsigned)(i * p + j);
    const cplx<FT> zero = cmk<FT>(0, 0);
    const cplx<FT> ident = cmk<FT>(i == j ? (FT)1 : (FT)0, 0);
    auto blk = [&](int s) { return rbase + 2 * ((long long)s * cb); };
    const unsigned ii = (unsigned)(i < p ? i : 0);
    const unsigned ee = valid ? eij : 0u;
    const unsigned et = valid ? (unsigned)(j * p + i) : 0u;

    // C D (lane (i, j) holds C[i][j] and D[i][j])
    auto prod_cd = [&](cplx<FT> cv, cplx<FT> dv) {
        cplx<FT> cr[p], dc[p];
#pragma unroll
        for (int l = 0; l < p; ++l) {
            cr[l] = shfl_c(cv, 8 * i + l);
            dc[l] = shfl_c(dv, 8 * l + j);
        }
        cplx<FT> mm = zero;
#pragma unroll
        for (int l = 0; l < p; ++l) mm = cfma(mm, cr[l], dc[l]);
        return mm;
    };
    // A - M C^T
    auto sub_mct = [&](cplx<FT> a, cplx<FT> mm, cplx<FT> cv) {
        cplx<FT> mr[p], fc[p];
#pragma unroll
        for (int l = 0; l < p; ++l) {
            mr[l] = shfl_c(mm, 8 * i + l);
            fc[l] = shfl_c(cv, 8 * j + l);
        }
#pragma unroll
        for (int l = 0; l < p; ++l) a = cfms(a, mr[l], fc[l]);
        return a;
    };
    // Gauss-Jordan inverse of the (identity padded) block, no pivoting
    auto gj_inverse = [&](cplx<FT> a) {
#pragma unroll
        for (int q = 0; q < p; ++q) {
            const cplx<FT> aiq = shfl_c(a, 8 * i + q);
            const cplx<FT> aqj = shfl_c(a, 8 * q + j);
            const cplx<FT> piv = cinv_dev(bcast_c(a, 9 * q));
            const cplx<FT> t = cmul(aiq, piv);
            const cplx<FT> rowq = csel(j == q, piv, cmul(aqj, piv));
            const cplx<FT> other = csel(j == q, cmk<FT>(-t.re, -t.im), cfms(a, t, aqj));
            a = csel(i == q, rowq, other);
        }
        return a;
    };
    // Block operands are prefetched kRing blocks ahead into a ring that is
    // indexed by compile-time slots (the block loop is unrolled by kRing):
    // each slot keeps its registers, so no copy waits for a load in flight,
    // and the wait before a block's use covers only loads issued kRing
    // blocks earlier (and the stores issued before them).
    constexpr int kRing = sizeof(FT) == 4 ? 4 : 2;
    // elimination chain over blocks s = s0 + dir t, t = 0..count-1; the
    // coupling of block s to the block before it in the chain is F_s
    // (dir > 0) or F_{s+1}^T (dir < 0); with keep_last_raw the last block is
    // stored uninverted (for the join)
    auto chain = [&](auto fac_tag, int s0, int count, int dir, bool keep_last_raw) {
        // a compile-time copy of `factor`: the solve-only loop then holds no
        // global store, so its waits count loads only
        constexpr bool factor = decltype(fac_tag)::value;
        struct In {
            cplx<FT> y, gt, w, tl, f;
        };
        auto load = [&](int t) {
            const int tt = t < count ? t : count - 1;
            const int sc = s0 + dir * tt;
            const int s1 = sc + 1 < P ? sc + 1 : P - 1;
            const FT* bs = blk(sc);
            const FT* b1 = blk(s1);
            In r;
            r.y = ld_c(bs, 3 * pp + ii);
            r.gt = ld_c(b1, 3 * pp + (unsigned)p + ii);
            if constexpr (factor) {
                r.w = ld_c(bs, ee);
                r.tl = ld_c(b1, 2 * pp + ee);
                r.f = dir > 0 ? ld_c(bs, pp + ee) : ld_c(b1, pp + et);
            } else {
                r.w = r.tl = zero;
                r.f = ld_c(m_base, (unsigned)sc * pp + ee);  // stored M_s or N_s
            }
            return r;
        };
        cplx<FT> dprev = zero;  // inverse of the previous block of the chain
        cplx<FT> zc = zero;     // previous z (or w) in column layout
        auto step = [&](const In& cur, int t) {
            const int s = s0 + dir * t;
            const bool more = s + 1 < P;
            const cplx<FT> g = csel(i < p, cadd(cur.y, csel(more, cur.gt, zero)), zero);
            const cplx<FT> fv = csel(valid, cur.f, zero);
            cplx<FT> mm = zero;
            if constexpr (factor) {
                cplx<FT> a = csel(valid, cadd(cur.w, csel(more, cur.tl, zero)), ident);
                if (t >= 1) {
                    mm = prod_cd(fv, dprev);
                    a = sub_mct(a, mm, fv);
                    if (valid) st_c(m_base, (unsigned)s * pp + eij, mm);
                }
                if (!(keep_last_raw && t == count - 1)) a = gj_inverse(a);
                if (valid) st_c(dinv_base, (unsigned)s * pp + eij, a);
                dprev = a;
            } else {
                mm = csel(t >= 1, fv, zero);
            }
            const cplx<FT> zr = csub(g, row_sum(cmul(mm, zc)));
            if (j == 0 && i < p) st_c(z_base, (unsigned)(s * p + i), zr);
            zc = shfl_c(zr, 8 * j);
        };
        In ring[kRing];
#pragma unroll
        for (int u = 0; u < kRing; ++u) ring[u] = load(u);
        // whole groups of kRing blocks without control flow around the
        // loads (load() clamps past the end), then the last < kRing blocks
        int t0 = 0;
        for (; t0 + kRing <= count; t0 += kRing) {
#pragma unroll
            for (int u = 0; u < kRing; ++u) {
                step(ring[u], t0 + u);
                ring[u] = load(t0 + u + kRing);
            }
        }
#pragma unroll
        for (int u = 0; u + 1 < kRing; ++u)
            if (t0 + u < count) step(ring[u], t0 + u);
    };
    // x_s = D_s^-1 (z_s - C x_prev) for s = s0 + dir t, where x_prev is the
    // solution of the block before s (xc, column layout) and C = F_{s+1}^T
    // (dir < 0) or F_s (dir > 0)
    auto backsub = [&](int s0, int count, int dir, cplx<FT> xc) {
        struct In {
            cplx<FT> dv, cf;
        };
        auto load = [&](int t) {
            const int tt = t < count ? t : count - 1;
            const int sc = s0 + dir * tt;
            const int s1 = sc + 1 < P ? sc + 1 : P - 1;
            In r;
            r.dv = ld_c(dinv_base, (unsigned)sc * pp + ee);
            r.cf = dir < 0 ? ld_c(blk(s1), pp + et) : ld_c(blk(sc), pp + ee);
            return r;
        };
        auto step = [&](const In& bc, int t) {
            const int s = s0 + dir * t;
            const bool has_prev = dir < 0 ? (s + 1 < P) : (s >= 1);
            const cplx<FT> dv = csel(valid, bc.dv, ident);
            const cplx<FT> cf = csel(valid && has_prev, bc.cf, zero);
            const cplx<FT> zs = csel(i < p, ld_c(z_base, (unsigned)(s * p) + ii), zero);  // LDS
            const cplx<FT> wr = csub(zs, row_sum(cmul(cf, xc)));
            const cplx<FT> wc = shfl_c(wr, 8 * j);
            const cplx<FT> xr = row_sum(cmul(dv, wc));
            if (j == 0 && i < p) st_c(z_base, (unsigned)(s * p + i), xr);  // z_s is dead now
            xc = shfl_c(xr, 8 * j);
        };
        In ring[kRing];
#pragma unroll
        for (int u = 0; u < kRing; ++u) ring[u] = load(u);
        // whole groups of kRing blocks without control flow around the
        // loads (load() clamps past the end), then the last < kRing blocks
        int t0 = 0;
        for (; t0 + kRing <= count; t0 += kRing) {
#pragma unroll
            for (int u = 0; u < kRing; ++u) {
                step(ring[u], t0 + u);
                ring[u] = load(t0 + u + kRing);
            }
        }
#pragma unroll
        for (int u = 0; u + 1 < kRing; ++u)
            if (t0 + u < count) step(ring[u], t0 + u);
        // x of blocks s0 .. s0 + dir (count - 1) from LDS to the workspace
        // in one coalesced sweep (no global store inside the block loop)
        wave_lds_sync();
        const int lo = dir > 0 ? s0 : s0 - (count - 1);
        for (int e = lane; e < count * p; e += kWave) {
            const unsigned at = (unsigned)(lo * p + e);
            st_c(x_base, at, ld_c(z_base, at));
        }
    };

    const auto run_chain = [&](int s0, int count, int dir, bool keep_last_raw) {
        if (factor) chain(BoolTag<true>{}, s0, count, dir, keep_last_raw);
        else chain(BoolTag<false>{}, s0, count, dir, keep_last_raw);
    };
    if constexpr (NW == 1) {
        run_chain(0, P, 1, false);
        __syncthreads();  // z_s and the block factors written by other lanes
        backsub(P - 1, P, -1, zero);
        return;
    }
    if (wv == 0) run_chain(0, h, 1, false);
    else run_chain(P - 1, P - h, -1, true);
    __syncthreads();  // both halves eliminated
    if (wv == 1) {
        // join at block h
        const cplx<FT> dv = csel(valid, ld_c(dinv_base, (unsigned)(h - 1) * pp + ee), ident);
        const cplx<FT> fh = csel(valid, ld_c(blk(h), pp + ee), zero);
        const cplx<FT> zprev = csel(i < p, ld_c(z_base, (unsigned)((h - 1) * p) + ii), zero);
        const cplx<FT> wh = csel(i < p, ld_c(z_base, (unsigned)(h * p) + ii), zero);
        const cplx<FT> zpc = shfl_c(zprev, 8 * j);
        cplx<FT> mh, dinvh;
        if (factor) {
            mh = prod_cd(fh, dv);
            cplx<FT> a = csel(valid, ld_c(dinv_base, (unsigned)h * pp + ee), ident);  // G_h
            a = sub_mct(a, mh, fh);
            dinvh = gj_inverse(a);
            if (valid) {
                st_c(m_base, (unsigned)(P - 1) * pp + eij, mh);
                st_c(dinv_base, (unsigned)h * pp + eij, dinvh);
            }
        } else {
            mh = csel(valid, ld_c(m_base, (unsigned)(P - 1) * pp + ee), zero);
            dinvh = csel(valid, ld_c(dinv_base, (unsigned)h * pp + ee), ident);
        }
        const cplx<FT> zr = csub(wh, row_sum(cmul(mh, zpc)));
        const cplx<FT> zcol = shfl_c(zr, 8 * j);
        const cplx<FT> xr = row_sum(cmul(dinvh, zcol));
        if (j == 0 && i < p) {
            st_c(z_base, (unsigned)(h * p + i), zr);
            st_c(x_base, (unsigned)(h * p + i), xr);
        }
    }
    __syncthreads();  // x_h written
    const cplx<FT> xh = csel(i < p, ld_c(x_base, (unsigned)(h * p) + ii), zero);
    const cplx<FT> xhc = shfl_c(xh, 8 * j);
    if (wv == 0) backsub(h - 1, h, -1, xhc);
    else if (P - h - 1 > 0) backsub(h + 1, P - h - 1, 1, xhc);
}

// Entry-parallel block operations for the cyclic reduction below (lane
// 8i + j holds entry (i, j); the same layout as pass R above), on K
// independent blocks at once.  The operands are staged in a per-wave LDS
// area (rows padded to 9 entries, so the eight rows of a column read sit in
// different banks) and every lane reads the row and column entries it needs
// directly: a product costs one write per operand and 2p reads, of which the
// row reads are broadcasts within a row group, against 2p wave shuffles
// (each a full crossbar pass) in the shuffle form.  The item loops run
// innermost, so the K blocks' LDS traffic and arithmetic interleave.
template <typename FT, int K>
struct BlkStage {
    FT* base;  // this wave's area: slots x K blocks of 8 x 9 complex
    int i, j;
    __device__ __forceinline__ unsigned at(int slot, int c, int r, int col) const {
        return (unsigned)(((slot * K + c) * 8 + r) * 9 + col);
    }
    __device__ __forceinline__ void put(int slot, int c, cplx<FT> v) const { st_c(base, at(slot, c, i, j), v); }
    __device__ __forceinline__ cplx<FT> get(int slot, int c, int r, int col) const {
        return ld_c(base, at(slot, c, r, col));
    }
};
// out = C D for the staged slots sc (C) and sd (D)
template <int p, typename FT, int K>
__device__ __forceinline__ void stage_prod(const BlkStage<FT, K>& S, int sc, int sd, cplx<FT> (&out)[K]) {
#pragma unroll
    for (int c = 0; c < K; ++c) out[c] = cmk<FT>(0, 0);
#pragma unroll
    for (int l = 0; l < p; ++l) {
#pragma unroll
        for (int c = 0; c < K; ++c) out[c] = cfma(out[c], S.get(sc, c, S.i, l), S.get(sd, c, l, S.j));
    }
}
// Gauss-Jordan inverses of identity-padded blocks through LDS slot `slot`,
// no pivoting (every block is a Schur complement of A_n, whose Hermitian
// part is definite)
template <int p, typename FT, int K>
__device__ __forceinline__ void stage_inverse(const BlkStage<FT, K>& S, int slot, cplx<FT> (&a)[K]) {
    const int i = S.i, j = S.j;
#pragma unroll
    for (int q = 0; q < p; ++q) {
#pragma unroll
        for (int c = 0; c < K; ++c) S.put(slot, c, a[c]);
        wave_lds_sync();
        cplx<FT> aiq[K], aqj[K], piv[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            aiq[c] = S.get(slot, c, i, q);
            aqj[c] = S.get(slot, c, q, j);
            piv[c] = cinv_dev(S.get(slot, c, q, q));
        }
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const cplx<FT> t = cmul(aiq[c], piv[c]);
            const cplx<FT> rowq = csel(j == q, piv[c], cmul(aqj[c], piv[c]));
            const cplx<FT> other = csel(j == q, cmk<FT>(-t.re, -t.im), cfms(a[c], t, aqj[c]));
            a[c] = csel(i == q, rowq, other);
        }
    }
}
// LDS of the four-wave reduction: the g vectors (P * p complex) and five
// staging slots of K blocks per wave
template <typename FT>
struct CrLds {
    static constexpr int kK = sizeof(FT) == 4 ? 4 : 2;
    static constexpr int kSlots = 5;
    static constexpr int kG = 2 * kMaxP * kWave * 4;               // FT elements of g
    static constexpr int kWaveStage = 2 * kSlots * kK * 8 * 9;      // FT elements per wave
    static constexpr int kTotal = kG + 4 * kWaveStage;
};

// One system spread over G workgroups (a lone long chain, see
// tdsez_propagate): workgroup g owns the blocks k0 .. k0 + Pl - 1 of the
// separator system, k0 = g Pl.  Its last block ("super" block of g) stays to
// the top of the local reduction; block k0 - 1, the super block of g - 1,
// enters as a kept neighbour on the left that is never eliminated (its
// diagonal and right-hand-side contributions from this workgroup's side
// accumulate in dS, dg).  The G super blocks then form a block tridiagonal
// system that every workgroup solves itself (so only one grid barrier is
// needed), and the local back substitution follows.
template <typename FT>
struct SpanCtx {
    int k0, Pl, g, G;
    FT* xch;   // this solve's exchange entries (G of XchLayout), or nullptr
    FT* gfac;  // this workgroup's factors of the super-block system
};
// per workgroup: reduced S, C (coupling to the left super block), dS (pp
// each), g and dg (p each), complex
__host__ __device__ inline long long xch_entry(int p) { return 3LL * p * p + 2LL * p; }
// per super block j: Dinv, M, C (pp each) and z (p), complex; G + 1 entries
// per workgroup (the last one for the join of the two-sided elimination)
__host__ __device__ inline long long gfac_entry(int p) { return 3LL * p * p + p; }

__device__ __forceinline__ void grid_barrier() { cooperative_groups::this_grid().sync(); }

// Pass R on four waves (systems with more than 128 chunks): block cyclic
// reduction of the separator system, so that the solve is log2(P) levels
// deep and every level's block operations are shared by the four waves.
// Level l works on the active blocks a_0 < ... < a_n, n = ceil(P / 2^l) - 1,
// a_q = (q + 1) 2^l - 1 for q < n and a_n = P - 1 (the last block stays to
// the end).  The blocks at even positions q < n are eliminated; with Sigma_e
// the current diagonal block, C_e its coupling to the active block on its
// left (T[e][left]) and C_r that of the active block r on its right
// (T[r][e]):
//   D_e = Sigma_e^-1,  U_e = D_e C_e,  V_e = D_e C_r^T,  h_e = D_e g_e.
// Every kept block r, with eliminated neighbours e (left) and e' (right)
// where they exist:
//   Sigma_r -= C_r V_e + C_e'^T U_e',   g_r -= V_e^T g_e + U_e'^T g_e',
//   C_r <- -C_r U_e   (its coupling to the next active block on the left).
// The blocks stay complex symmetric (D_e^T = D_e), which gives the
// transposes above.  At the top x_{P-1} = Sigma_{P-1}^-1 g_{P-1}; then, from
// the top level down, x_e = h_e - U_e x_left - V_e x_right.  Level 0 reads
// Sigma_s = W_s + TL_{s+1} and g_s = yR_s + gT_{s+1} from the chunk blocks;
// the updated Sigma and C overwrite the W and F slots, g lives in LDS (gl:
// P * p complex) and h, then x, in the x slots.  D, U and V are stored (Dinv,
// M and V slots), so a solve with the same matrix (factor == false) repeats
// only the g updates and the back substitution.  Each wave takes K items of
// a phase at a time (absent neighbours enter as zero blocks, so there are
// no per-item branches).  Two barriers per level on the way up, one on the
// way down; every wave reaches all of them.  SPAN: the workgroup's share of
// a system on several workgroups (SpanCtx); the levels run over its Pl
// blocks, the left neighbour block k0 - 1 is kept at every level.
template <int PP, typename FT, int NW, bool SPAN>
__device__ __forceinline__ void pass_reduced_cr(const SysDesc& sd, int tid, FT* __restrict__ red, bool factor,
                                                FT* __restrict__ lds, const SpanCtx<FT>& sc) {
    static_assert(NW == 4, "the LDS layout holds four waves");
    constexpr int p = PP;
    constexpr int K = CrLds<FT>::kK;
    FT* gl = lds;
    const int P = sd.P;
    const int k0 = sc.k0, Pl = sc.Pl;
    const bool ext = SPAN && sc.g > 0;  // a kept neighbour block on the left (k0 - 1)
    const int wv = tid >> 6, lane = tid & 63;
    const long long cb = RedLayout<FT>::chunk_block(p);
    FT* rbase = red + 2 * sd.red_off;
    FT* d_base = rbase + 2 * RedLayout<FT>::dinv(p, P);
    FT* u_base = rbase + 2 * RedLayout<FT>::mblk(p, P);
    FT* v_base = rbase + 2 * RedLayout<FT>::vblk(p, P);
    FT* x_base = rbase + 2 * RedLayout<FT>::xvec(p, P);
    const int i = lane >> 3, j = lane & 7;
    const bool valid = (i < p) && (j < p);
    constexpr unsigned pp = (unsigned)(p * p);
    const unsigned ii = (unsigned)(i < p ? i : 0);
    const unsigned ee = valid ? (unsigned)(i * p + j) : 0u;
    const unsigned et = valid ? (unsigned)(j * p + i) : 0u;
    const cplx<FT> zero = cmk<FT>(0, 0);
    const cplx<FT> ident = cmk<FT>(i == j ? (FT)1 : (FT)0, 0);
    const BlkStage<FT, K> S{lds + CrLds<FT>::kG + wv * CrLds<FT>::kWaveStage, i, j};
    // local block s -> its chunk block (global index k0 + s)
    auto blk = [&](int s) { return rbase + 2 * ((long long)(k0 + s) * cb); };
    // entry e of stored local block s of a factor array, zero where `on` is false
    auto ld_f = [&](const FT* base, int s, unsigned e, bool on) {
        return csel(valid && on, ld_c(base, (unsigned)(k0 + s) * pp + e), zero);
    };
    auto st_blk = [&](FT* base, int s, cplx<FT> v) {
        if (valid) st_c(base, (unsigned)(k0 + s) * pp + ee, v);
    };
    // (a workgroup's last block takes no TL / gT from the next workgroup's
    // first chunk: that workgroup adds them to its dS, dg)
    auto load_sig = [&](int s, int l) {
        cplx<FT> a = ld_c(blk(s), ee);
        if (l == 0 && s + 1 < Pl) a = cadd(a, ld_c(blk(s + 1), 2 * pp + ee));
        return csel(valid, a, ident);
    };
    // g_s in row layout (lane (i, j) holds g_s[i]), zero where `on` is false
    auto load_g = [&](int s, int l, bool on) {
        cplx<FT> g;
        if (l == 0) {
            g = ld_c(blk(s), 3 * pp + ii);
            if (s + 1 < Pl) g = cadd(g, ld_c(blk(s + 1), 3 * pp + (unsigned)p + ii));
        } else {
            g = ld_c(gl, (unsigned)(s * p) + ii);
        }
        return csel(i < p && on, g, zero);
    };
    // row layout -> column layout (lane (i, j) gets v[j])
    auto colv = [&](cplx<FT> v) { return shfl_c(v, 8 * j); };
    auto ld_x = [&](int s, bool on) { return csel(i < p && on, ld_c(x_base, (unsigned)((k0 + s) * p) + ii), zero); };
    auto st_x = [&](int s, cplx<FT> v) {
        if (j == 0 && i < p) st_c(x_base, (unsigned)((k0 + s) * p + i), v);
    };
    auto st_gl = [&](int s, cplx<FT> v) {
        if (j == 0 && i < p) st_c(gl, (unsigned)(s * p + i), v);
    };
    // exchange entry of workgroup w (SPAN)
    auto xe = [&](int w) { return sc.xch + 2 * (long long)w * xch_entry(p); };

    int nlev = 0;
    while ((1 << nlev) < Pl) ++nlev;
    for (int l = 0; l < nlev; ++l) {
        const int st = 1 << l;
        const int n = (Pl + st - 1) / st - 1;
        // eliminations: positions q = 0, 2, .. < n
        const int ne = (n + 1) / 2;
        for (int t0 = wv; t0 < ne; t0 += NW * K) {
            int e[K];
            bool ok[K];
            cplx<FT> a[K], g[K], ce[K], crt[K], h[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int t = t0 + NW * c;
                ok[c] = t < ne;
                const int q = 2 * (ok[c] ? t : t0);
                e[c] = (q + 1) * st - 1;
                const int r = q + 1 < n ? e[c] + st : Pl - 1;
                a[c] = factor ? load_sig(e[c], l) : csel(valid, ld_c(d_base, (unsigned)(k0 + e[c]) * pp + ee), ident);
                g[c] = load_g(e[c], l, true);
                if (factor) {
                    ce[c] = csel(valid && (q > 0 || ext), ld_c(blk(e[c]), pp + ee), zero);
                    crt[c] = csel(valid, ld_c(blk(r), pp + et), zero);
                }
            }
            if (factor) stage_inverse<p, FT, K>(S, 0, a);
#pragma unroll
            for (int c = 0; c < K; ++c) h[c] = row_sum(cmul(a[c], colv(g[c])));
            if (factor) {
                cplx<FT> u[K], v[K];
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    S.put(0, c, a[c]);
                    S.put(1, c, ce[c]);
                    S.put(2, c, crt[c]);
                }
                wave_lds_sync();
                stage_prod<p, FT, K>(S, 0, 1, u);
                stage_prod<p, FT, K>(S, 0, 2, v);
                wave_lds_sync();
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    if (ok[c]) {
                        st_blk(d_base, e[c], a[c]);
                        st_blk(u_base, e[c], u[c]);
                        st_blk(v_base, e[c], v[c]);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < K; ++c)
                if (ok[c]) st_x(e[c], h[c]);
        }
        __syncthreads();
        // kept blocks: odd positions, and the last one (Pl - 1); with ext one
        // more item (t == nk) for the left neighbour block
        const int nk = n / 2 + 1;
        const int nit = nk + (ext ? 1 : 0);
        for (int t0 = wv; t0 < nit; t0 += NW * K) {
            int r[K];
            bool ok[K], hl[K], isl[K];
            cplx<FT> g[K], ge[K], ge2[K], vte[K], ute2[K];
            cplx<FT> sg[K], cr[K], ve[K], ue[K], c2t[K], ue2[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int t = t0 + NW * c;
                ok[c] = t < nit;
                const int tt = ok[c] ? t : t0;
                isl[c] = ext && tt == nk;
                const int q = isl[c] ? -1 : (2 * tt + 1 < n ? 2 * tt + 1 : n);
                r[c] = isl[c] ? -1 : (q < n ? (q + 1) * st - 1 : Pl - 1);
                hl[c] = !isl[c] && (q & 1) != 0;                 // eliminated left neighbour
                const bool hr = isl[c] || (hl[c] && q + 1 < n);  // eliminated right neighbour
                const int e = isl[c] ? 0 : q * st - 1;
                const int e2 = hr ? (q + 2) * st - 1 : e;
                const int rr = isl[c] ? 0 : r[c];
                if (isl[c]) {
                    // the left neighbour's partial sums (level 0: chunk k0's
                    // TL and gT, its contribution to block k0 - 1)
                    g[c] = csel(i < p, l == 0 ? ld_c(blk(0), 3 * pp + (unsigned)p + ii) : ld_c(xe(sc.g), 3 * pp + ii + (unsigned)p),
                                zero);
                } else {
                    g[c] = load_g(rr, l, true);
                }
                ge[c] = load_g(e, l, hl[c]);
                ge2[c] = load_g(e2, l, hr);
                vte[c] = ld_f(v_base, e, et, hl[c]);
                ute2[c] = ld_f(u_base, e2, et, hr);
                if (factor) {
                    if (isl[c])
                        sg[c] = csel(valid, l == 0 ? ld_c(blk(0), 2 * pp + ee) : ld_c(xe(sc.g), 2 * pp + ee), zero);
                    else
                        sg[c] = load_sig(rr, l);
                    cr[c] = csel(valid && hl[c], ld_c(blk(rr), pp + ee), zero);
                    ve[c] = ld_f(v_base, e, ee, hl[c]);
                    ue[c] = ld_f(u_base, e, ee, hl[c]);
                    c2t[c] = csel(valid && hr, ld_c(blk(e2), pp + et), zero);
                    ue2[c] = ld_f(u_base, e2, ee, hr);
                }
            }
            if (factor) {
                cplx<FT> p1[K], p2[K], p3[K];
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    S.put(0, c, cr[c]);
                    S.put(1, c, ve[c]);
                    S.put(2, c, ue[c]);
                    S.put(3, c, c2t[c]);
                    S.put(4, c, ue2[c]);
                }
                wave_lds_sync();
                stage_prod<p, FT, K>(S, 0, 1, p1);
                stage_prod<p, FT, K>(S, 0, 2, p2);
                stage_prod<p, FT, K>(S, 3, 4, p3);
                wave_lds_sync();
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    if (ok[c]) {
                        const cplx<FT> sn = csub(csub(sg[c], p1[c]), p3[c]);
                        if (isl[c]) {
                            if (valid) st_c(xe(sc.g), 2 * pp + ee, sn);
                        } else {
                            if (valid) st_c(blk(r[c]), ee, sn);
                            if (valid && hl[c]) st_c(blk(r[c]), pp + ee, cmk<FT>(-p2[c].re, -p2[c].im));
                        }
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const cplx<FT> gn = csub(csub(g[c], row_sum(cmul(vte[c], colv(ge[c])))),
                                         row_sum(cmul(ute2[c], colv(ge2[c]))));
                if (ok[c]) {
                    if (isl[c]) {
                        if (j == 0 && i < p) st_c(xe(sc.g), 3 * pp + (unsigned)p + (unsigned)i, gn);
                    } else {
                        st_gl(r[c], gn);
                    }
                }
            }
        }
        __syncthreads();
    }
    if constexpr (SPAN) {
        // export this workgroup's reduced super block (and, with a single
        // block, the left neighbour's contribution), then solve the super
        // system redundantly in every workgroup
        if (wv == 0) {
            FT* xw = xe(sc.g);
            if (factor) {
                const cplx<FT> sgm = load_sig(Pl - 1, nlev);
                if (valid) {
                    st_c(xw, ee, sgm);
                    st_c(xw, pp + ee, ld_c(blk(Pl - 1), pp + ee));
                }
                if (nlev == 0 && ext && valid) st_c(xw, 2 * pp + ee, ld_c(blk(0), 2 * pp + ee));
            }
            const cplx<FT> gs = load_g(Pl - 1, nlev, true);
            if (j == 0 && i < p) st_c(xw, 3 * pp + (unsigned)i, gs);
            if (nlev == 0 && ext && j == 0 && i < p) st_c(xw, 3 * pp + (unsigned)(p + i), ld_c(blk(0), 3 * pp + (unsigned)(p + i)));
        }
        grid_barrier();
        // The G super blocks: Sigma_j = S_j + dS_{j+1}, g_j = gs_j + dg_{j+1},
        // T[j][j-1] = C_j.  Eliminated from both ends at once (h = G / 2):
        // wave 0 forward over j = 0 .. h-1,
        //   M_j = C_j Delta_{j-1}^-1,  Delta_j = Sigma_j - M_j C_j^T,  z_j = g_j - M_j z_{j-1},
        // wave 1 backward over j = G-1 .. h,
        //   N_j = C_{j+1}^T G_{j+1}^-1,  G_j = Sigma_j - N_j C_{j+1},  w_j = g_j - N_j w_{j+1},
        // wave 1 joins at h (M_h = C_h Delta_{h-1}^-1, Delta'_h = G_h - M_h C_h^T,
        // x_h = Delta'_h^-1 (w_h - M_h z_{h-1})), then each wave substitutes
        // outwards only as far as this workgroup's two super blocks (g - 1,
        // g).  Every workgroup repeats the same operations, so the values it
        // writes for a super block are those of its neighbours, bit for bit.
        // Per-workgroup storage (gf): Delta^-1 or G^-1, M or N, C_j, z or w;
        // entry G holds the join's M_h and x_h.  Inputs are loaded one block
        // ahead (they come from the other workgroups' fresh writes).
        const int G = sc.G, h = G / 2;
        auto gf = [&](int jj) { return sc.gfac + 2 * (long long)jj * gfac_entry(p); };
        const int need_lo = sc.g > 0 ? sc.g - 1 : 0, need_hi = sc.g;
        if (wv <= 1) {
            const BlkStage<FT, 1> S1{lds + CrLds<FT>::kG + wv * CrLds<FT>::kWaveStage, i, j};
            const int dir = wv == 0 ? 1 : -1;
            const int j0 = wv == 0 ? 0 : G - 1;
            const int cnt = wv == 0 ? h : G - h;
            struct SupIn {
                cplx<FT> rhs, a, cc, cct, cs, m;
            };
            // block jj's inputs; the coupling to the block eliminated before it
            // is C_jj (forward) or C_{jj+1}^T (backward; C_{jj+1} kept as cct's
            // transpose partner in cc)
            auto sup_load = [&](int t) {
                const int tt = t < cnt ? t : cnt - 1;
                const int jc = j0 + dir * tt;
                const bool more = jc + 1 < G;
                const bool has_prev = dir > 0 ? jc > 0 : more;
                const FT* x0 = xe(jc);
                const FT* x1 = xe(more ? jc + 1 : jc);
                const FT* xc = dir > 0 ? x0 : x1;  // the coupling's owner
                SupIn r;
                r.rhs = cadd(csel(i < p, ld_c(x0, 3 * pp + ii), zero),
                             csel(i < p && more, ld_c(x1, 3 * pp + (unsigned)p + ii), zero));
                if (factor) {
                    r.a = cadd(csel(valid, ld_c(x0, ee), ident), csel(valid && more, ld_c(x1, 2 * pp + ee), zero));
                    // forward: cc = C_jj, cct = C_jj^T; backward: cc = C_{jj+1}^T, cct = C_{jj+1}
                    r.cc = csel(valid && has_prev, ld_c(xc, pp + (dir > 0 ? ee : et)), zero);
                    r.cct = csel(valid && has_prev, ld_c(xc, pp + (dir > 0 ? et : ee)), zero);
                    r.cs = csel(valid && jc > 0, ld_c(x0, pp + ee), zero);  // C_jj
                    r.m = zero;
                } else {
                    r.a = r.cc = r.cct = r.cs = zero;
                    r.m = csel(valid && has_prev, ld_c(gf(jc), pp + ee), zero);
                }
                return r;
            };
            cplx<FT> dprev = zero, zprev = zero;  // previous block's inverse (entry), z or w (row)
            SupIn cur = sup_load(0);
            for (int t = 0; t < cnt; ++t) {
                const SupIn nxt = sup_load(t + 1);
                const int jj = j0 + dir * t;
                const bool raw = wv == 1 && jj == h;  // kept uninverted for the join
                cplx<FT> m = cur.m;
                if (factor) {
                    cplx<FT> a[1] = {cur.a};
                    if (t > 0) {
                        cplx<FT> mm[1], mc[1];
                        S1.put(0, 0, cur.cc);
                        S1.put(1, 0, dprev);
                        wave_lds_sync();
                        stage_prod<p, FT, 1>(S1, 0, 1, mm);
                        wave_lds_sync();
                        m = mm[0];
                        S1.put(0, 0, m);
                        S1.put(1, 0, cur.cct);
                        wave_lds_sync();
                        stage_prod<p, FT, 1>(S1, 0, 1, mc);
                        wave_lds_sync();
                        a[0] = csub(a[0], mc[0]);
                    }
                    if (!raw) stage_inverse<p, FT, 1>(S1, 0, a);
                    FT* gj = gf(jj);
                    if (valid) {
                        st_c(gj, ee, a[0]);
                        st_c(gj, pp + ee, m);
                        st_c(gj, 2 * pp + ee, cur.cs);  // C_jj, for the substitution
                    }
                    dprev = a[0];
                }
                const cplx<FT> z = csub(cur.rhs, row_sum(cmul(m, colv(zprev))));
                if (j == 0 && i < p) st_c(gf(jj), 3 * pp + (unsigned)i, z);
                zprev = z;
                cur = nxt;
            }
        }
        __syncthreads();
        FT* gj_join = gf(G);
        if (wv == 1) {
            const BlkStage<FT, 1> S1{lds + CrLds<FT>::kG + CrLds<FT>::kWaveStage, i, j};
            const FT* gh = gf(h);
            const cplx<FT> ch = csel(valid && h > 0, ld_c(xe(h), pp + ee), zero);
            const cplx<FT> cht = csel(valid && h > 0, ld_c(xe(h), pp + et), zero);
            const cplx<FT> dv = csel(valid && h > 0, ld_c(gf(h > 0 ? h - 1 : 0), ee), zero);
            const cplx<FT> zp = csel(i < p && h > 0, ld_c(gf(h > 0 ? h - 1 : 0), 3 * pp + ii), zero);
            const cplx<FT> wh = csel(i < p, ld_c(gh, 3 * pp + ii), zero);
            cplx<FT> mh, dinv;
            if (factor) {
                cplx<FT> mm[1], mc[1];
                S1.put(0, 0, ch);
                S1.put(1, 0, dv);
                wave_lds_sync();
                stage_prod<p, FT, 1>(S1, 0, 1, mm);
                wave_lds_sync();
                mh = mm[0];
                S1.put(0, 0, mh);
                S1.put(1, 0, cht);
                wave_lds_sync();
                stage_prod<p, FT, 1>(S1, 0, 1, mc);
                wave_lds_sync();
                cplx<FT> a[1] = {csub(csel(valid, ld_c(gh, ee), ident), mc[0])};
                stage_inverse<p, FT, 1>(S1, 0, a);
                dinv = a[0];
                if (valid) {
                    st_c(gf(h), ee, dinv);
                    st_c(gj_join, pp + ee, mh);
                }
            } else {
                mh = csel(valid, ld_c(gj_join, pp + ee), zero);
                dinv = csel(valid, ld_c(gh, ee), ident);
            }
            const cplx<FT> zr = csub(wh, row_sum(cmul(mh, colv(zp))));
            const cplx<FT> xh = row_sum(cmul(dinv, colv(zr)));
            if (j == 0 && i < p) st_c(gj_join, 3 * pp + (unsigned)i, xh);
            if ((h == need_lo || h == need_hi) && j == 0 && i < p)
                st_c(x_base, (unsigned)(((h + 1) * Pl - 1) * p + i), xh);
        }
        __syncthreads();
        if (wv <= 1) {
            // x_j = Delta_j^-1 (z_j - C_{j+1}^T x_{j+1}), j = h-1 .. need_lo   (wave 0)
            // x_j = G_j^-1 (w_j - C_j x_{j-1}),       j = h+1 .. need_hi   (wave 1)
            const int dir = wv == 0 ? -1 : 1;
            const int j0 = h + dir;
            const int cnt = wv == 0 ? (need_lo < h ? h - need_lo : 0) : (need_hi > h ? need_hi - h : 0);
            struct BkIn {
                cplx<FT> w, cp, dv;
            };
            auto bk_load = [&](int t) {
                const int tt = t < cnt ? t : (cnt > 0 ? cnt - 1 : 0);
                const int jc = j0 + dir * tt;
                const int jq = jc >= 0 && jc < G ? jc : h;
                const FT* gjq = gf(jq);
                BkIn r;
                r.w = csel(i < p, ld_c(gjq, 3 * pp + ii), zero);
                // the coupling to the block solved before: C_{j+1}^T (stored
                // as C of block j+1, read transposed) or C_j
                r.cp = wv == 0 ? csel(valid, ld_c(gf(jq + 1 <= G - 1 ? jq + 1 : jq), 2 * pp + et), zero)
                               : csel(valid, ld_c(gjq, 2 * pp + ee), zero);
                r.dv = csel(valid, ld_c(gjq, ee), ident);
                return r;
            };
            cplx<FT> xprev = csel(i < p, ld_c(gj_join, 3 * pp + ii), zero);  // x_h
            BkIn bc = bk_load(0);
            for (int t = 0; t < cnt; ++t) {
                const BkIn bn = bk_load(t + 1);
                const int jj = j0 + dir * t;
                const cplx<FT> w = csub(bc.w, row_sum(cmul(bc.cp, colv(xprev))));
                const cplx<FT> x = row_sum(cmul(bc.dv, colv(w)));
                if ((jj == need_lo || jj == need_hi) && j == 0 && i < p)
                    st_c(x_base, (unsigned)(((jj + 1) * Pl - 1) * p + i), x);
                xprev = x;
                bc = bn;
            }
        }
        __syncthreads();
    } else {
        if (wv == 0) {
            cplx<FT> d[K];
            d[0] = factor ? load_sig(Pl - 1, nlev) : csel(valid, ld_c(d_base, (unsigned)(k0 + Pl - 1) * pp + ee), ident);
#pragma unroll
            for (int c = 1; c < K; ++c) d[c] = ident;
            if (factor) {
                stage_inverse<p, FT, K>(S, 0, d);
                st_blk(d_base, Pl - 1, d[0]);
            }
            st_x(Pl - 1, row_sum(cmul(d[0], colv(load_g(Pl - 1, nlev, true)))));
        }
        __syncthreads();
    }
    for (int l = nlev - 1; l >= 0; --l) {
        const int st = 1 << l;
        const int n = (Pl + st - 1) / st - 1;
        const int ne = (n + 1) / 2;
        for (int t0 = wv; t0 < ne; t0 += NW * K) {
            int e[K];
            bool ok[K];
            cplx<FT> xe_[K], xr[K], xl[K], u[K], v[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int t = t0 + NW * c;
                ok[c] = t < ne;
                const int q = 2 * (ok[c] ? t : t0);
                e[c] = (q + 1) * st - 1;
                const int r = q + 1 < n ? e[c] + st : Pl - 1;
                const bool hasl = q > 0 || ext;
                const int lft = q > 0 ? e[c] - st : -1;  // -1: the left neighbour block k0 - 1
                xe_[c] = ld_x(e[c], true);
                xr[c] = ld_x(r, true);
                xl[c] = ld_x(hasl ? lft : e[c], hasl);
                u[c] = ld_f(u_base, e[c], ee, hasl);
                v[c] = ld_f(v_base, e[c], ee, true);
            }
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const cplx<FT> x = csub(csub(xe_[c], row_sum(cmul(v[c], colv(xr[c])))), row_sum(cmul(u[c], colv(xl[c]))));
                if (ok[c]) st_x(e[c], x);
            }
        }
        __syncthreads();
    }
}

template <int PP, typename FT>
__device__ __forceinline__ void pass_reduced(const SysDesc& sd, int lane, FT* __restrict__ red, bool factor,
                                             FT* __restrict__ zl) {
    pass_reduced_w<PP, FT, 1>(sd, lane, red, factor, zl);
}
template <int PP, typename FT>
__device__ __forceinline__ void pass_reduced2(const SysDesc& sd, int tid, FT* __restrict__ red, bool factor,
                                              FT* __restrict__ zl) {
    pass_reduced_w<PP, FT, 2>(sd, tid, red, factor, zl);
}

// Pass B: interior values of the chunk from its separator values.
//   x_I = L^-T D^-1 (yhat - F x_left - L^-1 A_{I,right} x_right)
// The fill rows make the left-separator term a dot product per row; the
// right-separator term reaches only the last p pivots (a p-row forward
// substitution).  The state gets the increment (or, with assign, is
// overwritten by the solution); with dtot != nullptr the increment is also
// written (first == true) or added to dtot.
template <int PP, typename FT, bool XT = false>
__device__ __forceinline__ void pass_backsub(const SysDesc& sd, int k, const FT* __restrict__ band,
                             double* __restrict__ st, double* __restrict__ dtot, bool first,
                             const FT* __restrict__ fac, const FT* __restrict__ red, double alpha,
                             double Ebar, bool assign = false) {
    const bool cap = XT && sd.cap != 0;
    constexpr int NM = kNumMats;
    constexpr int IT = 2 * PP + 2;
    const int LS = sd.LS, P = sd.P, m = sd.m;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const int kk = col - 1;
    const FT* __restrict__ bnd = band + sd.band_off;
    double* __restrict__ cst = st + 2 * sd.state_off;
    double* __restrict__ dst = dtot ? dtot + 2 * sd.state_off : nullptr;
    const FT* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
    const unsigned fstride = (unsigned)(IT * P);
    const FT* x_base = red + 2 * (sd.red_off + RedLayout<FT>::xvec(PP, P));
    const FT a_f = (FT)alpha;
    const FT eb_f = (FT)Ebar;
    cplx<FT> xl[PP], xr[PP];
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        xl[t] = kk >= 1 ? ld_c(x_base, (unsigned)((kk - 1) * PP + t)) : cmk<FT>(0, 0);
        xr[t] = ld_c(x_base, (unsigned)(kk * PP + t));
    }
    auto Aentry = [&](int lrow, int d) {
        const unsigned rb = (unsigned)lrow * rowstride + (unsigned)col;
        FT s = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
        FT h = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
        FT dd = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
        if (cap) s += a_f * bnd[rb + (unsigned)((kMatW * (PP + 1) + d) * LS)];
        return cmk<FT>(s, a_f * (h + eb_f * dd));
    };
    auto fitem = [&](int j, int item) {
        return ld_c(fc, (unsigned)j * fstride + (unsigned)(item * P) + (unsigned)kk);
    };
    // the state (and increment) of a row are loaded ahead with its factor
    // row, so that the update below is a plain store
    const double* dsrc = (dst && !first) ? dst : cst;  // dummy source when unused
    auto load_sd = [&](int lrow, cplx<double>& c, cplx<double>& d) {
        const unsigned at = (unsigned)lrow * (unsigned)LS + (unsigned)col;
        c = cmk<double>(cst[2 * at], cst[2 * at + 1]);
        d = cmk<double>(dsrc[2 * at], dsrc[2 * at + 1]);
    };
    auto update = [&](int lrow, cplx<FT> x, cplx<double> c, cplx<double> d) {
        const unsigned at = (unsigned)lrow * (unsigned)LS + (unsigned)col;
        if (assign) {
            cst[2 * at] = (double)x.re;
            cst[2 * at + 1] = (double)x.im;
        } else {
            cst[2 * at] = c.re + (double)x.re;
            cst[2 * at + 1] = c.im + (double)x.im;
        }
        if (dst) {
            if (first) {
                dst[2 * at] = (double)x.re;
                dst[2 * at + 1] = (double)x.im;
            } else {
                dst[2 * at] = d.re + (double)x.re;
                dst[2 * at + 1] = d.im + (double)x.im;
            }
        }
    };
    cplx<double> sepc[PP], sepd[PP];
#pragma unroll
    for (int t = 0; t < PP; ++t) load_sd(m + t, sepc[t], sepd[t]);
    // u = L^-1 A_{I,right} x_right on pivots m-p+q, q = 0..p-1
    cplx<FT> ur[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        const int j = m - PP + q;
        cplx<FT> u = cmk<FT>(0, 0);
        // A[j][m+t] is band row m+t, diagonal p+t-q (<= p for t <= q)
#pragma unroll
        for (int t = 0; t <= q; ++t) u = cfma(u, Aentry(m + t, PP + t - q), xr[t]);
        // L[j][i] for pivots i = m-p..j-1 is item j-i-1 of pivot i
#pragma unroll
        for (int q2 = 0; q2 < q; ++q2) u = cfms(u, fitem(m - PP + q2, q - q2 - 1), ur[q2]);
        ur[q] = u;
    }
    // back substitution over the interior pivots, window of the next p
    // values; each pivot's factor row (with the row's state) is loaded ahead
    // of its use through a ring of row buffers
    struct FRow {
        cplx<FT> it[IT];  // items 0..p-1 l, p dinv, p+1 yhat, p+2..2p+1 f
        cplx<double> c, d;
    };
    auto load_frow = [&](int j) {
        // j < 0 (past the last pivot) reloads pivot 0; the row is not used
        const int jj = j < 0 ? 0 : j;
        FRow r;
#pragma unroll
        for (int it = 0; it < IT; ++it) r.it[it] = fitem(jj, it);
        load_sd(jj, r.c, r.d);
        return r;
    };
    cplx<FT> xw[PP + 1];
#pragma unroll
    for (int t = 0; t <= PP; ++t) xw[t] = cmk<FT>(0, 0);
    auto back_row = [&](int j, const FRow& fr, cplx<FT> ucorr) {
        cplx<FT> yh = csub(fr.it[PP + 1], ucorr);
#pragma unroll
        for (int t = 0; t < PP; ++t) yh = cfms(yh, fr.it[PP + 2 + t], xl[t]);
        cplx<FT> xj = cmul(fr.it[PP], yh);
#pragma unroll
        for (int i = 1; i <= PP; ++i) xj = cfms(xj, fr.it[i - 1], xw[i]);
#pragma unroll
        for (int i = PP; i >= 2; --i) xw[i] = xw[i - 1];
        xw[1] = xj;
        update(j, xj, fr.c, fr.d);
    };
    // Pivots are visited in order j = m-1, m-2, ..., 0; the one with ordinal
    // t = m-1-j uses ring slot t % kRing, which is refilled with the pivot
    // kRing further on right after its use.  Slot indices are compile-time
    // constants (no register moves) and kRing - 1 rows stay in flight (two
    // for FP64, whose rows are twice the size).
    constexpr int kRing = sizeof(FT) == 4 ? 4 : 3;
    FRow fr[kRing];
#pragma unroll
    for (int t = 0; t < kRing; ++t) fr[t] = load_frow(m - 1 - t);
#pragma unroll
    for (int q = PP - 1; q >= 0; --q) {
        const int t = PP - 1 - q;
        back_row(m - PP + q, fr[t % kRing], ur[q]);
        fr[t % kRing] = load_frow(m - 1 - t - kRing);
    }
    int j = m - PP - 1;
    for (; j >= kRing - 1; j -= kRing) {
#pragma unroll
        for (int u = 0; u < kRing; ++u) {
            back_row(j - u, fr[(PP + u) % kRing], cmk<FT>(0, 0));
            fr[(PP + u) % kRing] = load_frow(j - u - kRing);
        }
    }
#pragma unroll
    for (int u = 0; u + 1 < kRing; ++u)
        if (j - u >= 0) back_row(j - u, fr[(PP + u) % kRing], cmk<FT>(0, 0));
#pragma unroll
    for (int t = 0; t < PP; ++t) update(m + t, xr[t], sepc[t], sepd[t]);
}

// FP64 band entry of the refinement residual from its FP32 rounding and the
// 8-bit code of diagonal d in `codes` (see kLoScale).
__device__ __forceinline__ double band_entry(float hi, unsigned long long codes, int d) {
    const int q = (int)(signed char)(unsigned char)(codes >> (8 * d));
    return (double)hi * fma((double)q, kLoScale, 1.0);
}

// Pass C (refinement sweep): residual of the current iterate in FP64,
//   r = B c_n - A c = -S dtot - i a H (2 c - dtot),   dtot = c - c_n,
// from S, H0, D to within 2^-32 of their FP64 entries (the FP32 bands and
// an 8-bit correction per entry: 5 instead of 8 bytes), so the sweeps
// converge to the Crank-Nicolson step of bands that differ from the FP64
// ones by less than 2.4e-10 relative, then forward substitution with the
// stored factor rows (yhat, and the chunk's separator right-hand sides
// yR, gT).  The absorber W (extended kernels) is read in FP64.
template <int PP, typename FT, bool XT = false>
__device__ __forceinline__ void pass_residual(const SysDesc& sd, int k, const FT* __restrict__ band,
                              const double* __restrict__ band64, const unsigned long long* __restrict__ bandlo,
                              const double* __restrict__ st,
                              const double* __restrict__ dtot, FT* __restrict__ fac,
                              FT* __restrict__ red, double alpha, double Ebar, double nrm[2]) {
    static_assert(sizeof(FT) == 4, "the refinement residual belongs to the FP32 factorisation");
    const bool cap = XT && sd.cap != 0;
    constexpr int NM = kNumMats;
    constexpr int IT = 2 * PP + 2;
    const int L = sd.L, LS = sd.LS, P = sd.P;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const int kk = col - 1;
    const FT* __restrict__ bnd = band + sd.band_off;
    const double* __restrict__ bnd64 = band64 + sd.band_off;
    const unsigned long long* __restrict__ blo = bandlo + 3 * sd.state_off;
    const double* __restrict__ cst = st + 2 * sd.state_off;
    const double* __restrict__ dst = dtot + 2 * sd.state_off;
    FT* __restrict__ fc = fac + 2 * sd.fac_off;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
    const unsigned fstride = (unsigned)(IT * P);
    auto fitem = [&](int j, int item) {
        return ld_c(fc, (unsigned)j * fstride + (unsigned)(item * P) + (unsigned)kk);
    };
    // windows of v = 2c - dtot and of dtot: slot PP is the newest row
    cplx<double> vw[PP + 1], dw[PP + 1], hacc[PP + 1], sacc[PP + 1];
    cplx<double> wacc[XT ? PP + 1 : 1];  // pending (W v) (absorber)
    cplx<FT> y[PP + 1];
    cplx<FT> gT[PP];
#pragma unroll
    for (int i = 0; i <= PP; ++i) {
        hacc[i] = cmk<double>(0, 0);
        sacc[i] = cmk<double>(0, 0);
        y[i] = cmk<FT>(0, 0);
    }
#pragma unroll
    for (int i = 0; i < (XT ? PP + 1 : 1); ++i) wacc[i] = cmk<double>(0, 0);
    // squared norms of the residual and of its two terms (S dtot and
    // a (W + i H) v), the scale of the relative residual
    double rn2 = 0.0, ref2 = 0.0;
#pragma unroll
    for (int t = 0; t < PP; ++t) gT[t] = cmk<FT>(0, 0);
    vw[0] = dw[0] = cmk<double>(0, 0);
#pragma unroll
    for (int d = 0; d < PP; ++d) {
        unsigned at = (unsigned)(L - PP + d) * (unsigned)LS + (unsigned)(col - 1);
        cplx<double> c = cmk<double>(cst[2 * at], cst[2 * at + 1]);
        cplx<double> dd = cmk<double>(dst[2 * at], dst[2 * at + 1]);
        dw[d + 1] = dd;
        vw[d + 1] = cmk<double>(2.0 * c.re - dd.re, 2.0 * c.im - dd.im);
    }
    // streamed row r (0 <= r < L + p; rows >= L are the next chunk's halo),
    // loaded one row ahead of its use
    struct RowIn {
        float bS[PP + 1], bH[PP + 1], bD[PP + 1];
        unsigned long long qS, qH, qD;
        double bW[XT ? PP + 1 : 1];
        cplx<double> c, dd;
    };
    auto load_row = [&](int r) {
        if (r >= L + PP) r = L + PP - 1;  // past the end: reload the last row (unused)
        const bool own = r < L;
        const int lr = own ? r : r - L;
        const unsigned cc = (unsigned)(own ? col : col + 1);
        const unsigned rb = (unsigned)lr * rowstride + cc;
        const unsigned lb = (unsigned)lr * (unsigned)(3 * LS) + cc;
        RowIn in;
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            in.bS[d] = bnd[rb + (unsigned)((0 * (PP + 1) + d) * LS)];
            in.bH[d] = bnd[rb + (unsigned)((1 * (PP + 1) + d) * LS)];
            in.bD[d] = bnd[rb + (unsigned)((2 * (PP + 1) + d) * LS)];
        }
        in.qS = blo[lb];
        in.qH = blo[lb + (unsigned)LS];
        in.qD = blo[lb + 2u * (unsigned)LS];
        if constexpr (XT) {
#pragma unroll
            for (int d = 0; d <= PP; ++d) in.bW[d] = cap ? bnd64[rb + (unsigned)((kMatW * (PP + 1) + d) * LS)] : 0.0;
        }
        const unsigned sat = (unsigned)lr * (unsigned)LS + cc;
        in.c = cmk<double>(cst[2 * sat], cst[2 * sat + 1]);
        in.dd = cmk<double>(dst[2 * sat], dst[2 * sat + 1]);
        return in;
    };
    // count: the completed row r - p is a row of this chunk (r >= p)
    auto stream_row = [&](const RowIn& in, bool own, bool count) {
        double h[PP + 1], sb[PP + 1];
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            sb[d] = band_entry(in.bS[d], in.qS, d);
            h[d] = band_entry(in.bH[d], in.qH, d) + Ebar * band_entry(in.bD[d], in.qD, d);
        }
#pragma unroll
        for (int d = 0; d < PP; ++d) {
            vw[d] = vw[d + 1];
            dw[d] = dw[d + 1];
            hacc[d] = hacc[d + 1];
            sacc[d] = sacc[d + 1];
        }
        dw[PP] = in.dd;
        vw[PP] = cmk<double>(2.0 * in.c.re - in.dd.re, 2.0 * in.c.im - in.dd.im);
        cplx<double> hs = cmk<double>(0, 0), ss = cmk<double>(0, 0);
        if (own) {
#pragma unroll
            for (int d = 0; d <= PP; ++d) {
                hs.re += h[d] * vw[PP - d].re;
                hs.im += h[d] * vw[PP - d].im;
                ss.re += sb[d] * dw[PP - d].re;
                ss.im += sb[d] * dw[PP - d].im;
            }
        }
        hacc[PP] = hs;
        sacc[PP] = ss;
#pragma unroll
        for (int d = 1; d <= PP; ++d) {
            hacc[PP - d].re += h[d] * vw[PP].re;
            hacc[PP - d].im += h[d] * vw[PP].im;
            sacc[PP - d].re += sb[d] * dw[PP].re;
            sacc[PP - d].im += sb[d] * dw[PP].im;
        }
        // completed residual of row r - p: -S dtot - a (W + i H) v
        double tr = -alpha * hacc[0].im, ti = alpha * hacc[0].re;  // i a H v
        if constexpr (XT) {
#pragma unroll
            for (int d = 0; d < PP; ++d) wacc[d] = wacc[d + 1];
            cplx<double> ws = cmk<double>(0, 0);
            if (own) {
#pragma unroll
                for (int d = 0; d <= PP; ++d) {
                    ws.re += in.bW[d] * vw[PP - d].re;
                    ws.im += in.bW[d] * vw[PP - d].im;
                }
            }
            wacc[PP] = ws;
#pragma unroll
            for (int d = 1; d <= PP; ++d) {
                wacc[PP - d].re += in.bW[d] * vw[PP].re;
                wacc[PP - d].im += in.bW[d] * vw[PP].im;
            }
            tr += alpha * wacc[0].re;
            ti += alpha * wacc[0].im;
        }
        const double rr = -sacc[0].re - tr, ri = -sacc[0].im - ti;
        if (count) {
            rn2 += rr * rr + ri * ri;
            ref2 += sacc[0].re * sacc[0].re + sacc[0].im * sacc[0].im + tr * tr + ti * ti;
        }
        return cmk<FT>((FT)rr, (FT)ri);
    };
    auto shift_y = [&]() {
#pragma unroll
        for (int i = 1; i <= PP; ++i) y[i - 1] = y[i];
        y[PP] = cmk<FT>(0, 0);
    };
    // factor row of pivot j (l, dinv, f), loaded one pivot ahead
    struct FRow {
        cplx<FT> l[PP], dinv, f[PP];
    };
    auto load_frow = [&](int j) {
        if (j > sd.m - 1) j = sd.m - 1;
        FRow fr;
#pragma unroll
        for (int i = 0; i < PP; ++i) fr.l[i] = fitem(j, i);
        fr.dinv = fitem(j, PP);
#pragma unroll
        for (int t = 0; t < PP; ++t) fr.f[t] = fitem(j, PP + 2 + t);
        return fr;
    };
    // band/state rows two ahead, factor rows one ahead of their use
    RowIn cur = load_row(0);
    RowIn nx1 = load_row(1);
#pragma unroll
    for (int r = 0; r < PP; ++r) {
        RowIn nx2 = load_row(r + 2);
        (void)stream_row(cur, true, false);
        shift_y();
        cur = nx1;
        nx1 = nx2;
    }
    FRow fcur = load_frow(0);
    for (int r = PP; r < L; ++r) {
        RowIn nx2 = load_row(r + 2);
        FRow fnxt = load_frow(r - PP + 1);
        const int j = r - PP;
        cplx<FT> yj = cadd(y[0], stream_row(cur, true, true));
        const unsigned fb = (unsigned)j * fstride + (unsigned)kk;
        st_c(fc, fb + (unsigned)((PP + 1) * P), yj);
#pragma unroll
        for (int i = 1; i <= PP; ++i) y[i] = cfms(y[i], fcur.l[i - 1], yj);
#pragma unroll
        for (int t = 0; t < PP; ++t) gT[t] = cfms(gT[t], cmul(fcur.f[t], fcur.dinv), yj);
        shift_y();
        cur = nx1;
        nx1 = nx2;
        fcur = fnxt;
    }
#pragma unroll
    for (int t = 0; t < PP; ++t) {
        RowIn nx2 = load_row(L + t + 2);
        y[t] = cadd(y[t], stream_row(cur, false, true));
        cur = nx1;
        nx1 = nx2;
    }
    FT* rb = red + 2 * (sd.red_off + (long long)k * RedLayout<FT>::chunk_block(PP));
    const int pp = PP * PP;
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        st_c(rb, (unsigned)(3 * pp + i), y[i]);
        st_c(rb, (unsigned)(3 * pp + PP + i), gT[i]);
    }
    nrm[0] = rn2;
    nrm[1] = ref2;
}

// Extended per-step series (the time series of section V.D) of c_n from
// the FP64 bands: one lane's partial sums over its chunk rows, each pair of
// rows (r, r-d) counted by the owner of row r:
//   xs[0] c^H H0 c    xs[1] c^H V c    xs[2] c^H Mi c
//   xs[3] <v> = sum K[r][r-d] Im(conj(c_r) c_{r-d})   (eq. vel_elem, Vel = -(i/2) K)
//   xs[4] c^H Q c (a_Q)    xs[5] c^H W c (absorber)
//   xs[6], xs[7] Re, Im of c_0^H S c (autocorrelation, M-weighted overlap)
//   xs[8 + 2k], xs[9 + 2k] Re, Im of (S phi_k)^T c (projection on state k)
constexpr int kExtSums = 8 + 2 * kMaxPop;
template <int PP>
__device__ __forceinline__ void pass_extobs(const SysDesc& sd, int k, const double* __restrict__ band64,
                                            const double* __restrict__ st, const double* __restrict__ c0,
                                            const double* __restrict__ proj, double xs[kExtSums]) {
    constexpr int NM = kNumMats;
    const int L = sd.L, LS = sd.LS, npop = sd.npop;
    const bool aq = sd.aq != 0, cap = sd.cap != 0, autoc = c0 != nullptr;
    int col = k + 1;
    asm volatile("" : "+v"(col));
    const double* __restrict__ bnd = band64 + sd.band_off;
    const double* __restrict__ cst = st + 2 * sd.state_off;
    const double* __restrict__ zst = autoc ? c0 + 2 * sd.state_off : cst;
    const double* __restrict__ pj = proj ? proj + sd.proj_off : nullptr;
    const unsigned rowstride = (unsigned)(NM * (PP + 1) * LS);
#pragma unroll
    for (int i = 0; i < kExtSums; ++i) xs[i] = 0.0;
    cplx<double> cw[PP + 1], zw[PP + 1];  // c and c_0 rows r-p..r (slot PP newest)
    cw[0] = zw[0] = cmk<double>(0, 0);
#pragma unroll
    for (int d = 0; d < PP; ++d) {
        const unsigned at = (unsigned)(L - PP + d) * (unsigned)LS + (unsigned)(col - 1);
        cw[d + 1] = cmk<double>(cst[2 * at], cst[2 * at + 1]);
        zw[d + 1] = cmk<double>(zst[2 * at], zst[2 * at + 1]);
    }
    auto band = [&](unsigned rb, int mat, int d) { return bnd[rb + (unsigned)((mat * (PP + 1) + d) * LS)]; };
    for (int r = 0; r < L; ++r) {
        const unsigned at = (unsigned)r * (unsigned)LS + (unsigned)col;
        const cplx<double> cr = cmk<double>(cst[2 * at], cst[2 * at + 1]);
        const cplx<double> zr = cmk<double>(zst[2 * at], zst[2 * at + 1]);
#pragma unroll
        for (int d = 0; d < PP; ++d) {
            cw[d] = cw[d + 1];
            zw[d] = zw[d + 1];
        }
        cw[PP] = cr;
        zw[PP] = zr;
        const unsigned rb = (unsigned)r * rowstride + (unsigned)col;
#pragma unroll
        for (int d = 0; d <= PP; ++d) {
            const cplx<double> cd = cw[PP - d];
            const double wgt = d == 0 ? 1.0 : 2.0;
            const double o = wgt * (cr.re * cd.re + cr.im * cd.im);  // 2 Re conj(c_r) c_{r-d}
            xs[0] += band(rb, kMatH0, d) * o;
            xs[1] += band(rb, kMatV, d) * o;
            xs[2] += band(rb, kMatMi, d) * o;
            if (d > 0) xs[3] += band(rb, kMatK, d) * (cr.re * cd.im - cr.im * cd.re);
            if (aq) xs[4] += band(rb, kMatQ, d) * o;
            if (cap) xs[5] += band(rb, kMatW, d) * o;
            if (autoc) {
                // conj(z_r) c_{r-d} + conj(z_{r-d}) c_r (d > 0)
                const double sv = band(rb, kMatS, d);
                const cplx<double> zd = zw[PP - d];
                double are = zr.re * cd.re + zr.im * cd.im, aim = zr.re * cd.im - zr.im * cd.re;
                if (d > 0) {
                    are += zd.re * cr.re + zd.im * cr.im;
                    aim += zd.re * cr.im - zd.im * cr.re;
                }
                xs[6] += sv * are;
                xs[7] += sv * aim;
            }
        }
        for (int q = 0; q < npop; ++q) {
            const double ps = pj[((long long)q * L + r) * LS + col];
            xs[8 + 2 * q] += ps * cr.re;
            xs[9 + 2 * q] += ps * cr.im;
        }
    }
}

__device__ inline void latch(int* status, int code, int sys, int step) {
    if (atomicCAS(&status[0], 0, code) == 0) {
        status[1] = sys;
        status[2] = step;
    }
}



}  // namespace
}  // namespace tdsez
