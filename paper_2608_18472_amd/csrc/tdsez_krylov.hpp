// Pieces shared by the tensor-product propagators (2D and 3D, constant
// mass, x-polarised field): the vector kernels of conjugate-orthogonal CG,
// its device-side scalar schedule, the per-axis MFMA contractions of the
// fast-diagonalisation preconditioner, the per-axis generalised
// eigendecomposition, and the Crank-Nicolson step loop itself
// (section V.B in the increment form A_n Delta = -i dt H_n c_n).
//
// A tensor-product system supplies its own operator and preconditioner
// through an object with these members (FP64 and FP32 versions of the
// first two):
//   apply(in, y, w, a, b, Ebar, out, obs_part, flag, stream, dotp):
//       out = w y + a S c_in + b (H0 + Ebar D) c_in   (y optional),
//       with per-block partial sums of Re c^H S c and Re c^H D c when
//       obs_part is given, or of c_in^T out when dotp is given;
//   precond(in, out, flag, stream, rzp): out = P^-1 in, P the separable
//       part, with per-block partial sums of in^T out when rzp is given;
//   nblk_apply(fp32), nblk_precond(): the number of those partial sums;
//   accel(in, part, stream): per-block partial sums of Re c^H G c for the
//       acceleration (G the force stencil of dV/dx); returns their number,
//       0 when the system has no force stencil;
// apply and precond return at once when *flag is set (the solve has
// converged).
// Complex vectors are planar (real plane, then imaginary plane).
//
// Everything here has internal linkage: each translation unit that
// includes the header gets its own kernels.
#pragma once
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tdsez_internal.hpp"

namespace tdsez {

__global__ void basis_kernel(const double* __restrict__ br, int nbr, int p, int nq,
                             const double* __restrict__ xq, double* __restrict__ Bv,
                             double* __restrict__ dB);

namespace {

// M[i][j] of a 1D lower half band by rows (band[j*(p+1) + d] = M[j][j-d])
__device__ inline double band_ij(const double* __restrict__ band, int p, int i, int j) {
    const int hi = i > j ? i : j;
    const int d = i > j ? i - j : j - i;
    return band[hi * (p + 1) + d];
}

// lower half band by rows -> dense symmetric (column-major = row-major)
__global__ void band_to_dense_kernel(const double* __restrict__ band, int N, int p, double* __restrict__ out) {
    const long long total = (long long)N * N;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / N), j = (int)(e % N);
        const int d = i > j ? i - j : j - i;
        out[e] = d <= p ? band_ij(band, p, i, j) : 0.0;
    }
}

// natural interleaved complex <-> planar
__global__ void to_planar_kernel(const double* __restrict__ z, long long n, double* __restrict__ re,
                                 double* __restrict__ im) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        re[e] = z[2 * e];
        im[e] = z[2 * e + 1];
    }
}
__global__ void from_planar_kernel(const double* __restrict__ re, const double* __restrict__ im, long long n,
                                   double* __restrict__ z) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        z[2 * e] = re[e];
        z[2 * e + 1] = im[e];
    }
}

// M[i][j] of a 1D lower half band by rows, for |i - j| <= p; pairs with an
// index outside 0..n-1 give 0 (the load index is clamped, so no branch)
template <typename FT>
__device__ inline FT band_at(const FT* __restrict__ band, int p, int n, int i, int j) {
    const bool ok = i >= 0 && i < n && j >= 0 && j < n;
    const int hi = i > j ? i : j;
    const int d = i > j ? i - j : j - i;
    const FT v = band[ok ? hi * (p + 1) + d : 0];
    return ok ? v : FT(0);
}

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 512;

// partial sums over blocks: sum u v (complex, unconjugated) or sum |u|^2,
// accumulated in FP64 whatever the storage precision
template <typename FT>
__global__ __launch_bounds__(kRedThreads) void dot_kernel(long long n, const FT* __restrict__ ur,
                                                          const FT* __restrict__ ui, const FT* __restrict__ vr,
                                                          const FT* __restrict__ vi, bool abs2,
                                                          double* __restrict__ part, const double* __restrict__ flag) {
    if (flag && *flag != 0.0) return;
    __shared__ double sr[kRedThreads], si[kRedThreads];
    double ar = 0.0, ai = 0.0;
    for (long long e = blockIdx.x * (long long)kRedThreads + threadIdx.x; e < n; e += (long long)gridDim.x * kRedThreads) {
        const double a = ur[e], b = ui[e];
        if (abs2) {
            ar += a * a + b * b;
        } else {
            const double c = vr[e], d = vi[e];
            ar += a * c - b * d;
            ai += a * d + b * c;
        }
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sr[threadIdx.x] += sr[threadIdx.x + s];
            si[threadIdx.x] += si[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sr[0];
        part[2 * blockIdx.x + 1] = si[0];
    }
}

// c += x (x in FT, c in FP64)
template <typename FT>
__global__ void add_kernel(long long n, const FT* __restrict__ xr, const FT* __restrict__ xi,
                           double* __restrict__ cr, double* __restrict__ ci, const double* __restrict__ flag) {
    if (flag && *flag != 0.0) return;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        cr[e] += (double)xr[e];
        ci[e] += (double)xi[e];
    }
}

// r = b - q (q in FP32, r and b in FP64; planar, 2n values)
__global__ void sub32_kernel(long long n2, const double* __restrict__ b, const float* __restrict__ q,
                             double* __restrict__ r) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n2; e += (long long)gridDim.x * blockDim.x)
        r[e] = b[e] - (double)q[e];
}

// FP64 -> FP32 copy
__global__ void to_fp32_kernel(long long n, const double* __restrict__ src, float* __restrict__ dst,
                               const double* __restrict__ flag = nullptr) {
    if (flag && *flag != 0.0) return;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        dst[e] = (float)src[e];
}

// dst = src, or 0 with src == nullptr (a fill kernel rather than a memset,
// so that a step stays free of memset nodes)
template <typename FT>
__global__ void copy_kernel(long long n, const FT* __restrict__ src, FT* __restrict__ dst,
                            const double* __restrict__ flag) {
    if (flag && *flag != 0.0) return;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        dst[e] = src ? src[e] : FT(0);
}

// ------------------------------------------------------------ per-axis transforms
// The preconditioner's four per-axis transforms are dense contractions of a
// planar complex vector (two Ny x Nx row-major planes) with the per-axis
// eigenvector matrices, so they run on the matrix cores: one workgroup of
// four waves per 32 x 32 output tile and both planes, K in chunks of 32
// staged through LDS (next chunk prefetched into registers while the
// current one is multiplied), each wave one 16 x 16 sub-tile per plane by
// 16x16x4 MFMA steps (FP64: v_mfma_f64_16x16x4_f64, FP32:
// v_mfma_f32_16x16x4_f32).  MFMA operand layout of one step: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; element r of the 16 x 16
// accumulator is C[4 (l / 16) + r][l % 16] in FP32 and C[l / 16 + 4 r][l % 16]
// in FP64 (the row interleave differs between the two instructions).
//   LEFTQ = false: C = V Bq, V the vector (M x K row-major, ld K), Bq(k, n) =
//     Q[k qs0 + n qs1];
//   LEFTQ = true:  C = Aq V, Aq(m, k) = Q[m qs0 + k qs1], V (K x N row-major).
// C is M x N row-major (ld N); blockIdx.z runs over a batch of such
// products (3D: the y transforms of every z plane).  SCALE divides the
// result by c0 + c1 L, L the sum of the per-axis eigenvalues of the entry
// (the diagonal of the separable part in the eigenbasis; Crank-Nicolson:
// c0 = 1, c1 = i a), which needs both planes of an entry: every workgroup
// computes both.  flag != nullptr and *flag != 0 skips the launch.
constexpr int kGemmTile = 32, kGemmKc = 32, kGemmThreads = 256;
template <typename FT>
struct MfmaOps;
template <>
struct MfmaOps<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ inline acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // accumulator row of element r in lane group g = lane / 16
    static __device__ inline int row(int g, int r) { return g + 4 * r; }
};
template <>
struct MfmaOps<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ inline acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int g, int r) { return 4 * g + r; }
};

struct FdmScale {
    double c0r, c0i, c1r, c1i;       // the divisor c0 + c1 L
    const double* mu_m;              // L = mu_m[m] + lam_n[n % nx] (+ lam_hi[n / nx])
    const double* lam_n;
    const double* lam_hi;
    int nx;
};
// DOT (the last contraction of a preconditioner application z = P^-1 r):
// the workgroup also writes the partial sum of r^T z over its tile
// (unconjugated, FP64) to part[2 b], part[2 b + 1], b its block index,
// reading r (dr, di: same layout as the result) at the tile's entries.
template <typename FT, bool LEFTQ, bool SCALE, bool DOT = false>
__global__ __launch_bounds__(kGemmThreads) void fdm_gemm_kernel(
    int M, int N, int K, const FT* __restrict__ Q, int qs0, int qs1, const FT* __restrict__ vr,
    const FT* __restrict__ vi, FT* __restrict__ cr, FT* __restrict__ ci, long long vbs, long long cbs,
    FdmScale sc, const double* __restrict__ flag, const FT* __restrict__ dr = nullptr,
    const FT* __restrict__ di = nullptr, double* __restrict__ part = nullptr) {
    if (flag && *flag != 0.0) return;
    // batch blockIdx.z: the vector operand and the result advance by vbs, cbs
    vr += blockIdx.z * vbs;
    vi += blockIdx.z * vbs;
    cr += blockIdx.z * cbs;
    ci += blockIdx.z * cbs;
    constexpr int T = kGemmTile, KC = kGemmKc, NT = kGemmThreads;
    constexpr int PA = KC + 1, PB = T + 1;  // padded pitches
    // A chunk T x KC, B chunk KC x T; the vector operand has two planes
    __shared__ FT As[LEFTQ ? 1 : 2][T][PA];
    __shared__ FT Bs[LEFTQ ? 2 : 1][KC][PB];
    typedef typename MfmaOps<FT>::acc_t acc_t;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * T, n0 = blockIdx.x * T;
    const int wm = (wave >> 1) * 16, wn = (wave & 1) * 16;
    acc_t acc[2];
    for (int p = 0; p < 2; ++p)
        for (int r = 0; r < 4; ++r) acc[p][r] = FT(0);
    constexpr int PER = T * KC / NT;  // elements of one chunk per thread
    FT ra[LEFTQ ? 1 : 2][PER], rb[LEFTQ ? 2 : 1][PER];
    // global loads of chunk k0 into registers, the fastest index along the
    // operand's contiguous direction
    auto load = [&](int k0) {
        for (int t = 0; t < PER; ++t) {
            const int e = tid + NT * t;
            if constexpr (!LEFTQ) {
                {   // A = V (row-major, k contiguous): e -> (m, k)
                    const int m = e / KC, k = e % KC;
                    const int gm = m0 + m, gk = k0 + k;
                    const bool ok = gm < M && gk < K;
                    const long long at = ok ? (long long)gm * K + gk : 0;
                    ra[0][t] = ok ? vr[at] : FT(0);
                    ra[1][t] = ok ? vi[at] : FT(0);
                }
                {   // B = Q
                    int k, n;
                    if (qs0 == 1) { k = e % KC; n = e / KC; }
                    else { n = e % T; k = e / T; }
                    const int gk = k0 + k, gn = n0 + n;
                    const bool ok = gk < K && gn < N;
                    rb[0][t] = ok ? Q[(long long)gk * qs0 + (long long)gn * qs1] : FT(0);
                }
            } else {
                {   // A = Q
                    int m, k;
                    if (qs1 == 1) { m = e / KC; k = e % KC; }
                    else { k = e / T; m = e % T; }
                    const int gm = m0 + m, gk = k0 + k;
                    const bool ok = gm < M && gk < K;
                    ra[0][t] = ok ? Q[(long long)gm * qs0 + (long long)gk * qs1] : FT(0);
                }
                {   // B = V (row-major, n contiguous): e -> (k, n)
                    const int k = e / T, n = e % T;
                    const int gk = k0 + k, gn = n0 + n;
                    const bool ok = gk < K && gn < N;
                    const long long at = ok ? (long long)gk * N + gn : 0;
                    rb[0][t] = ok ? vr[at] : FT(0);
                    rb[1][t] = ok ? vi[at] : FT(0);
                }
            }
        }
    };
    auto stash = [&]() {
        for (int t = 0; t < PER; ++t) {
            const int e = tid + NT * t;
            if constexpr (!LEFTQ) {
                const int m = e / KC, k = e % KC;
                As[0][m][k] = ra[0][t];
                As[1][m][k] = ra[1][t];
                int kb, nb;
                if (qs0 == 1) { kb = e % KC; nb = e / KC; }
                else { nb = e % T; kb = e / T; }
                Bs[0][kb][nb] = rb[0][t];
            } else {
                int m, k;
                if (qs1 == 1) { m = e / KC; k = e % KC; }
                else { k = e / T; m = e % T; }
                As[0][m][k] = ra[0][t];
                const int kb = e / T, nb = e % T;
                Bs[0][kb][nb] = rb[0][t];
                Bs[1][kb][nb] = rb[1][t];
            }
        }
    };
    const int li = lane & 15, lk = lane >> 4;
    load(0);
    for (int k0 = 0; k0 < K; k0 += KC) {
        __syncthreads();  // the previous chunk's reads are done
        stash();
        __syncthreads();
        if (k0 + KC < K) load(k0 + KC);  // in flight during the products
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            if constexpr (!LEFTQ) {
                const FT b = Bs[0][kk + lk][wn + li];
                acc[0] = MfmaOps<FT>::step(As[0][wm + li][kk + lk], b, acc[0]);
                acc[1] = MfmaOps<FT>::step(As[1][wm + li][kk + lk], b, acc[1]);
            } else {
                const FT a = As[0][wm + li][kk + lk];
                acc[0] = MfmaOps<FT>::step(a, Bs[0][kk + lk][wn + li], acc[0]);
                acc[1] = MfmaOps<FT>::step(a, Bs[1][kk + lk][wn + li], acc[1]);
            }
        }
    }
    const int gn = n0 + wn + li;
    double pr = 0.0, pi = 0.0;
    for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + MfmaOps<FT>::row(lk, r);
        if (gm >= M || gn >= N) continue;
        FT a = acc[0][r], b = acc[1][r];
        if constexpr (SCALE) {
            double L = sc.mu_m[gm] + sc.lam_n[gn % sc.nx];
            if (sc.lam_hi) L += sc.lam_hi[gn / sc.nx];
            const double er = sc.c0r + sc.c1r * L, ei = sc.c0i + sc.c1i * L;
            const double s = 1.0 / (er * er + ei * ei);
            const double ad = a, bd = b;
            a = (FT)((ad * er + bd * ei) * s);
            b = (FT)((bd * er - ad * ei) * s);
        }
        const long long at = (long long)gm * N + gn;
        cr[at] = a;
        ci[at] = b;
        if constexpr (DOT) {
            const double xr = dr[blockIdx.z * cbs + at], xi = di[blockIdx.z * cbs + at];
            pr += xr * (double)a - xi * (double)b;
            pi += xr * (double)b + xi * (double)a;
        }
    }
    if constexpr (DOT) {
        __shared__ double red[2][kGemmThreads];
        red[0][tid] = pr;
        red[1][tid] = pi;
        __syncthreads();
        for (int s2 = kGemmThreads / 2; s2 > 0; s2 >>= 1) {
            if (tid < s2) {
                red[0][tid] += red[0][tid + s2];
                red[1][tid] += red[1][tid + s2];
            }
            __syncthreads();
        }
        if (tid == 0) {
            const long long b = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            part[2 * b] = red[0][0];
            part[2 * b + 1] = red[1][0];
        }
    }
}


// observables: sum the per-block partials of apply_kernel (fixed order per
// thread, then a tree over the block: deterministic)
// The observables of c_n from the operator's per-block partials (norm and
// dipole) and, where the system has the force stencil G (apart != null), the
// acceleration a = -Re c^H G c - E_n nu (section IV.A, constant mass).
__global__ __launch_bounds__(kRedThreads) void obs_finish_kernel(const double* __restrict__ part, int nblk,
                                                                 const double* __restrict__ apart, int nblk_a,
                                                                 double En, double* __restrict__ out,
                                                                 unsigned mask) {
    __shared__ double a[kRedThreads], b[kRedThreads], g[kRedThreads];
    double nu = 0.0, d = 0.0, f = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kRedThreads) {
        nu += part[2 * k];
        d += part[2 * k + 1];
    }
    for (int k = threadIdx.x; apart && k < nblk_a; k += kRedThreads) f += apart[k];
    a[threadIdx.x] = nu;
    b[threadIdx.x] = d;
    g[threadIdx.x] = f;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            a[threadIdx.x] += a[threadIdx.x + s];
            b[threadIdx.x] += b[threadIdx.x + s];
            g[threadIdx.x] += g[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (mask & TDSEZ_OBS_NORM) ? a[0] : 0.0;
        out[1] = (mask & TDSEZ_OBS_DIPOLE) ? b[0] : 0.0;
        out[2] = (apart && (mask & TDSEZ_OBS_ACCEL)) ? -g[0] - En * a[0] : 0.0;
    }
}

// COCG scalars on the device, one slot block per solve level (FP64 solve /
// outer refinement, FP32 inner solve): sc[0..1] rho, sc[2..3] alpha,
// sc[4..5] beta, sc[6] |r|^2, sc[7] |b|^2, sc[8] converged flag, sc[9]
// iterations (of the step; of the current sweep for the inner block),
// sc[10] squared relative tolerance, sc[11] refinement sweeps of the step,
// inner block only: sc[12] largest and sc[13] total inner iterations of the
// step's sweeps, sc[16 + s] the inner iterations of sweep s < kLogSweeps.
// One block sums the partials of the last
// dot (fixed order) and updates the scalars for `mode`:
//   0: rho = sum          1: alpha = rho / sum
//   2: beta = sum / rho, rho = sum
//   3: |r|^2 = sum (one more iteration when `count`); converged when
//      |r|^2 <= sc[10] |b|^2
//   4: |b|^2 = sum
enum { kScRho = 0, kScAlpha = 2, kScBeta = 4, kScR2 = 6, kScB2 = 7, kScDone = 8, kScIts = 9, kScTol2 = 10,
       kScSweeps = 11, kScItsMax = 12, kScItsSum = 13, kScSweepIts = 16, kScBlock = 24 };
// Refinement sweeps whose inner iteration counts are logged per step, and the
// ints of the per-step log: FP64 iterations, largest inner iterations of a
// sweep, sweeps, total inner iterations, then one count per logged sweep.
constexpr int kLogSweeps = 4, kLogStride = 4 + kLogSweeps;
__global__ __launch_bounds__(kRedThreads) void cocg_scalar_kernel(const double* __restrict__ part, int nblk,
                                                                  int mode, double* __restrict__ sc, bool count) {
    if (sc[kScDone] != 0.0) return;
    __shared__ double a[kRedThreads], b[kRedThreads];
    double re = 0.0, im = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kRedThreads) {
        re += part[2 * k];
        im += part[2 * k + 1];
    }
    a[threadIdx.x] = re;
    b[threadIdx.x] = im;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            a[threadIdx.x] += a[threadIdx.x + s];
            b[threadIdx.x] += b[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double sr = a[0], si = b[0];
    if (mode == 0) {
        sc[0] = sr;
        sc[1] = si;
    } else if (mode == 1) {
        // a zero p^T q only arises with a zero residual (exact start): no step
        const double den = sr * sr + si * si;
        sc[2] = den > 0.0 ? (sc[0] * sr + sc[1] * si) / den : 0.0;
        sc[3] = den > 0.0 ? (sc[1] * sr - sc[0] * si) / den : 0.0;
    } else if (mode == 2) {
        const double den = sc[0] * sc[0] + sc[1] * sc[1];
        sc[4] = den > 0.0 ? (sr * sc[0] + si * sc[1]) / den : 0.0;
        sc[5] = den > 0.0 ? (si * sc[0] - sr * sc[1]) / den : 0.0;
        sc[0] = sr;
        sc[1] = si;
    } else if (mode == 3) {
        sc[kScR2] = sr;
        const double bn = sc[kScB2] > 0.0 ? sc[kScB2] : 1.0;
        if (count) sc[kScIts] += 1.0;
        if (sr <= sc[kScTol2] * bn) sc[kScDone] = 1.0;
    } else {
        sc[kScB2] = sr;
    }
}

// Start of a refinement sweep (FP32 inner solve of A e = r): the inner
// solve is skipped when the outer residual has converged; its relative
// target is the FP32 floor kInner, or less work when that already reaches
// the outer tolerance.
__global__ void sweep_start_kernel(double* __restrict__ outer, double* __restrict__ inner, double kInner) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    // fold the previous sweep's inner iterations into the step's counts
    const int prev = (int)outer[kScSweeps] - 1;
    if (prev >= 0 && prev < kLogSweeps) inner[kScSweepIts + prev] = fmax(inner[kScSweepIts + prev], inner[kScIts]);
    inner[kScItsMax] = fmax(inner[kScItsMax], inner[kScIts]);
    inner[kScItsSum] += inner[kScIts];
    inner[kScIts] = 0.0;
    const bool done = outer[kScDone] != 0.0;
    inner[kScDone] = done ? 1.0 : 0.0;
    if (done) return;
    outer[kScSweeps] += 1.0;
    const double bn = outer[kScB2] > 0.0 ? outer[kScB2] : 1.0;
    const double r2 = outer[kScR2] > 0.0 ? outer[kScR2] : 1e-300;
    const double t2 = 0.25 * outer[kScTol2] * bn / r2;
    inner[kScTol2] = t2 > kInner * kInner ? t2 : kInner * kInner;
}

// End of a step: an unconverged solve latches ENOCONV (first step only);
// the step's counts (kLogStride ints) go to the host-visible log; the flags
// and counters are reset for the next step.
__global__ void step_end_kernel(double* __restrict__ outer, double* __restrict__ inner, int step,
                                int* __restrict__ status, int* __restrict__ log) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (outer[kScDone] == 0.0 && status[0] == 0) {
        status[0] = TDSEZ_ENOCONV;
        status[1] = step;
    }
    const int last = (int)outer[kScSweeps] - 1;
    if (last >= 0 && last < kLogSweeps) inner[kScSweepIts + last] = fmax(inner[kScSweepIts + last], inner[kScIts]);
    int* lg = log + (size_t)kLogStride * step;
    lg[1] = (int)fmax(inner[kScItsMax], inner[kScIts]);
    lg[2] = (int)outer[kScSweeps];
    lg[3] = (int)(inner[kScItsSum] + inner[kScIts]);
    for (int k = 0; k < kLogSweeps; ++k) {
        lg[4 + k] = (int)inner[kScSweepIts + k];
        inner[kScSweepIts + k] = 0.0;
    }
    // written last: the host takes a non-negative entry 0 as "the row is complete"
    __threadfence_system();
    lg[0] = (int)outer[kScIts];
    outer[kScDone] = 0.0;
    outer[kScIts] = 0.0;
    outer[kScSweeps] = 0.0;
    inner[kScIts] = 0.0;
    inner[kScItsMax] = 0.0;
    inner[kScItsSum] = 0.0;
}

// x += al p, r -= al q with al = sc[2..3]
template <typename FT>
__global__ void cocg_xr_dev_kernel(long long n, const double* __restrict__ sc, const FT* __restrict__ pr,
                                   const FT* __restrict__ pi, const FT* __restrict__ qr, const FT* __restrict__ qi,
                                   FT* __restrict__ xr, FT* __restrict__ xi, FT* __restrict__ rr,
                                   FT* __restrict__ ri) {
    if (sc[kScDone] != 0.0) return;
    const FT alr = (FT)sc[2], ali = (FT)sc[3];
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        xr[e] += alr * pr[e] - ali * pi[e];
        xi[e] += alr * pi[e] + ali * pr[e];
        rr[e] -= alr * qr[e] - ali * qi[e];
        ri[e] -= alr * qi[e] + ali * qr[e];
    }
}

// x += al p, r -= al q with al = sc[2..3], and the partial sums of |r|^2
// (FP64) per block into part[2 b] (part[2 b + 1] = 0); grid kRedBlocks
template <typename FT>
__global__ __launch_bounds__(kRedThreads) void cocg_xr_norm_kernel(long long n, const double* __restrict__ sc,
                                                                   const FT* __restrict__ pr, const FT* __restrict__ pi,
                                                                   const FT* __restrict__ qr, const FT* __restrict__ qi,
                                                                   FT* __restrict__ xr, FT* __restrict__ xi,
                                                                   FT* __restrict__ rr, FT* __restrict__ ri,
                                                                   double* __restrict__ part) {
    if (sc[kScDone] != 0.0) return;
    __shared__ double red[kRedThreads];
    const FT alr = (FT)sc[2], ali = (FT)sc[3];
    double acc = 0.0;
    for (long long e = blockIdx.x * (long long)kRedThreads + threadIdx.x; e < n; e += (long long)gridDim.x * kRedThreads) {
        xr[e] += alr * pr[e] - ali * pi[e];
        xi[e] += alr * pi[e] + ali * pr[e];
        const FT a = rr[e] - (alr * qr[e] - ali * qi[e]);
        const FT b = ri[e] - (alr * qi[e] + ali * qr[e]);
        rr[e] = a;
        ri[e] = b;
        acc += (double)a * (double)a + (double)b * (double)b;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0];
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

// Start of an inner solve: r32 = (float) r, e32 = 0, and the partial sums of
// |r32|^2 (FP64) per block into part; 2n values (both planes); grid
// kRedBlocks; skipped when *flag is set
__global__ __launch_bounds__(kRedThreads) void sweep_setup_kernel(long long n2, const double* __restrict__ r,
                                                                  float* __restrict__ r32, float* __restrict__ e32,
                                                                  double* __restrict__ part,
                                                                  const double* __restrict__ flag) {
    if (flag && *flag != 0.0) return;
    __shared__ double red[kRedThreads];
    double acc = 0.0;
    for (long long e = blockIdx.x * (long long)kRedThreads + threadIdx.x; e < n2; e += (long long)gridDim.x * kRedThreads) {
        const float v = (float)r[e];
        r32[e] = v;
        e32[e] = 0.f;
        acc += (double)v * (double)v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0];
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

// p = z + be p with be = sc[4..5]
template <typename FT>
__global__ void cocg_p_dev_kernel(long long n, const double* __restrict__ sc, const FT* __restrict__ zr,
                                  const FT* __restrict__ zi, FT* __restrict__ pr, FT* __restrict__ pi) {
    if (sc[kScDone] != 0.0) return;
    const FT ber = (FT)sc[4], bei = (FT)sc[5];
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const FT a = pr[e], b = pi[e];
        pr[e] = zr[e] + ber * a - bei * b;
        pi[e] = zi[e] + ber * b + bei * a;
    }
}

// ------------------------------------------------------------------ host side

inline int grid_for(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

inline tdsez_status blas_fail(rocblas_status s, const char* what) {
    return fail(TDSEZ_EHIP, "%s failed: rocblas status %d", what, (int)s);
}

// Generalised eigendecomposition T Q = S Q Lambda, Q^T S Q = I of one axis
// (FP64, rocSOLVER, once per system); Q column-major, N x N.
inline tdsez_status axis_eigen(rocblas_handle blas, const SystemData& ax, double** d_Q, double** d_l) {
    const int N = ax.N, p = ax.p;
    double *dS = nullptr, *dE = nullptr;
    rocblas_int* dinfo = nullptr;
    TDSEZ_HIP_TRY(hipMalloc(d_Q, sizeof(double) * (size_t)N * N));
    TDSEZ_HIP_TRY(hipMalloc(d_l, sizeof(double) * N));
    TDSEZ_HIP_TRY(hipMalloc(&dS, sizeof(double) * (size_t)N * N));
    TDSEZ_HIP_TRY(hipMalloc(&dE, sizeof(double) * N));
    TDSEZ_HIP_TRY(hipMalloc(&dinfo, sizeof(rocblas_int)));
    band_to_dense_kernel<<<grid_for((long long)N * N), 256>>>(ax.d_band[1], N, p, *d_Q);  // T
    band_to_dense_kernel<<<grid_for((long long)N * N), 256>>>(ax.d_band[0], N, p, dS);    // S
    TDSEZ_HIP_TRY(hipGetLastError());
    rocblas_set_stream(blas, nullptr);
    rocblas_status bs = rocsolver_dsygvd(blas, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, N,
                                         *d_Q, N, dS, N, *d_l, dE, dinfo);
    rocblas_int info = 0;
    hipError_t he = hipMemcpy(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost);
    (void)hipFree(dS);
    (void)hipFree(dE);
    (void)hipFree(dinfo);
    if (bs != rocblas_status_success) return blas_fail(bs, "rocsolver_dsygvd");
    if (he != hipSuccess) return fail(TDSEZ_EHIP, "hipMemcpy failed: %s", hipGetErrorString(he));
    if (info != 0) return fail(TDSEZ_ENOCONV, "per-axis generalised eigensolve failed (info %d)", (int)info);
    return TDSEZ_OK;
}

// Work vectors of the step loop, planar, n unknowns each.
enum { kC = 0, kX = 1, kR = 2, kZ = 3, kP = 4, kQ = 5, kB = 6, kT1 = 7, kT2 = 8, kNumVec64 = 9 };   // FP64
enum { kR32 = 0, kZ32 = 1, kP32 = 2, kQ32 = 3, kE32 = 4, kT132 = 5, kT232 = 6, kNumVec32 = 7 };     // FP32

struct CnWork {
    long long n = 0;
    double* w = nullptr;      // kNumVec64 planar FP64 vectors
    float* w32 = nullptr;     // kNumVec32 planar FP32 vectors (refined precision only)
    double* part = nullptr;   // 2 kRedBlocks reduction partials
    double* sc = nullptr;     // 2 kScBlock scalar slots (FP64 / outer, FP32 inner)
    int* status = nullptr;    // 4 ints: latched code, step
    double* obs_part = nullptr;
    int nblk_obs = 0;         // per-block observable partials written by apply
    double* acc_part = nullptr;  // per-block partials of Re c^H G c (op.accel), or nullptr
    double* dpart = nullptr;  // partials of the dot products fused into apply and the preconditioner
    double* re(int k) const { return w + (size_t)(2 * k) * n; }
    double* im(int k) const { return w + (size_t)(2 * k + 1) * n; }
    float* re32(int k) const { return w32 + (size_t)(2 * k) * n; }
    float* im32(int k) const { return w32 + (size_t)(2 * k + 1) * n; }
};

struct CnStats {
    long long iters_total = 0;
    int iters_max = 0;
    long long steps_total = 0;
    long long sweeps_total = 0;
};

// nsteps Crank-Nicolson steps of psi (device, interleaved complex, n
// entries) under the field E (device, nsteps + 1 samples, midpoint rule),
// the observables of every state (nsteps + 1 rows of 3: nu, d_x, 0) in
// obs_out when obs is set.  FP64: COCG to the relative residual tol.
// Refined: FP32 COCG sweeps on the FP64 residual until it meets tol.  The
// loop never waits for the device; each step enqueues an iteration budget
// taken from the counts of earlier steps (a host-visible log the device
// writes), and a step that exhausts its budget latches ENOCONV.
template <class Op>
tdsez_status cn_cocg_propagate(const CnWork& cw, Op& op, double* psi, const double* E, double dt, int nsteps,
                               bool mixed, unsigned obs, double* obs_out, double tol, int maxit, hipStream_t stream,
                               CnStats* stats, const char* what) {
    const long long n = cw.n;
    double* outer = cw.sc;             // FP64 solve / outer refinement scalars
    double* inner = cw.sc + kScBlock;  // FP32 inner solve scalars
    const double* fo = outer + kScDone;  // "converged" flags
    const double* fi = inner + kScDone;
    int* log = nullptr;
    int* log_dev = nullptr;
    TDSEZ_HIP_TRY(hipHostMalloc((void**)&log, sizeof(int) * kLogStride * ((size_t)nsteps + 1),
                                hipHostMallocMapped | hipHostMallocCoherent));
    struct LogGuard {
        int* p;
        ~LogGuard() { (void)hipHostFree(p); }
    } guard{log};
    for (size_t i = 0; i < kLogStride * ((size_t)nsteps + 1); ++i) log[i] = -1;
    TDSEZ_HIP_TRY(hipHostGetDevicePointer((void**)&log_dev, log, 0));
    const int g = grid_for(n);
    {
        // scalars: flags and counters cleared, tolerances set, no latched error
        double init[2 * kScBlock] = {};
        init[kScTol2] = tol * tol;
        TDSEZ_HIP_TRY(hipMemcpyAsync(cw.sc, init, sizeof(init), hipMemcpyHostToDevice, stream));
        TDSEZ_HIP_TRY(hipMemsetAsync(cw.status, 0, sizeof(int) * 4, stream));
        TDSEZ_HIP_TRY(hipStreamSynchronize(stream));  // init is a stack array
    }
    to_planar_kernel<<<g, 256, 0, stream>>>(psi, n, cw.re(kC), cw.im(kC));
    copy_kernel<double><<<g, 256, 0, stream>>>(2 * n, nullptr, cw.re(kX), nullptr);
    const double alpha = 0.5 * dt;
    auto dot_dev = [&](int u, int v, bool abs2, int mode, bool count, const double* flag) {
        dot_kernel<double><<<kRedBlocks, kRedThreads, 0, stream>>>(n, cw.re(u), cw.im(u), cw.re(v), cw.im(v), abs2,
                                                                   cw.part, flag);
        cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.part, kRedBlocks, mode, outer, count);
    };
    std::vector<double> Eh((size_t)nsteps + 1);
    TDSEZ_HIP_TRY(hipMemcpyAsync(Eh.data(), E, sizeof(double) * Eh.size(), hipMemcpyDeviceToHost, stream));
    TDSEZ_HIP_TRY(hipStreamSynchronize(stream));
    // FP32 inner solves reduce the FP64 residual by this factor per sweep
    // (within an order of the FP32 accuracy of the inner operator: two
    // sweeps then reach 1e-12 from a residual of 1e-1)
    constexpr double kInnerTol = 2e-6;
    // iteration budgets of a step: a margin above the largest count among
    // the last logged steps (the log lags the host by however many steps are
    // queued), capped by maxit; sweeps: a fixed budget
    constexpr int kMargin = 3, kWindow = 8;
    int known = -1;  // last step whose log entry has arrived
    auto budget = [&](int col, int first, int margin) {
        volatile const int* lg = log;
        while (known + 1 < nsteps && lg[kLogStride * (known + 1) + 0] >= 0) ++known;
        int mx = -1;
        for (int j = known; j >= 0 && j > known - kWindow; --j) mx = std::max(mx, (int)lg[kLogStride * j + col]);
        const int b = mx < 0 ? first : mx + margin;
        return std::min(std::max(b, 1), maxit);
    };
    for (int step = 0; step <= nsteps; ++step) {
        const double Eb = step < nsteps ? 0.5 * (Eh[step] + Eh[step + 1]) : Eh[step];
        // b = -i dt H c (and the observables of c)
        op.apply(kC, -1, 0.0, 0.0, 0.0, 0.0, 0.0, -2.0 * alpha, Eb, kB, cw.obs_part, nullptr, stream);
        if (obs) {
            const int na = (obs & TDSEZ_OBS_ACCEL) && cw.acc_part ? op.accel(kC, cw.acc_part, stream) : 0;
            obs_finish_kernel<<<1, kRedThreads, 0, stream>>>(cw.obs_part, cw.nblk_obs, na ? cw.acc_part : nullptr, na,
                                                             Eh[step], obs_out + 3 * (size_t)step, obs);
        }
        if (step == nsteps) break;
        // A x = b, A = S + i a H, warm start from the previous increment: r = b - A x.
        // The refined path forms this first residual with the FP32 operator: its
        // rounding (relative 1e-7 of A x) only perturbs the first sweep's right-hand
        // side, and the FP64 residual that ends the sweep removes it.
        if (!mixed) {
            op.apply(kX, kB, 1.0, 0.0, -1.0, 0.0, 0.0, -alpha, Eb, kR, nullptr, nullptr, stream);
        } else {
            to_fp32_kernel<<<g, 256, 0, stream>>>(2 * n, cw.re(kX), cw.re32(kE32), nullptr);
            op.apply32(kE32, 1.0, 0.0, 0.0, alpha, Eb, kQ32, nullptr, stream);
            sub32_kernel<<<g, 256, 0, stream>>>(2 * n, cw.re(kB), cw.re32(kQ32), cw.re(kR));
        }
        dot_dev(kB, kB, true, 4, false, nullptr);
        dot_dev(kR, kR, true, 3, false, nullptr);
        // The dot products of an iteration are fused into the kernels that
        // produce their operands (p^T q into the operator, |r|^2 into the
        // update, r^T z into the last preconditioner contraction); one block
        // then sums the partials in a fixed order and updates the scalars.
        const int na64 = op.nblk_apply(false), na32 = op.nblk_apply(true), nz = op.nblk_precond();
        if (!mixed) {
            // COCG in FP64; every kernel returns once the residual has met tol
            const int K = budget(0, 12, kMargin);
            op.precond(kR, kZ, fo, stream, cw.dpart);
            cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.dpart, nz, 0, outer, false);  // rho = r^T z
            copy_kernel<double><<<g, 256, 0, stream>>>(2 * n, cw.re(kZ), cw.re(kP), fo);
            for (int it = 0; it < K; ++it) {
                op.apply(kP, -1, 0.0, 0.0, 1.0, 0.0, 0.0, alpha, Eb, kQ, nullptr, fo, stream, cw.dpart);  // q = A p
                cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.dpart, na64, 1, outer, false);  // alpha
                cocg_xr_norm_kernel<double><<<kRedBlocks, kRedThreads, 0, stream>>>(
                    n, outer, cw.re(kP), cw.im(kP), cw.re(kQ), cw.im(kQ), cw.re(kX), cw.im(kX), cw.re(kR), cw.im(kR),
                    cw.part);
                cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.part, kRedBlocks, 3, outer, true);  // converged?
                op.precond(kR, kZ, fo, stream, cw.dpart);
                cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.dpart, nz, 2, outer, false);  // beta, rho
                cocg_p_dev_kernel<double><<<g, 256, 0, stream>>>(n, outer, cw.re(kZ), cw.im(kZ), cw.re(kP),
                                                                 cw.im(kP));
            }
        } else {
            // iterative refinement: FP64 residual r = b - A x, FP32 COCG on
            // A e = r (same preconditioner in FP32), x += e
            // per sweep: a margin of 2 over that sweep's recent counts (the
            // counts of successive sweeps differ; one budget for all would
            // enqueue the first sweep's count for every sweep)
            const int Kall = budget(1, 12, kMargin);
            const int Ks = budget(2, 3, 1);
            for (int sw = 0; sw < Ks; ++sw) {
                // a sweep that no recent step needed (count 0) only has to
                // finish a residual that the sweeps before it nearly met: a
                // short budget (a step that still misses tol latches ENOCONV)
                const int Kw = sw < kLogSweeps ? budget(4 + sw, 12, 2) : 0;
                const int Ki = Kw > 2 ? std::min(Kw, Kall) : std::min(4, Kall);
                sweep_start_kernel<<<1, 64, 0, stream>>>(outer, inner, kInnerTol);
                sweep_setup_kernel<<<kRedBlocks, kRedThreads, 0, stream>>>(2 * n, cw.re(kR), cw.re32(kR32),
                                                                           cw.re32(kE32), cw.part, fo);
                cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.part, kRedBlocks, 4, inner, false);  // |b|^2
                op.precond32(kR32, kZ32, fi, stream, cw.dpart);
                cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.dpart, nz, 0, inner, false);
                copy_kernel<float><<<g, 256, 0, stream>>>(2 * n, cw.re32(kZ32), cw.re32(kP32), fi);
                for (int it = 0; it < Ki; ++it) {
                    op.apply32(kP32, 1.0, 0.0, 0.0, alpha, Eb, kQ32, fi, stream, cw.dpart);  // q = A p
                    cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.dpart, na32, 1, inner, false);
                    cocg_xr_norm_kernel<float><<<kRedBlocks, kRedThreads, 0, stream>>>(
                        n, inner, cw.re32(kP32), cw.im32(kP32), cw.re32(kQ32), cw.im32(kQ32), cw.re32(kE32),
                        cw.im32(kE32), cw.re32(kR32), cw.im32(kR32), cw.part);
                    cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.part, kRedBlocks, 3, inner, true);
                    op.precond32(kR32, kZ32, fi, stream, cw.dpart);
                    cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(cw.dpart, nz, 2, inner, false);
                    cocg_p_dev_kernel<float><<<g, 256, 0, stream>>>(n, inner, cw.re32(kZ32), cw.im32(kZ32),
                                                                    cw.re32(kP32), cw.im32(kP32));
                }
                add_kernel<float><<<g, 256, 0, stream>>>(n, cw.re32(kE32), cw.im32(kE32), cw.re(kX), cw.im(kX), fo);
                op.apply(kX, kB, 1.0, 0.0, -1.0, 0.0, 0.0, -alpha, Eb, kR, nullptr, fo, stream);  // r = b - A x
                dot_dev(kR, kR, true, 3, false, fo);
            }
        }
        step_end_kernel<<<1, 64, 0, stream>>>(outer, inner, step, cw.status, log_dev);
        add_kernel<double><<<g, 256, 0, stream>>>(n, cw.re(kX), cw.im(kX), cw.re(kC), cw.im(kC), nullptr);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    from_planar_kernel<<<g, 256, 0, stream>>>(cw.re(kC), cw.im(kC), n, psi);
    TDSEZ_HIP_TRY(hipGetLastError());
    // the call ends here: statistics and the latched convergence failure
    TDSEZ_HIP_TRY(hipStreamSynchronize(stream));
    int stat[4] = {0, 0, 0, 0};
    TDSEZ_HIP_TRY(hipMemcpy(stat, cw.status, sizeof(stat), hipMemcpyDeviceToHost));
    for (int st = 0; st < nsteps; ++st) {
        const int* lg = log + (size_t)kLogStride * st;
        const int it = mixed ? lg[3] : lg[0];
        stats->iters_total += it;
        stats->iters_max = std::max(stats->iters_max, it);
        stats->sweeps_total += lg[2];
        stats->steps_total += 1;
    }
    if (stat[0] == TDSEZ_ENOCONV)
        return fail(TDSEZ_ENOCONV, "%s step %d: residual above %g after its iteration budget (maxit %d)", what,
                    stat[1], tol, maxit);
    return TDSEZ_OK;
}

}  // namespace
}  // namespace tdsez
