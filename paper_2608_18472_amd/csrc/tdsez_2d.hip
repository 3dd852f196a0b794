// Two-dimensional tensor-product propagation (constant mass, x-polarised
// field): Crank-Nicolson steps of section V.B on the basis N_ix(x) N_iy(y).
//
// Matrices, with the 1D half bands of each axis (tdsez_assemble.hip) and the
// non-separable potential stencil assembled here:
//   S2 = Sx (x) Sy,  T2 = Tx (x) Sy + Sx (x) Ty,  D2 = Dx (x) Sy,
//   V2[(iy,ix),(jy,jx)] = sum_q wx wy V(x_q, y_q) N_ix N_jx N_iy N_jy.
// Unknown (iy, ix) has the row-major index iy*Nx + ix.  Complex vectors are
// held planar on the device (real plane, then imaginary plane, each Ny x Nx
// row-major) so that the per-axis transforms are plain real GEMMs.
//
// Each step solves the increment form A_n Delta = -i dt H_n c_n with
// A_n = S2 + i a H_n, H_n = T2 + V2 + Ebar_n D2, a = dt/2, by conjugate-
// orthogonal CG (A_n is complex symmetric) preconditioned with the exact
// inverse of the separable part P = S2 + i a T2: with T Q = S Q Lambda and
// Q^T S Q = I on each axis (generalised eigendecomposition, once per system),
//   P^-1 R = Q_y [ (Q_y^T R Q_x) / (1 + i a (mu_iy + lambda_ix)) ] Q_x^T,
// i.e. four per-axis contractions (hand-written MFMA kernels, both planes
// per launch, the diagonal scaling fused into the second).  The field and
// the potential are the only parts left to the iteration.  The operator
// itself is one stencil kernel over the (2p+1)^2 neighbours of every
// unknown: the separable parts from the per-axis bands, V2 from a half
// stencil (symmetric: the other half is read from the neighbour's row).
//
// The step loop never waits for the host: every iteration kernel reads a
// device-side "converged" flag that the residual-norm kernel sets, and
// returns at once when it is set, so a step enqueues a fixed budget of
// iterations (from the counts of earlier steps, read back asynchronously)
// and the iterations past convergence cost only their launches.  A step
// that exhausts its budget latches ENOCONV, reported when the call ends.
// rocSOLVER computes the per-axis eigendecompositions once, at assembly.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "tdsez_internal.hpp"

struct tdsez_system2d_s;

namespace tdsez {

__global__ void basis_kernel(const double* __restrict__ br, int nbr, int p, int nq,
                             const double* __restrict__ xq, double* __restrict__ Bv,
                             double* __restrict__ dB);

namespace {

// number of stored stencil offsets: (dy, dx) with dy > 0, or dy == 0 and dx >= 0
__host__ __device__ inline int half_count(int p) { return (p + 1) + p * (2 * p + 1); }
// index of a stored offset
__host__ __device__ inline int half_index(int p, int dy, int dx) {
    return dy == 0 ? dx : (p + 1) + (dy - 1) * (2 * p + 1) + (dx + p);
}

// M[i][j] of a 1D lower half band by rows (band[j*(p+1) + d] = M[j][j-d])
__device__ inline double band_ij(const double* __restrict__ band, int p, int i, int j) {
    const int hi = i > j ? i : j;
    const int d = i > j ? i - j : j - i;
    return band[hi * (p + 1) + d];
}

// V2 half stencil, one thread per (row, stored offset).  Sums over the spans
// shared by the two x B-splines and by the two y B-splines, x innermost.
__global__ void v2_kernel(int Nx, int Ny, int p, int nq, int nelx, int nely, const double* __restrict__ brx,
                          const double* __restrict__ bry, const double* __restrict__ gw,
                          const double* __restrict__ Bx, const double* __restrict__ By,
                          const double* __restrict__ Vq, double* __restrict__ V2h) {
    const int nh = half_count(p);
    const long long total = (long long)Nx * Ny * nh;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int h = (int)(e / ((long long)Nx * Ny));
        const long long row = e % ((long long)Nx * Ny);
        const int iy = (int)(row / Nx), ix = (int)(row % Nx);
        int dy, dx;
        if (h <= p) {
            dy = 0;
            dx = h;
        } else {
            dy = 1 + (h - p - 1) / (2 * p + 1);
            dx = (h - p - 1) % (2 * p + 1) - p;
        }
        const int jy = iy + dy, jx = ix + dx;
        double sum = 0.0;
        if (jy < Ny && jx >= 0 && jx < Nx) {
            // global B-spline indices are unknown + 1
            const int gxa = ix + 1, gxb = jx + 1, gya = iy + 1, gyb = jy + 1;
            const int gxh = gxa > gxb ? gxa : gxb, gxl = gxa > gxb ? gxb : gxa;
            const int gyh = gya > gyb ? gya : gyb, gyl = gya > gyb ? gyb : gya;
            const int ex0 = gxh - p > 0 ? gxh - p : 0, ex1 = gxl < nelx - 1 ? gxl : nelx - 1;
            const int ey0 = gyh - p > 0 ? gyh - p : 0, ey1 = gyl < nely - 1 ? gyl : nely - 1;
            const int nqx = nelx * nq;
            for (int ey = ey0; ey <= ey1; ++ey) {
                const double hy = 0.5 * (bry[ey + 1] - bry[ey]);
                for (int qy = 0; qy < nq; ++qy) {
                    const long long iqy = (long long)ey * nq + qy;
                    const double wy = gw[qy] * hy * By[iqy * (p + 1) + (gya - ey)] * By[iqy * (p + 1) + (gyb - ey)];
                    double sx = 0.0;
                    for (int ex = ex0; ex <= ex1; ++ex) {
                        const double hx = 0.5 * (brx[ex + 1] - brx[ex]);
                        for (int qx = 0; qx < nq; ++qx) {
                            const long long iqx = (long long)ex * nq + qx;
                            sx += gw[qx] * hx * Bx[iqx * (p + 1) + (gxa - ex)] * Bx[iqx * (p + 1) + (gxb - ex)] *
                                  Vq[iqy * nqx + iqx];
                        }
                    }
                    sum += wy * sx;
                }
            }
        }
        V2h[e] = sum;
    }
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

constexpr int kStencilThreads = 256;  // threads (and outputs) per stencil tile
// Tile shape: a tile row spans one 128-byte line of a plane (16 FP64 or 32
// FP32 values), so every stencil load uses whole lines.
template <typename FT>
struct TileShape {
    static constexpr int TX = 128 / (int)sizeof(FT);
    static constexpr int TY = kStencilThreads / TX;
};
template <typename FT>
dim3 stencil_grid(int Nx, int Ny) {
    return dim3((Nx + TileShape<FT>::TX - 1) / TileShape<FT>::TX, (Ny + TileShape<FT>::TY - 1) / TileShape<FT>::TY);
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

// out = w y + a S2 c + b (T2 + V2 + Ebar D2) c   (planar complex; y may be
// null), for one TX x TY tile of outputs with the input tile and a p-wide
// halo in LDS, in three stages:
//  (1) x pass: every row of the haloed tile is convolved with the x bands at
//      the thread's column, s = Sx c and h = (Tx + Ebar Dx) c (and Dx c for
//      the observables), kept in LDS;
//  (2) y pass: S2 c = Sy s and (T2 + Ebar D2) c = Sy h + Ty s at the output,
//      so the separable part costs O(p) per unknown instead of O(p^2);
//  (3) the potential, over the stored half of the stencil: for each stored
//      offset e = (dy, dx), V2[i][i+e] c_{i+e} from this row's plane entry
//      and V2[i][i-e] c_{i-e} = V2[i-e][i] c_{i-e} from the same plane at
//      row i - e (clamped into the plane where i - e is outside: c is zero
//      there).  The two reads of a plane are issued together, so the second
//      finds most of its lines already on their way.
// With obs != null every block writes partial sums of Re c^H S2 c and
// Re c^H D2 c (FP64).  Four tiles per CU (<= 128 VGPRs) let the 1024 tiles
// of a 512 x 512 grid run in one round.
template <int PP, typename FT>
__global__ __launch_bounds__(kStencilThreads, 4) void apply_kernel(
    int Nx, int Ny, const FT* __restrict__ Sxb, const FT* __restrict__ Txb, const FT* __restrict__ Dxb,
    const FT* __restrict__ Syb, const FT* __restrict__ Tyb, const FT* __restrict__ V2h, const FT* __restrict__ cre,
    const FT* __restrict__ cim, const FT* __restrict__ yre, const FT* __restrict__ yim, FT wre, FT wim, FT are,
    FT aim, FT bre, FT bim, FT Ebar, FT* __restrict__ ore, FT* __restrict__ oim, double* __restrict__ obs,
    const double* __restrict__ flag) {
    if (flag && *flag != 0.0) return;  // the solve has converged
    constexpr int TX = TileShape<FT>::TX, TY = TileShape<FT>::TY;
    constexpr int K = 2 * PP + 1;
    constexpr int WX = TX + 2 * PP, WY = TY + 2 * PP;
    __shared__ FT tre[WY][WX], tim[WY][WX];
    __shared__ FT s_re[WY][TX], s_im[WY][TX], h_re[WY][TX], h_im[WY][TX];
    __shared__ FT d_re[WY][TX], d_im[WY][TX];
    __shared__ double red[2][kStencilThreads];
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int ix = x0 + tx, iy = y0 + ty;
    const long long plane = (long long)Nx * Ny;
    for (int t = threadIdx.x; t < WX * WY; t += kStencilThreads) {
        const int ly = t / WX, lx = t % WX;
        const int gy = y0 + ly - PP, gx = x0 + lx - PP;
        FT vr = 0, vi = 0;
        if (gy >= 0 && gy < Ny && gx >= 0 && gx < Nx) {
            vr = cre[(long long)gy * Nx + gx];
            vi = cim[(long long)gy * Nx + gx];
        }
        tre[ly][lx] = vr;
        tim[ly][lx] = vi;
    }
    // x factors of the thread's column
    FT sx[K], hx[K], dx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int jx = ix + k - PP;
        sx[k] = band_at(Sxb, PP, Nx, ix, jx);
        dx[k] = band_at(Dxb, PP, Nx, ix, jx);
        hx[k] = band_at(Txb, PP, Nx, ix, jx) + Ebar * dx[k];
    }
    __syncthreads();
    // (1) x pass over the tile rows (halo rows included)
    for (int ly = ty; ly < WY; ly += TY) {
        FT sr = 0, si = 0, hr = 0, hi = 0, dr = 0, di = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const FT zr = tre[ly][tx + k], zi = tim[ly][tx + k];
            sr += sx[k] * zr;
            si += sx[k] * zi;
            hr += hx[k] * zr;
            hi += hx[k] * zi;
            dr += dx[k] * zr;
            di += dx[k] * zi;
        }
        s_re[ly][tx] = sr;
        s_im[ly][tx] = si;
        h_re[ly][tx] = hr;
        h_im[ly][tx] = hi;
        d_re[ly][tx] = dr;
        d_im[ly][tx] = di;
    }
    // (3) potential, from the input tile (independent of the x pass)
    const int ixc = ix < Nx ? ix : Nx - 1, iyc = iy < Ny ? iy : Ny - 1;
    const long long row = (long long)iyc * Nx + ixc;
    const int cy = ty + PP, cx = tx + PP;  // this unknown in the tile
    FT vr = 0, vi = 0;
    {
        // dy = 0: the diagonal, then e = (0, dx) and its mirror (0, -dx)
        const FT v0 = V2h[row];
        vr += v0 * tre[cy][cx];
        vi += v0 * tim[cy][cx];
#pragma unroll
        for (int e = 1; e <= PP; ++e) {
            const FT* __restrict__ pl = V2h + (long long)half_index(PP, 0, e) * plane;
            const int jx = ixc - e < 0 ? 0 : ixc - e;
            const FT vd = pl[row];
            const FT vm = pl[(long long)iyc * Nx + jx];
            vr += vd * tre[cy][cx + e] + vm * tre[cy][cx - e];
            vi += vd * tim[cy][cx + e] + vm * tim[cy][cx - e];
        }
    }
    // dy = 1..p: e = (dy, dx), dx = -p..p, and the mirrors -e
#pragma unroll 1
    for (int dy = 1; dy <= PP; ++dy) {
        const FT* __restrict__ pl = V2h + (long long)half_index(PP, dy, -PP) * plane;
        const long long mrow = (long long)(iyc - dy < 0 ? 0 : iyc - dy) * Nx;
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
            const int e = kx - PP;
            int jx = ixc - e;
            jx = jx < 0 ? 0 : (jx >= Nx ? Nx - 1 : jx);
            const FT vd = pl[(long long)kx * plane + row];
            const FT vm = pl[(long long)kx * plane + mrow + jx];
            vr += vd * tre[cy + dy][cx + e] + vm * tre[cy - dy][cx - e];
            vi += vd * tim[cy + dy][cx + e] + vm * tim[cy - dy][cx - e];
        }
    }
    __syncthreads();
    // (2) y pass
    FT Sr = 0, Si = 0, Hr = 0, Hi = 0, Dr = 0, Di = 0;
#pragma unroll
    for (int ky = 0; ky < K; ++ky) {
        const int jy = iy + ky - PP;
        const FT sy = band_at(Syb, PP, Ny, iy, jy), tyv = band_at(Tyb, PP, Ny, iy, jy);
        const FT a_r = s_re[ty + ky][tx], a_i = s_im[ty + ky][tx];
        Sr += sy * a_r;
        Si += sy * a_i;
        Hr += sy * h_re[ty + ky][tx] + tyv * a_r;
        Hi += sy * h_im[ty + ky][tx] + tyv * a_i;
        if (obs) {
            Dr += sy * d_re[ty + ky][tx];
            Di += sy * d_im[ty + ky][tx];
        }
    }
    double nu = 0.0, dip = 0.0;
    if (ix < Nx && iy < Ny) {
        // a S2 c + b ((T2 + Ebar D2) c + V2 c)
        const FT gr = Hr + vr, gi = Hi + vi;
        FT accr = are * Sr - aim * Si + bre * gr - bim * gi;
        FT acci = are * Si + aim * Sr + bre * gi + bim * gr;
        const long long orow = (long long)iy * Nx + ix;
        if (yre) {
            const FT yr = yre[orow], yi = yim[orow];
            accr += wre * yr - wim * yi;
            acci += wre * yi + wim * yr;
        }
        ore[orow] = accr;
        oim[orow] = acci;
        if (obs) {
            const double c0r = tre[cy][cx], c0i = tim[cy][cx];
            nu = c0r * (double)Sr + c0i * (double)Si;
            dip = c0r * (double)Dr + c0i * (double)Di;
        }
    }
    if (obs) {
        red[0][threadIdx.x] = nu;
        red[1][threadIdx.x] = dip;
        __syncthreads();
        for (int s = kStencilThreads / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                red[0][threadIdx.x] += red[0][threadIdx.x + s];
                red[1][threadIdx.x] += red[1][threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
            obs[2 * blk] = red[0][0];
            obs[2 * blk + 1] = red[1][0];
        }
    }
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
// C is M x N row-major (ld N).  SCALE divides the result by
// 1 + i a (mu_m + lambda_n) (the diagonal of the separable part in the
// eigenbasis), which needs both planes of an entry: every workgroup computes
// both.  flag != nullptr and *flag != 0 skips the launch (converged solve).
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

template <typename FT, bool LEFTQ, bool SCALE>
__global__ __launch_bounds__(kGemmThreads) void fdm_gemm_kernel(
    int M, int N, int K, const FT* __restrict__ Q, int qs0, int qs1, const FT* __restrict__ vr,
    const FT* __restrict__ vi, FT* __restrict__ cr, FT* __restrict__ ci, double alpha,
    const double* __restrict__ lam_n, const double* __restrict__ mu_m, const double* __restrict__ flag) {
    if (flag && *flag != 0.0) return;
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
    for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + MfmaOps<FT>::row(lk, r);
        if (gm >= M || gn >= N) continue;
        FT a = acc[0][r], b = acc[1][r];
        if constexpr (SCALE) {
            const double t = alpha * (mu_m[gm] + lam_n[gn]);
            const double s = 1.0 / (1.0 + t * t);
            const double ad = a, bd = b;
            a = (FT)((ad + t * bd) * s);
            b = (FT)((bd - t * ad) * s);
        }
        cr[(long long)gm * N + gn] = a;
        ci[(long long)gm * N + gn] = b;
    }
}


// observables: sum the per-block partials of apply_kernel (fixed order per
// thread, then a tree over the block: deterministic)
__global__ __launch_bounds__(kRedThreads) void obs_finish_kernel(const double* __restrict__ part, int nblk,
                                                                 double* __restrict__ out, unsigned mask) {
    __shared__ double a[kRedThreads], b[kRedThreads];
    double nu = 0.0, d = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kRedThreads) {
        nu += part[2 * k];
        d += part[2 * k + 1];
    }
    a[threadIdx.x] = nu;
    b[threadIdx.x] = d;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            a[threadIdx.x] += a[threadIdx.x + s];
            b[threadIdx.x] += b[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (mask & TDSEZ_OBS_NORM) ? a[0] : 0.0;
        out[1] = (mask & TDSEZ_OBS_DIPOLE) ? b[0] : 0.0;
        out[2] = 0.0;
    }
}

// COCG scalars on the device, one slot block per solve level (FP64 solve /
// outer refinement, FP32 inner solve): sc[0..1] rho, sc[2..3] alpha,
// sc[4..5] beta, sc[6] |r|^2, sc[7] |b|^2, sc[8] converged flag, sc[9]
// iterations (of the step; of the current sweep for the inner block),
// sc[10] squared relative tolerance, sc[11] refinement sweeps of the step,
// inner block only: sc[12] largest and sc[13] total inner iterations of the
// step's sweeps.  One block sums the partials of the last
// dot (fixed order) and updates the scalars for `mode`:
//   0: rho = sum          1: alpha = rho / sum
//   2: beta = sum / rho, rho = sum
//   3: |r|^2 = sum (one more iteration when `count`); converged when
//      |r|^2 <= sc[10] |b|^2
//   4: |b|^2 = sum
enum { kScRho = 0, kScAlpha = 2, kScBeta = 4, kScR2 = 6, kScB2 = 7, kScDone = 8, kScIts = 9, kScTol2 = 10,
       kScSweeps = 11, kScItsMax = 12, kScItsSum = 13, kScBlock = 16 };
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
// the step's counts (FP64 iterations, largest inner iterations of a sweep,
// sweeps, total inner iterations) go to the host-visible log; the flags and
// counters are reset for the next step.
__global__ void step_end_kernel(double* __restrict__ outer, double* __restrict__ inner, int step,
                                int* __restrict__ status, int* __restrict__ log) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (outer[kScDone] == 0.0 && status[0] == 0) {
        status[0] = TDSEZ_ENOCONV;
        status[1] = step;
    }
    log[4 * step + 0] = (int)outer[kScIts];
    log[4 * step + 1] = (int)fmax(inner[kScItsMax], inner[kScIts]);
    log[4 * step + 2] = (int)outer[kScSweeps];
    log[4 * step + 3] = (int)(inner[kScItsSum] + inner[kScIts]);
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

}  // namespace
}  // namespace tdsez

using namespace tdsez;

struct tdsez_system2d_s {
    SystemData ax, ay;         // per-axis 1D matrices (V = 0, m = 1)
    int Nx = 0, Ny = 0, p = 0, order = 0, nq = 0;
    double* d_V2h = nullptr;   // half stencil, [offset][row]
    double* d_Qx = nullptr;    // generalised eigenvectors (column-major), T Q = S Q Lambda
    double* d_Qy = nullptr;
    double* d_lx = nullptr;
    double* d_my = nullptr;
    double* d_work = nullptr;  // planar vectors: c, x, r, z, p, q, b, t1, t2 (2 planes each)
    double* d_part = nullptr;  // reduction partials
    double* d_obs_part = nullptr;
    double* d_sc = nullptr;    // COCG scalars and flags (device), two slot blocks
    int* d_status = nullptr;   // latched failure of a propagation: code, step
    // FP32 copies for TDSEZ_FP32_REFINED, made by the first such call
    float* d_V2h32 = nullptr;
    float* d_bands32 = nullptr;  // Sx, Tx, Dx (Nx (p+1) each), then Sy, Ty (Ny (p+1) each)
    float* d_Qx32 = nullptr;
    float* d_Qy32 = nullptr;
    float* d_work32 = nullptr;   // planar FP32 vectors: r, z, p, q, e, t1, t2 (2 planes each)
    rocblas_handle blas = nullptr;
    long long iters_total = 0;
    int iters_max = 0;
    long long steps_total = 0;
    long long sweeps_total = 0;
};

namespace {

tdsez_status blas_fail(rocblas_status s, const char* what) {
    return fail(TDSEZ_EHIP, "%s failed: rocblas status %d", what, (int)s);
}

#define TD2_BLAS(expr)                                  \
    do {                                                \
        rocblas_status s_ = (expr);                     \
        if (s_ != rocblas_status_success) return blas_fail(s_, #expr); \
    } while (0)

void free2d(tdsez_system2d_s* s) {
    for (int m = 0; m < 6; ++m) {
        (void)hipFree(s->ax.d_band[m]);
        (void)hipFree(s->ay.d_band[m]);
    }
    (void)hipFree(s->ax.d_H0);
    (void)hipFree(s->ay.d_H0);
    (void)hipFree(s->d_V2h);
    (void)hipFree(s->d_Qx);
    (void)hipFree(s->d_Qy);
    (void)hipFree(s->d_lx);
    (void)hipFree(s->d_my);
    (void)hipFree(s->d_work);
    (void)hipFree(s->d_part);
    (void)hipFree(s->d_obs_part);
    (void)hipFree(s->d_sc);
    (void)hipFree(s->d_status);
    (void)hipFree(s->d_V2h32);
    (void)hipFree(s->d_bands32);
    (void)hipFree(s->d_Qx32);
    (void)hipFree(s->d_Qy32);
    (void)hipFree(s->d_work32);
    if (s->blas) rocblas_destroy_handle(s->blas);
}

int grid_for(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

// generalised eigendecomposition T Q = S Q Lambda of one axis (FP64, on the GPU)
tdsez_status axis_eigen(tdsez_system2d_s* s, const SystemData& ax, double** d_Q, double** d_l) {
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
    rocblas_set_stream(s->blas, nullptr);
    rocblas_status bs = rocsolver_dsygvd(s->blas, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, N,
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

// FP32 copies of the operator and preconditioner data (first
// TDSEZ_FP32_REFINED call; synchronous)
tdsez_status ensure_fp32(tdsez_system2d_s* s) {
    if (s->d_work32) return TDSEZ_OK;
    const int Nx = s->Nx, Ny = s->Ny, p = s->p;
    const long long plane = (long long)Nx * Ny;
    const long long nv2 = (long long)half_count(p) * plane;
    const long long bx = (long long)Nx * (p + 1), by = (long long)Ny * (p + 1);
    float *v2 = nullptr, *bands = nullptr, *qx = nullptr, *qy = nullptr, *work = nullptr;
    hipError_t he = hipSuccess;
    auto H = [&](hipError_t e) { if (he == hipSuccess) he = e; };
    H(hipMalloc(&v2, sizeof(float) * nv2));
    H(hipMalloc(&bands, sizeof(float) * (3 * bx + 2 * by)));
    H(hipMalloc(&qx, sizeof(float) * (size_t)Nx * Nx));
    H(hipMalloc(&qy, sizeof(float) * (size_t)Ny * Ny));
    H(hipMalloc(&work, sizeof(float) * (size_t)plane * 2 * 7));
    if (he != hipSuccess) {
        (void)hipFree(v2); (void)hipFree(bands); (void)hipFree(qx); (void)hipFree(qy); (void)hipFree(work);
        return fail(TDSEZ_ENOMEM, "2D FP32 workspace allocation failed");
    }
    to_fp32_kernel<<<grid_for(nv2), 256>>>(nv2, s->d_V2h, v2);
    to_fp32_kernel<<<grid_for(bx), 256>>>(bx, s->ax.d_band[0], bands);
    to_fp32_kernel<<<grid_for(bx), 256>>>(bx, s->ax.d_band[1], bands + bx);
    to_fp32_kernel<<<grid_for(bx), 256>>>(bx, s->ax.d_band[3], bands + 2 * bx);
    to_fp32_kernel<<<grid_for(by), 256>>>(by, s->ay.d_band[0], bands + 3 * bx);
    to_fp32_kernel<<<grid_for(by), 256>>>(by, s->ay.d_band[1], bands + 3 * bx + by);
    to_fp32_kernel<<<grid_for((long long)Nx * Nx), 256>>>((long long)Nx * Nx, s->d_Qx, qx);
    to_fp32_kernel<<<grid_for((long long)Ny * Ny), 256>>>((long long)Ny * Ny, s->d_Qy, qy);
    H(hipGetLastError());
    H(hipDeviceSynchronize());
    s->d_V2h32 = v2;
    s->d_bands32 = bands;
    s->d_Qx32 = qx;
    s->d_Qy32 = qy;
    s->d_work32 = work;
    if (he != hipSuccess) return fail(TDSEZ_EHIP, "2D FP32 copies: %s", hipGetErrorString(he));
    return TDSEZ_OK;
}

}  // namespace

extern "C" {

tdsez_status tdsez_assemble_2d(const double* breaks_x, int nbx, const double* breaks_y, int nby, int order, int nq,
                               const double* V_q, tdsez_system2d* out) {
    if (!out) return fail(TDSEZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (!breaks_x || !breaks_y || !V_q) return fail(TDSEZ_EINVAL, "NULL argument");
    if (order < 2) return fail(TDSEZ_EINVAL, "order must be >= 2");
    if (order - 1 > kMaxP) return fail(TDSEZ_EUNSUPPORTED, "order %d > %d", order, kMaxP + 1);
    if (nq < 1 || nq > 32) return fail(TDSEZ_EINVAL, "nq must be in 1..32");
    for (int a = 0; a < 2; ++a) {
        const double* br = a ? breaks_y : breaks_x;
        const int nb = a ? nby : nbx;
        if (nb < 2) return fail(TDSEZ_EINVAL, "need at least 2 breakpoints per axis");
        for (int i = 0; i + 1 < nb; ++i)
            if (!(br[i + 1] > br[i]) || !std::isfinite(br[i]) || !std::isfinite(br[i + 1]))
                return fail(TDSEZ_EINVAL, "breakpoints must be finite and strictly increasing");
    }
    const int p = order - 1;
    const int Nx = nbx - 1 + p - 2, Ny = nby - 1 + p - 2;
    if (Nx < 2 * p + 1 || Ny < 2 * p + 1) return fail(TDSEZ_EINVAL, "need at least 2p+1 unknowns per axis");
    const long long nqx = (long long)(nbx - 1) * nq, nqy = (long long)(nby - 1) * nq;
    for (long long i = 0; i < nqx * nqy; ++i)
        if (!std::isfinite(V_q[i])) return fail(TDSEZ_EINVAL, "V_q[%lld] is not finite", i);
    auto* s = new tdsez_system2d_s();
    s->Nx = Nx;
    s->Ny = Ny;
    s->p = p;
    s->order = order;
    s->nq = nq;
    auto bail = [&](tdsez_status st) {
        free2d(s);
        delete s;
        return st;
    };
    tdsez_status st = assemble_device(breaks_x, nbx, order, nq, nullptr, nullptr, nullptr, &s->ax);
    if (st) return bail(st);
    st = assemble_device(breaks_y, nby, order, nq, nullptr, nullptr, nullptr, &s->ay);
    if (st) return bail(st);
    if (rocblas_create_handle(&s->blas) != rocblas_status_success)
        return bail(fail(TDSEZ_EHIP, "rocblas_create_handle failed"));
    // V2: basis values at the quadrature points of each axis, then the stencil
    {
        double gx[32], gw[32];
        gauss_legendre_host(nq, gx, gw);
        std::vector<double> xq(nqx), yq(nqy);
        for (int e = 0; e + 1 < nbx; ++e)
            for (int q = 0; q < nq; ++q)
                xq[(size_t)e * nq + q] = 0.5 * (breaks_x[e + 1] + breaks_x[e]) + 0.5 * (breaks_x[e + 1] - breaks_x[e]) * gx[q];
        for (int e = 0; e + 1 < nby; ++e)
            for (int q = 0; q < nq; ++q)
                yq[(size_t)e * nq + q] = 0.5 * (breaks_y[e + 1] + breaks_y[e]) + 0.5 * (breaks_y[e + 1] - breaks_y[e]) * gx[q];
        double *dbx = nullptr, *dby = nullptr, *dgw = nullptr, *dxq = nullptr, *dyq = nullptr, *dBx = nullptr,
               *dBy = nullptr, *ddB = nullptr, *dVq = nullptr;
        auto clean = [&]() {
            (void)hipFree(dbx); (void)hipFree(dby); (void)hipFree(dgw); (void)hipFree(dxq); (void)hipFree(dyq);
            (void)hipFree(dBx); (void)hipFree(dBy); (void)hipFree(ddB); (void)hipFree(dVq);
        };
        hipError_t he = hipSuccess;
        auto H = [&](hipError_t e) { if (he == hipSuccess) he = e; };
        H(hipMalloc(&dbx, sizeof(double) * nbx));
        H(hipMalloc(&dby, sizeof(double) * nby));
        H(hipMalloc(&dgw, sizeof(double) * nq));
        H(hipMalloc(&dxq, sizeof(double) * nqx));
        H(hipMalloc(&dyq, sizeof(double) * nqy));
        H(hipMalloc(&dBx, sizeof(double) * nqx * (p + 1)));
        H(hipMalloc(&dBy, sizeof(double) * nqy * (p + 1)));
        H(hipMalloc(&ddB, sizeof(double) * (nqx > nqy ? nqx : nqy) * (p + 1)));
        H(hipMalloc(&dVq, sizeof(double) * nqx * nqy));
        H(hipMalloc(&s->d_V2h, sizeof(double) * (size_t)half_count(p) * Nx * Ny));
        if (he == hipSuccess) {
            H(hipMemcpy(dbx, breaks_x, sizeof(double) * nbx, hipMemcpyHostToDevice));
            H(hipMemcpy(dby, breaks_y, sizeof(double) * nby, hipMemcpyHostToDevice));
            H(hipMemcpy(dgw, gw, sizeof(double) * nq, hipMemcpyHostToDevice));
            H(hipMemcpy(dxq, xq.data(), sizeof(double) * nqx, hipMemcpyHostToDevice));
            H(hipMemcpy(dyq, yq.data(), sizeof(double) * nqy, hipMemcpyHostToDevice));
            H(hipMemcpy(dVq, V_q, sizeof(double) * nqx * nqy, hipMemcpyHostToDevice));
        }
        if (he == hipSuccess) {
            basis_kernel<<<grid_for(nqx), 256>>>(dbx, nbx, p, nq, dxq, dBx, ddB);
            basis_kernel<<<grid_for(nqy), 256>>>(dby, nby, p, nq, dyq, dBy, ddB);
            v2_kernel<<<4096, 256>>>(Nx, Ny, p, nq, nbx - 1, nby - 1, dbx, dby, dgw, dBx, dBy, dVq, s->d_V2h);
            H(hipGetLastError());
            H(hipDeviceSynchronize());
        }
        clean();
        if (he != hipSuccess) return bail(fail(TDSEZ_EHIP, "2D assembly: %s", hipGetErrorString(he)));
    }
    st = axis_eigen(s, s->ax, &s->d_Qx, &s->d_lx);
    if (st) return bail(st);
    st = axis_eigen(s, s->ay, &s->d_Qy, &s->d_my);
    if (st) return bail(st);
    const long long plane = (long long)Nx * Ny;
    if (hipMalloc(&s->d_work, sizeof(double) * (size_t)plane * 2 * 9) != hipSuccess ||
        hipMalloc(&s->d_part, sizeof(double) * 2 * kRedBlocks) != hipSuccess ||
        hipMalloc(&s->d_sc, sizeof(double) * 2 * kScBlock) != hipSuccess ||
        hipMalloc(&s->d_status, sizeof(int) * 4) != hipSuccess ||
        hipMalloc(&s->d_obs_part, sizeof(double) * 2 * (size_t)stencil_grid<double>(Nx, Ny).x *
                                      stencil_grid<double>(Nx, Ny).y) !=
            hipSuccess)
        return bail(fail(TDSEZ_ENOMEM, "2D workspace allocation failed"));
    *out = s;
    return TDSEZ_OK;
}

tdsez_status tdsez_system2d_size(tdsez_system2d s, int* nx, int* ny, int* halfbw) {
    if (!s) return fail(TDSEZ_EINVAL, "system is NULL");
    if (nx) *nx = s->Nx;
    if (ny) *ny = s->Ny;
    if (halfbw) *halfbw = s->p;
    return TDSEZ_OK;
}

tdsez_status tdsez_get_v2(tdsez_system2d s, double* host_out) {
    if (!s || !host_out) return fail(TDSEZ_EINVAL, "NULL argument");
    const int p = s->p, w = 2 * p + 1, nh = half_count(p);
    const long long plane = (long long)s->Nx * s->Ny;
    std::vector<double> h((size_t)nh * plane);
    TDSEZ_HIP_TRY(hipMemcpy(h.data(), s->d_V2h, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
    for (int iy = 0; iy < s->Ny; ++iy)
        for (int ix = 0; ix < s->Nx; ++ix) {
            const long long row = (long long)iy * s->Nx + ix;
            for (int dy = -p; dy <= p; ++dy)
                for (int dx = -p; dx <= p; ++dx) {
                    const int jy = iy + dy, jx = ix + dx;
                    double v = 0.0;
                    if (jy >= 0 && jy < s->Ny && jx >= 0 && jx < s->Nx) {
                        if (dy > 0 || (dy == 0 && dx >= 0))
                            v = h[(size_t)half_index(p, dy, dx) * plane + row];
                        else
                            v = h[(size_t)half_index(p, -dy, -dx) * plane + (long long)jy * s->Nx + jx];
                    }
                    host_out[row * w * w + (dy + p) * w + (dx + p)] = v;
                }
        }
    return TDSEZ_OK;
}

tdsez_status tdsez_propagate_2d(tdsez_system2d s, double* psi, const double* E, double dt, int nsteps,
                                tdsez_precision prec, unsigned obs, double* obs_out, double tol, int maxit,
                                void* stream_v) {
    if (!s || !psi || !E) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TDSEZ_EINVAL, "dt must be > 0");
    if (nsteps < 0) return fail(TDSEZ_EINVAL, "nsteps < 0");
    if (obs & ~3u) return fail(TDSEZ_EINVAL, "2D observables: TDSEZ_OBS_NORM and TDSEZ_OBS_DIPOLE only");
    if (obs && !obs_out) return fail(TDSEZ_EINVAL, "obs requested but obs_out is NULL");
    if (prec != TDSEZ_FP64 && prec != TDSEZ_FP32_REFINED) return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    if (!(tol > 0.0) || maxit < 1) return fail(TDSEZ_EINVAL, "tol must be > 0 and maxit >= 1");
    const bool mixed = prec == TDSEZ_FP32_REFINED;
    if (mixed) {
        if (tdsez_status st = ensure_fp32(s)) return st;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    const int Nx = s->Nx, Ny = s->Ny, p = s->p;
    const long long n = (long long)Nx * Ny;
    double* w = s->d_work;
    auto vre = [&](int k) { return w + (size_t)(2 * k) * n; };
    auto vim = [&](int k) { return w + (size_t)(2 * k + 1) * n; };
    float* w32 = s->d_work32;
    auto fre = [&](int k) { return w32 + (size_t)(2 * k) * n; };
    auto fim = [&](int k) { return w32 + (size_t)(2 * k + 1) * n; };
    enum { C = 0, X = 1, R = 2, Z = 3, PV = 4, Q = 5, B = 6, T1 = 7, T2 = 8 };   // FP64 vectors
    enum { R32 = 0, Z32 = 1, P32 = 2, Q32 = 3, E32 = 4, T132 = 5, T232 = 6 };  // FP32 vectors
    double* outer = s->d_sc;             // FP64 solve / outer refinement scalars
    double* inner = s->d_sc + kScBlock;  // FP32 inner solve scalars
    const double* fo = outer + kScDone;  // "converged" flags
    const double* fi = inner + kScDone;
    // host-visible per-step log (coherent pinned memory written by the
    // device, read by the host without waiting)
    int* log = nullptr;
    int* log_dev = nullptr;
    TDSEZ_HIP_TRY(hipHostMalloc((void**)&log, sizeof(int) * 4 * ((size_t)nsteps + 1),
                                hipHostMallocMapped | hipHostMallocCoherent));
    struct LogGuard {
        int* p;
        ~LogGuard() { (void)hipHostFree(p); }
    } guard{log};
    for (size_t i = 0; i < 4 * ((size_t)nsteps + 1); ++i) log[i] = -1;
    TDSEZ_HIP_TRY(hipHostGetDevicePointer((void**)&log_dev, log, 0));
    const int g = grid_for(n);
    {
        // scalars: flags and counters cleared, tolerances set, no latched error
        double init[2 * kScBlock] = {};
        init[kScTol2] = tol * tol;
        TDSEZ_HIP_TRY(hipMemcpyAsync(s->d_sc, init, sizeof(init), hipMemcpyHostToDevice, stream));
        TDSEZ_HIP_TRY(hipMemsetAsync(s->d_status, 0, sizeof(int) * 4, stream));
        TDSEZ_HIP_TRY(hipStreamSynchronize(stream));  // init is a stack array
    }
    to_planar_kernel<<<g, 256, 0, stream>>>(psi, n, vre(C), vim(C));
    copy_kernel<double><<<g, 256, 0, stream>>>(2 * n, nullptr, vre(X), nullptr);
    const dim3 sgrid = stencil_grid<double>(Nx, Ny);
    const dim3 sgrid32 = stencil_grid<float>(Nx, Ny);
    const int nblk = (int)(sgrid.x * sgrid.y);
    const double alpha = 0.5 * dt;
    const double* Sx = s->ax.d_band[0];
    const double* Tx = s->ax.d_band[1];
    const double* Dx = s->ax.d_band[3];
    const double* Sy = s->ay.d_band[0];
    const double* Ty = s->ay.d_band[1];
    const long long bx = (long long)Nx * (p + 1), by = (long long)Ny * (p + 1);
    const float* b32 = s->d_bands32;
    // out = w y + a S2 in + b (T2 + V2 + Eb D2) in, in FP64 (apply) or FP32
    // (apply32); skipped when *flag is set
    auto apply = [&](int in, int yv, double wr, double wi, double ar, double ai, double br, double bi, double Eb,
                     int outv, double* obsp, const double* flag) {
        const double* yr = yv >= 0 ? vre(yv) : nullptr;
        const double* yi = yv >= 0 ? vim(yv) : nullptr;
        switch (p) {
#define TD2_CASE(PV_)                                                                                        \
    case PV_:                                                                                                \
        apply_kernel<PV_, double><<<sgrid, kStencilThreads, 0, stream>>>(                                    \
            Nx, Ny, Sx, Tx, Dx, Sy, Ty, s->d_V2h, vre(in), vim(in), yr, yi, wr, wi, ar, ai, br, bi, Eb,       \
            vre(outv), vim(outv), obsp, flag);                                                               \
        break;
            TD2_CASE(1) TD2_CASE(2) TD2_CASE(3) TD2_CASE(4) TD2_CASE(5) TD2_CASE(6) TD2_CASE(7)
#undef TD2_CASE
            default: break;
        }
    };
    auto apply32 = [&](int in, double ar, double ai, double br, double bi, double Eb, int outv) {
        switch (p) {
#define TD2_CASE(PV_)                                                                                         \
    case PV_:                                                                                                 \
        apply_kernel<PV_, float><<<sgrid32, kStencilThreads, 0, stream>>>(                                      \
            Nx, Ny, b32, b32 + bx, b32 + 2 * bx, b32 + 3 * bx, b32 + 3 * bx + by, s->d_V2h32, fre(in), fim(in), \
            nullptr, nullptr, 0.f, 0.f, (float)ar, (float)ai, (float)br, (float)bi, (float)Eb, fre(outv),      \
            fim(outv), nullptr, fi);                                                                          \
        break;
            TD2_CASE(1) TD2_CASE(2) TD2_CASE(3) TD2_CASE(4) TD2_CASE(5) TD2_CASE(6) TD2_CASE(7)
#undef TD2_CASE
            default: break;
        }
    };
    // partial sums of a dot into d_part, then the one-block scalar update
    auto dot_dev = [&](int u, int v, bool abs2, int mode, bool count, const double* flag) {
        dot_kernel<double><<<kRedBlocks, kRedThreads, 0, stream>>>(n, vre(u), vim(u), vre(v), vim(v), abs2, s->d_part,
                                                                   flag);
        cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(s->d_part, kRedBlocks, mode, outer, count);
    };
    auto dot32 = [&](int u, int v, bool abs2, int mode, bool count) {
        dot_kernel<float><<<kRedBlocks, kRedThreads, 0, stream>>>(n, fre(u), fim(u), fre(v), fim(v), abs2, s->d_part, fi);
        cocg_scalar_kernel<<<1, kRedThreads, 0, stream>>>(s->d_part, kRedBlocks, mode, inner, count);
    };
    // z = P^-1 r: four per-axis contractions (section II.C tensor structure),
    // the scaling fused into the second
    const dim3 ggrid((Nx + kGemmTile - 1) / kGemmTile, (Ny + kGemmTile - 1) / kGemmTile);
    auto precond = [&](int rin, int zout) {
        fdm_gemm_kernel<double, false, false><<<ggrid, kGemmThreads, 0, stream>>>(
            Ny, Nx, Nx, s->d_Qx, 1, Nx, vre(rin), vim(rin), vre(T1), vim(T1), 0.0, nullptr, nullptr, fo);
        fdm_gemm_kernel<double, true, true><<<ggrid, kGemmThreads, 0, stream>>>(
            Ny, Nx, Ny, s->d_Qy, Ny, 1, vre(T1), vim(T1), vre(T2), vim(T2), alpha, s->d_lx, s->d_my, fo);
        fdm_gemm_kernel<double, false, false><<<ggrid, kGemmThreads, 0, stream>>>(
            Ny, Nx, Nx, s->d_Qx, Nx, 1, vre(T2), vim(T2), vre(T1), vim(T1), 0.0, nullptr, nullptr, fo);
        fdm_gemm_kernel<double, true, false><<<ggrid, kGemmThreads, 0, stream>>>(
            Ny, Nx, Ny, s->d_Qy, 1, Ny, vre(T1), vim(T1), vre(zout), vim(zout), 0.0, nullptr, nullptr, fo);
    };
    auto precond32 = [&](int rin, int zout) {
        fdm_gemm_kernel<float, false, false><<<ggrid, kGemmThreads, 0, stream>>>(
            Ny, Nx, Nx, s->d_Qx32, 1, Nx, fre(rin), fim(rin), fre(T132), fim(T132), 0.0, nullptr, nullptr, fi);
        fdm_gemm_kernel<float, true, true><<<ggrid, kGemmThreads, 0, stream>>>(
            Ny, Nx, Ny, s->d_Qy32, Ny, 1, fre(T132), fim(T132), fre(T232), fim(T232), alpha, s->d_lx, s->d_my, fi);
        fdm_gemm_kernel<float, false, false><<<ggrid, kGemmThreads, 0, stream>>>(
            Ny, Nx, Nx, s->d_Qx32, Nx, 1, fre(T232), fim(T232), fre(T132), fim(T132), 0.0, nullptr, nullptr, fi);
        fdm_gemm_kernel<float, true, false><<<ggrid, kGemmThreads, 0, stream>>>(
            Ny, Nx, Ny, s->d_Qy32, 1, Ny, fre(T132), fim(T132), fre(zout), fim(zout), 0.0, nullptr, nullptr, fi);
    };
    std::vector<double> Eh((size_t)nsteps + 1);
    TDSEZ_HIP_TRY(hipMemcpyAsync(Eh.data(), E, sizeof(double) * Eh.size(), hipMemcpyDeviceToHost, stream));
    TDSEZ_HIP_TRY(hipStreamSynchronize(stream));
    // FP32 inner solves reduce the FP64 residual by this factor per sweep
    // (near the FP32 accuracy of the inner operator)
    constexpr double kInnerTol = 1e-5;
    // iteration budgets of a step: a margin above the largest count among
    // the last logged steps (the log lags the host by however many steps are
    // queued), capped by maxit; sweeps: a fixed budget
    constexpr int kMargin = 3, kWindow = 8;
    int known = -1;  // last step whose log entry has arrived
    auto budget = [&](int col, int first, int margin) {
        volatile const int* lg = log;
        while (known + 1 < nsteps && lg[4 * (known + 1) + 0] >= 0) ++known;
        int mx = -1;
        for (int j = known; j >= 0 && j > known - kWindow; --j) mx = std::max(mx, (int)lg[4 * j + col]);
        const int b = mx < 0 ? first : mx + margin;
        return std::min(std::max(b, 1), maxit);
    };
    for (int step = 0; step <= nsteps; ++step) {
        const double Eb = step < nsteps ? 0.5 * (Eh[step] + Eh[step + 1]) : Eh[step];
        // b = -i dt H c (and the observables of c)
        apply(C, -1, 0.0, 0.0, 0.0, 0.0, 0.0, -2.0 * alpha, Eb, B, s->d_obs_part, nullptr);
        if (obs) obs_finish_kernel<<<1, kRedThreads, 0, stream>>>(s->d_obs_part, nblk, obs_out + 3 * (size_t)step, obs);
        if (step == nsteps) break;
        // A x = b, A = S2 + i a H, warm start from the previous increment
        apply(X, B, 1.0, 0.0, -1.0, 0.0, 0.0, -alpha, Eb, R, nullptr, nullptr);  // r = b - A x
        dot_dev(B, B, true, 4, false, nullptr);
        dot_dev(R, R, true, 3, false, nullptr);
        if (!mixed) {
            // COCG in FP64; every kernel returns once the residual has met tol
            const int K = budget(0, 12, kMargin);
            precond(R, Z);
            copy_kernel<double><<<g, 256, 0, stream>>>(2 * n, vre(Z), vre(PV), fo);
            dot_dev(R, Z, false, 0, false, fo);
            for (int it = 0; it < K; ++it) {
                apply(PV, -1, 0.0, 0.0, 1.0, 0.0, 0.0, alpha, Eb, Q, nullptr, fo);  // q = A p
                dot_dev(PV, Q, false, 1, false, fo);                                // alpha = rho / p^T q
                cocg_xr_dev_kernel<double><<<g, 256, 0, stream>>>(n, outer, vre(PV), vim(PV), vre(Q), vim(Q),
                                                                  vre(X), vim(X), vre(R), vim(R));
                dot_dev(R, R, true, 3, true, fo);                                   // converged?
                precond(R, Z);
                dot_dev(R, Z, false, 2, false, fo);  // beta = r^T z / rho, rho = r^T z
                cocg_p_dev_kernel<double><<<g, 256, 0, stream>>>(n, outer, vre(Z), vim(Z), vre(PV), vim(PV));
            }
        } else {
            // iterative refinement: FP64 residual r = b - A x, FP32 COCG on
            // A e = r (same preconditioner in FP32), x += e
            const int Ki = budget(1, 12, kMargin);
            const int Ks = budget(2, 3, 1);
            for (int sw = 0; sw < Ks; ++sw) {
                sweep_start_kernel<<<1, 64, 0, stream>>>(outer, inner, kInnerTol);
                to_fp32_kernel<<<g, 256, 0, stream>>>(2 * n, vre(R), fre(R32), fo);
                copy_kernel<float><<<g, 256, 0, stream>>>(2 * n, nullptr, fre(E32), fo);
                dot32(R32, R32, true, 4, false);
                precond32(R32, Z32);
                copy_kernel<float><<<g, 256, 0, stream>>>(2 * n, fre(Z32), fre(P32), fi);
                dot32(R32, Z32, false, 0, false);
                for (int it = 0; it < Ki; ++it) {
                    apply32(P32, 1.0, 0.0, 0.0, alpha, Eb, Q32);  // q = A p
                    dot32(P32, Q32, false, 1, false);
                    cocg_xr_dev_kernel<float><<<g, 256, 0, stream>>>(n, inner, fre(P32), fim(P32), fre(Q32), fim(Q32),
                                                                     fre(E32), fim(E32), fre(R32), fim(R32));
                    dot32(R32, R32, true, 3, true);
                    precond32(R32, Z32);
                    dot32(R32, Z32, false, 2, false);
                    cocg_p_dev_kernel<float><<<g, 256, 0, stream>>>(n, inner, fre(Z32), fim(Z32), fre(P32), fim(P32));
                }
                add_kernel<float><<<g, 256, 0, stream>>>(n, fre(E32), fim(E32), vre(X), vim(X), fo);
                apply(X, B, 1.0, 0.0, -1.0, 0.0, 0.0, -alpha, Eb, R, nullptr, fo);  // r = b - A x
                dot_dev(R, R, true, 3, false, fo);
            }
        }
        step_end_kernel<<<1, 64, 0, stream>>>(outer, inner, step, s->d_status, log_dev);
        add_kernel<double><<<g, 256, 0, stream>>>(n, vre(X), vim(X), vre(C), vim(C), nullptr);
        TDSEZ_HIP_TRY(hipGetLastError());
    }
    from_planar_kernel<<<g, 256, 0, stream>>>(vre(C), vim(C), n, psi);
    TDSEZ_HIP_TRY(hipGetLastError());
    // the call ends here: statistics and the latched convergence failure
    TDSEZ_HIP_TRY(hipStreamSynchronize(stream));
    int stat[4] = {0, 0, 0, 0};
    TDSEZ_HIP_TRY(hipMemcpy(stat, s->d_status, sizeof(stat), hipMemcpyDeviceToHost));
    for (int st = 0; st < nsteps; ++st) {
        const int it = mixed ? log[4 * st + 3] : log[4 * st + 0];
        s->iters_total += it;
        s->iters_max = std::max(s->iters_max, it);
        s->sweeps_total += log[4 * st + 2];
        s->steps_total += 1;
    }
    if (stat[0] == TDSEZ_ENOCONV)
        return fail(TDSEZ_ENOCONV, "2D step %d: residual above %g after its iteration budget (maxit %d)", stat[1], tol,
                    maxit);
    return TDSEZ_OK;
}

tdsez_status tdsez_system2d_stats(tdsez_system2d s, long* steps, long* iterations, int* max_iterations,
                                  long* sweeps) {
    if (!s) return fail(TDSEZ_EINVAL, "system is NULL");
    if (steps) *steps = (long)s->steps_total;
    if (iterations) *iterations = (long)s->iters_total;
    if (max_iterations) *max_iterations = s->iters_max;
    if (sweeps) *sweeps = (long)s->sweeps_total;
    s->steps_total = s->iters_total = s->sweeps_total = 0;
    s->iters_max = 0;
    return TDSEZ_OK;
}

void tdsez_system2d_destroy(tdsez_system2d s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    free2d(s);
    delete s;
}

}  // extern "C"
