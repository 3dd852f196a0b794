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
#include <cmath>
#include <cstring>
#include <vector>

#include "tdsez_krylov.hpp"

namespace tdsez {
namespace {

// number of stored stencil offsets: (dy, dx) with dy > 0, or dy == 0 and dx >= 0
__host__ __device__ inline int half_count(int p) { return (p + 1) + p * (2 * p + 1); }
// index of a stored offset
__host__ __device__ inline int half_index(int p, int dy, int dx) {
    return dy == 0 ? dx : (p + 1) + (dy - 1) * (2 * p + 1) + (dx + p);
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
// Re c^H D2 c (FP64); with dotp != null (and obs null) the partial sum of
// c^T out (unconjugated, FP64).  Four tiles per CU (<= 128 VGPRs) let the 1024 tiles
// of a 512 x 512 grid run in one round.
template <int PP, typename FT>
__global__ __launch_bounds__(kStencilThreads, 4) void apply_kernel(
    int Nx, int Ny, const FT* __restrict__ Sxb, const FT* __restrict__ Txb, const FT* __restrict__ Dxb,
    const FT* __restrict__ Syb, const FT* __restrict__ Tyb, const FT* __restrict__ V2h, const FT* __restrict__ cre,
    const FT* __restrict__ cim, const FT* __restrict__ yre, const FT* __restrict__ yim, FT wre, FT wim, FT are,
    FT aim, FT bre, FT bim, FT Ebar, FT* __restrict__ ore, FT* __restrict__ oim, double* __restrict__ obs,
    const double* __restrict__ flag, double* __restrict__ dotp) {
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
        const double c0r = tre[cy][cx], c0i = tim[cy][cx];
        if (obs) {
            nu = c0r * (double)Sr + c0i * (double)Si;
            dip = c0r * (double)Dr + c0i * (double)Di;
        } else if (dotp) {
            // c^T (A c), unconjugated (the Krylov step's p^T q)
            nu = c0r * (double)accr - c0i * (double)acci;
            dip = c0r * (double)acci + c0i * (double)accr;
        }
    }
    double* const red_out = obs ? obs : dotp;
    if (red_out) {
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
            red_out[2 * blk] = red[0][0];
            red_out[2 * blk + 1] = red[1][0];
        }
    }
}

// Per-tile partial sums of Re c^H G2 c for a half stencil G2 (the force
// stencil of dV/dx, section IV.A): the potential stage of apply_kernel with
// G2 in place of V2, then Re(conj(c_i) (G2 c)_i) summed over the tile
// (FP64, fixed order).
template <int PP>
__global__ __launch_bounds__(kStencilThreads) void form2_kernel(int Nx, int Ny, const double* __restrict__ G2h,
                                                                const double* __restrict__ cre,
                                                                const double* __restrict__ cim,
                                                                double* __restrict__ part) {
    constexpr int TX = TileShape<double>::TX, TY = TileShape<double>::TY;
    constexpr int K = 2 * PP + 1;
    constexpr int WX = TX + 2 * PP, WY = TY + 2 * PP;
    __shared__ double tre[WY][WX], tim[WY][WX];
    __shared__ double red[kStencilThreads];
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int ix = x0 + tx, iy = y0 + ty;
    const long long plane = (long long)Nx * Ny;
    for (int t = threadIdx.x; t < WX * WY; t += kStencilThreads) {
        const int ly = t / WX, lx = t % WX;
        const int gy = y0 + ly - PP, gx = x0 + lx - PP;
        double vr = 0, vi = 0;
        if (gy >= 0 && gy < Ny && gx >= 0 && gx < Nx) {
            vr = cre[(long long)gy * Nx + gx];
            vi = cim[(long long)gy * Nx + gx];
        }
        tre[ly][lx] = vr;
        tim[ly][lx] = vi;
    }
    __syncthreads();
    const int ixc = ix < Nx ? ix : Nx - 1, iyc = iy < Ny ? iy : Ny - 1;
    const long long row = (long long)iyc * Nx + ixc;
    const int cy = ty + PP, cx = tx + PP;
    double gr = 0, gi = 0;
    {
        const double v0 = G2h[row];
        gr += v0 * tre[cy][cx];
        gi += v0 * tim[cy][cx];
#pragma unroll
        for (int e = 1; e <= PP; ++e) {
            const double* __restrict__ pl = G2h + (long long)half_index(PP, 0, e) * plane;
            const int jx = ixc - e < 0 ? 0 : ixc - e;
            const double vd = pl[row];
            const double vm = pl[(long long)iyc * Nx + jx];
            gr += vd * tre[cy][cx + e] + vm * tre[cy][cx - e];
            gi += vd * tim[cy][cx + e] + vm * tim[cy][cx - e];
        }
    }
#pragma unroll 1
    for (int dy = 1; dy <= PP; ++dy) {
        const double* __restrict__ pl = G2h + (long long)half_index(PP, dy, -PP) * plane;
        const long long mrow = (long long)(iyc - dy < 0 ? 0 : iyc - dy) * Nx;
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
            const int e = kx - PP;
            int jx = ixc - e;
            jx = jx < 0 ? 0 : (jx >= Nx ? Nx - 1 : jx);
            const double vd = pl[(long long)kx * plane + row];
            const double vm = pl[(long long)kx * plane + mrow + jx];
            gr += vd * tre[cy + dy][cx + e] + vm * tre[cy - dy][cx - e];
            gi += vd * tim[cy + dy][cx + e] + vm * tim[cy - dy][cx - e];
        }
    }
    red[threadIdx.x] = (ix < Nx && iy < Ny) ? tre[cy][cx] * gr + tim[cy][cx] * gi : 0.0;
    __syncthreads();
    for (int s = kStencilThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

}  // namespace
}  // namespace tdsez

using namespace tdsez;

struct tdsez_system2d_s {
    SystemData ax, ay;         // per-axis 1D matrices (V = 0, m = 1)
    int Nx = 0, Ny = 0, p = 0, order = 0, nq = 0;
    double* d_V2h = nullptr;   // half stencil, [offset][row]
    double* d_G2h = nullptr;   // force stencil of dV/dx (half, [offset][row]), or nullptr
    double* d_acc_part = nullptr;  // per-tile partials of Re c^H G2 c
    double* d_Qx = nullptr;    // generalised eigenvectors (column-major), T Q = S Q Lambda
    double* d_Qy = nullptr;
    double* d_lx = nullptr;
    double* d_my = nullptr;
    double* d_work = nullptr;  // planar vectors: c, x, r, z, p, q, b, t1, t2 (2 planes each)
    double* d_part = nullptr;  // reduction partials
    double* d_obs_part = nullptr;
    double* d_dpart = nullptr;  // partial sums of the dot products fused into the operator and preconditioner
    double* d_sc = nullptr;    // COCG scalars and flags (device), two slot blocks
    int* d_status = nullptr;   // latched failure of a propagation: code, step
    // FP32 copies for TDSEZ_FP32_REFINED, made by the first such call
    float* d_V2h32 = nullptr;
    float* d_bands32 = nullptr;  // Sx, Tx, Dx (Nx (p+1) each), then Sy, Ty (Ny (p+1) each)
    float* d_Qx32 = nullptr;
    float* d_Qy32 = nullptr;
    float* d_work32 = nullptr;   // planar FP32 vectors: r, z, p, q, e, t1, t2 (2 planes each)
    rocblas_handle blas = nullptr;
    CnStats stats;
};

namespace {

void free2d(tdsez_system2d_s* s) {
    for (int m = 0; m < 6; ++m) {
        (void)hipFree(s->ax.d_band[m]);
        (void)hipFree(s->ay.d_band[m]);
    }
    (void)hipFree(s->ax.d_H0);
    (void)hipFree(s->ay.d_H0);
    (void)hipFree(s->d_V2h);
    (void)hipFree(s->d_G2h);
    (void)hipFree(s->d_acc_part);
    (void)hipFree(s->d_Qx);
    (void)hipFree(s->d_Qy);
    (void)hipFree(s->d_lx);
    (void)hipFree(s->d_my);
    (void)hipFree(s->d_work);
    (void)hipFree(s->d_part);
    (void)hipFree(s->d_obs_part);
    (void)hipFree(s->d_dpart);
    (void)hipFree(s->d_sc);
    (void)hipFree(s->d_status);
    (void)hipFree(s->d_V2h32);
    (void)hipFree(s->d_bands32);
    (void)hipFree(s->d_Qx32);
    (void)hipFree(s->d_Qy32);
    (void)hipFree(s->d_work32);
    if (s->blas) rocblas_destroy_handle(s->blas);
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

// The 2D operator and preconditioner for the shared step loop.
struct Op2D {
    tdsez_system2d_s* s;
    const CnWork& cw;
    double alpha;
    // out = w y + a S2 in + b (T2 + V2 + Eb D2) in
    int nblk_apply(bool fp32) const {
        const dim3 g = fp32 ? stencil_grid<float>(s->Nx, s->Ny) : stencil_grid<double>(s->Nx, s->Ny);
        return (int)(g.x * g.y);
    }
    int nblk_precond() const {
        return ((s->Nx + kGemmTile - 1) / kGemmTile) * ((s->Ny + kGemmTile - 1) / kGemmTile);
    }
    int accel(int in, double* part, hipStream_t stream) {
        if (!s->d_G2h) return 0;
        const dim3 g = stencil_grid<double>(s->Nx, s->Ny);
        switch (s->p) {
#define TD2_CASE(PV_)                                                                                        \
    case PV_:                                                                                                \
        form2_kernel<PV_><<<g, kStencilThreads, 0, stream>>>(s->Nx, s->Ny, s->d_G2h, cw.re(in), cw.im(in), part); \
        break;
            TD2_CASE(1) TD2_CASE(2) TD2_CASE(3) TD2_CASE(4) TD2_CASE(5) TD2_CASE(6) TD2_CASE(7)
#undef TD2_CASE
            default: return 0;
        }
        return (int)(g.x * g.y);
    }
    void apply(int in, int yv, double wr, double wi, double ar, double ai, double br, double bi, double Eb, int outv,
               double* obsp, const double* flag, hipStream_t stream, double* dotp = nullptr) {
        const int Nx = s->Nx, Ny = s->Ny;
        const double* yr = yv >= 0 ? cw.re(yv) : nullptr;
        const double* yi = yv >= 0 ? cw.im(yv) : nullptr;
        const dim3 sgrid = stencil_grid<double>(Nx, Ny);
        const double *Sx = s->ax.d_band[0], *Tx = s->ax.d_band[1], *Dx = s->ax.d_band[3];
        const double *Sy = s->ay.d_band[0], *Ty = s->ay.d_band[1];
        switch (s->p) {
#define TD2_CASE(PV_)                                                                                        \
    case PV_:                                                                                                \
        apply_kernel<PV_, double><<<sgrid, kStencilThreads, 0, stream>>>(                                    \
            Nx, Ny, Sx, Tx, Dx, Sy, Ty, s->d_V2h, cw.re(in), cw.im(in), yr, yi, wr, wi, ar, ai, br, bi, Eb,   \
            cw.re(outv), cw.im(outv), obsp, flag, dotp);                                                     \
        break;
            TD2_CASE(1) TD2_CASE(2) TD2_CASE(3) TD2_CASE(4) TD2_CASE(5) TD2_CASE(6) TD2_CASE(7)
#undef TD2_CASE
            default: break;
        }
    }
    void apply32(int in, double ar, double ai, double br, double bi, double Eb, int outv, const double* flag,
                 hipStream_t stream, double* dotp = nullptr) {
        const int Nx = s->Nx, Ny = s->Ny, p = s->p;
        const dim3 sgrid32 = stencil_grid<float>(Nx, Ny);
        const long long bx = (long long)Nx * (p + 1), by = (long long)Ny * (p + 1);
        const float* b32 = s->d_bands32;
        switch (p) {
#define TD2_CASE(PV_)                                                                                           \
    case PV_:                                                                                                   \
        apply_kernel<PV_, float><<<sgrid32, kStencilThreads, 0, stream>>>(                                        \
            Nx, Ny, b32, b32 + bx, b32 + 2 * bx, b32 + 3 * bx, b32 + 3 * bx + by, s->d_V2h32, cw.re32(in),        \
            cw.im32(in), nullptr, nullptr, 0.f, 0.f, (float)ar, (float)ai, (float)br, (float)bi, (float)Eb,      \
            cw.re32(outv), cw.im32(outv), nullptr, flag, dotp);                                                 \
        break;
            TD2_CASE(1) TD2_CASE(2) TD2_CASE(3) TD2_CASE(4) TD2_CASE(5) TD2_CASE(6) TD2_CASE(7)
#undef TD2_CASE
            default: break;
        }
    }
    // z = P^-1 r: four per-axis contractions (section II.C tensor structure),
    // the scaling 1 / (1 + i a (mu + lambda)) fused into the second
    template <typename FT>
    void precond_t(const FT* Qx, const FT* Qy, const FT* rr, const FT* ri, FT* t1r, FT* t1i, FT* t2r, FT* t2i, FT* zr,
                   FT* zi, const double* flag, hipStream_t stream, double* rzp) {
        const int Nx = s->Nx, Ny = s->Ny;
        const dim3 gg((Nx + kGemmTile - 1) / kGemmTile, (Ny + kGemmTile - 1) / kGemmTile);
        const FdmScale none{0, 0, 0, 0, nullptr, nullptr, nullptr, 1};
        const FdmScale cn{1.0, 0.0, 0.0, alpha, s->d_my, s->d_lx, nullptr, Nx};
        fdm_gemm_kernel<FT, false, false><<<gg, kGemmThreads, 0, stream>>>(Ny, Nx, Nx, Qx, 1, Nx, rr, ri, t1r, t1i, 0,
                                                                           0, none, flag);
        fdm_gemm_kernel<FT, true, true><<<gg, kGemmThreads, 0, stream>>>(Ny, Nx, Ny, Qy, Ny, 1, t1r, t1i, t2r, t2i, 0, 0,
                                                                         cn, flag);
        fdm_gemm_kernel<FT, false, false><<<gg, kGemmThreads, 0, stream>>>(Ny, Nx, Nx, Qx, Nx, 1, t2r, t2i, t1r, t1i, 0,
                                                                           0, none, flag);
        if (rzp)
            fdm_gemm_kernel<FT, true, false, true><<<gg, kGemmThreads, 0, stream>>>(
                Ny, Nx, Ny, Qy, 1, Ny, t1r, t1i, zr, zi, 0, 0, none, flag, rr, ri, rzp);
        else
            fdm_gemm_kernel<FT, true, false><<<gg, kGemmThreads, 0, stream>>>(Ny, Nx, Ny, Qy, 1, Ny, t1r, t1i, zr, zi, 0,
                                                                              0, none, flag);
    }
    void precond(int rin, int zout, const double* flag, hipStream_t stream, double* rzp = nullptr) {
        precond_t<double>(s->d_Qx, s->d_Qy, cw.re(rin), cw.im(rin), cw.re(kT1), cw.im(kT1), cw.re(kT2), cw.im(kT2),
                          cw.re(zout), cw.im(zout), flag, stream, rzp);
    }
    void precond32(int rin, int zout, const double* flag, hipStream_t stream, double* rzp = nullptr) {
        precond_t<float>(s->d_Qx32, s->d_Qy32, cw.re32(rin), cw.im32(rin), cw.re32(kT132), cw.im32(kT132),
                         cw.re32(kT232), cw.im32(kT232), cw.re32(zout), cw.im32(zout), flag, stream, rzp);
    }
};

}  // namespace

extern "C" {

tdsez_status tdsez_assemble_2d(const double* breaks_x, int nbx, const double* breaks_y, int nby, int order, int nq,
                               const double* V_q, const double* dVx_q, tdsez_system2d* out) {
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
    for (long long i = 0; dVx_q && i < nqx * nqy; ++i)
        if (!std::isfinite(dVx_q[i])) return fail(TDSEZ_EINVAL, "dVx_q[%lld] is not finite", i);
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
        if (dVx_q) {
            H(hipMalloc(&s->d_G2h, sizeof(double) * (size_t)half_count(p) * Nx * Ny));
            const dim3 g64 = stencil_grid<double>(Nx, Ny);
            H(hipMalloc(&s->d_acc_part, sizeof(double) * (size_t)g64.x * g64.y));
        }
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
            if (dVx_q) {
                // the force stencil: the same integral with dV/dx sampled
                H(hipDeviceSynchronize());
                H(hipMemcpy(dVq, dVx_q, sizeof(double) * nqx * nqy, hipMemcpyHostToDevice));
                v2_kernel<<<4096, 256>>>(Nx, Ny, p, nq, nbx - 1, nby - 1, dbx, dby, dgw, dBx, dBy, dVq, s->d_G2h);
                H(hipGetLastError());
            }
            H(hipDeviceSynchronize());
        }
        clean();
        if (he != hipSuccess) return bail(fail(TDSEZ_EHIP, "2D assembly: %s", hipGetErrorString(he)));
    }
    st = axis_eigen(s->blas, s->ax, &s->d_Qx, &s->d_lx);
    if (st) return bail(st);
    st = axis_eigen(s->blas, s->ay, &s->d_Qy, &s->d_my);
    if (st) return bail(st);
    const long long plane = (long long)Nx * Ny;
    if (hipMalloc(&s->d_work, sizeof(double) * (size_t)plane * 2 * 9) != hipSuccess ||
        hipMalloc(&s->d_part, sizeof(double) * 2 * kRedBlocks) != hipSuccess ||
        hipMalloc(&s->d_sc, sizeof(double) * 2 * kScBlock) != hipSuccess ||
        hipMalloc(&s->d_status, sizeof(int) * 4) != hipSuccess ||
        hipMalloc(&s->d_obs_part, sizeof(double) * 2 * (size_t)stencil_grid<double>(Nx, Ny).x *
                                      stencil_grid<double>(Nx, Ny).y) != hipSuccess)
        return bail(fail(TDSEZ_ENOMEM, "2D workspace allocation failed"));
    {
        const dim3 g64 = stencil_grid<double>(Nx, Ny), g32 = stencil_grid<float>(Nx, Ny);
        const size_t nb = std::max<size_t>({(size_t)g64.x * g64.y, (size_t)g32.x * g32.y,
                                            (size_t)((Nx + kGemmTile - 1) / kGemmTile) * ((Ny + kGemmTile - 1) / kGemmTile)});
        if (hipMalloc(&s->d_dpart, sizeof(double) * 2 * nb) != hipSuccess)
            return bail(fail(TDSEZ_ENOMEM, "2D workspace allocation failed"));
    }
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

tdsez_status tdsez_time_apply_2d(tdsez_system2d s, tdsez_precision prec, int reps, void* stream_v, double* ms_out) {
    if (!s || !ms_out) return fail(TDSEZ_EINVAL, "NULL argument");
    if (reps < 1) return fail(TDSEZ_EINVAL, "reps must be >= 1");
    if (prec != TDSEZ_FP64 && prec != TDSEZ_FP32_REFINED) return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    const bool mixed = prec == TDSEZ_FP32_REFINED;
    if (mixed) {
        if (tdsez_status st = ensure_fp32(s)) return st;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    CnWork cw;
    cw.n = (long long)s->Nx * s->Ny;
    cw.w = s->d_work;
    cw.w32 = s->d_work32;
    Op2D op{s, cw, 0.0};
    const int g = grid_for(2 * cw.n);
    // q = A p as in a Krylov iteration (inputs: a filled vector)
    if (mixed) copy_kernel<float><<<g, 256, 0, stream>>>(2 * cw.n, nullptr, cw.re32(kP32), nullptr);
    else copy_kernel<double><<<g, 256, 0, stream>>>(2 * cw.n, nullptr, cw.re(kP), nullptr);
    hipEvent_t e0, e1;
    TDSEZ_HIP_TRY(hipEventCreate(&e0));
    TDSEZ_HIP_TRY(hipEventCreate(&e1));
    TDSEZ_HIP_TRY(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r) {
        if (mixed) op.apply32(kP32, 1.0, 0.0, 0.0, 0.005, 0.01, kQ32, nullptr, stream);
        else op.apply(kP, -1, 0.0, 0.0, 1.0, 0.0, 0.0, 0.005, 0.01, kQ, nullptr, nullptr, stream);
    }
    TDSEZ_HIP_TRY(hipEventRecord(e1, stream));
    TDSEZ_HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    TDSEZ_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = (double)ms / reps;
    return TDSEZ_OK;
}

tdsez_status tdsez_propagate_2d(tdsez_system2d s, double* psi, const double* E, double dt, int nsteps,
                                tdsez_precision prec, unsigned obs, double* obs_out, double tol, int maxit,
                                void* stream_v) {
    if (!s || !psi || !E) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TDSEZ_EINVAL, "dt must be > 0");
    if (nsteps < 0) return fail(TDSEZ_EINVAL, "nsteps < 0");
    if (obs & ~7u) return fail(TDSEZ_EINVAL, "unknown observable bits 0x%x", obs);
    if ((obs & TDSEZ_OBS_ACCEL) && !s->d_G2h)
        return fail(TDSEZ_EUNSUPPORTED, "the acceleration needs dV/dx (dVx_q at tdsez_assemble_2d)");
    if (obs && !obs_out) return fail(TDSEZ_EINVAL, "obs requested but obs_out is NULL");
    if (prec != TDSEZ_FP64 && prec != TDSEZ_FP32_REFINED) return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    if (!(tol > 0.0) || maxit < 1) return fail(TDSEZ_EINVAL, "tol must be > 0 and maxit >= 1");
    const bool mixed = prec == TDSEZ_FP32_REFINED;
    if (mixed) {
        if (tdsez_status st = ensure_fp32(s)) return st;
    }
    CnWork cw;
    cw.n = (long long)s->Nx * s->Ny;
    cw.w = s->d_work;
    cw.w32 = s->d_work32;
    cw.part = s->d_part;
    cw.sc = s->d_sc;
    cw.status = s->d_status;
    cw.obs_part = s->d_obs_part;
    cw.acc_part = s->d_acc_part;
    cw.dpart = s->d_dpart;
    const dim3 sgrid = stencil_grid<double>(s->Nx, s->Ny);
    cw.nblk_obs = (int)(sgrid.x * sgrid.y);
    Op2D op{s, cw, 0.5 * dt};
    return cn_cocg_propagate(cw, op, psi, E, dt, nsteps, mixed, obs, obs_out, tol, maxit, (hipStream_t)stream_v,
                             &s->stats, "2D");
}

tdsez_status tdsez_system2d_stats(tdsez_system2d s, long* steps, long* iterations, int* max_iterations,
                                  long* sweeps) {
    if (!s) return fail(TDSEZ_EINVAL, "system is NULL");
    if (steps) *steps = (long)s->stats.steps_total;
    if (iterations) *iterations = (long)s->stats.iters_total;
    if (max_iterations) *max_iterations = s->stats.iters_max;
    if (sweeps) *sweeps = (long)s->stats.sweeps_total;
    s->stats = CnStats();
    return TDSEZ_OK;
}

void tdsez_system2d_destroy(tdsez_system2d s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    free2d(s);
    delete s;
}

}  // extern "C"
