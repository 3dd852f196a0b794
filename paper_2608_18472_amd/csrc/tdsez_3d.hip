// Three-dimensional tensor-product propagation (constant mass, x-polarised
// field): Crank-Nicolson steps of section V.B on the basis
// N_ix(x) N_iy(y) N_iz(z) of the tensor-product construction in section
// II.C -- the workload of the strong-scaling study in section VI (Table II:
// hydrogen on 97 cubic splines per axis).
//
// Matrices, from the per-axis half bands (tdsez_assemble.hip) and the
// potential assembled here:
//   S3 = Sz (x) Sy (x) Sx,  T3 = Sz Sy Tx + Sz Ty Sx + Tz Sy Sx,
//   D3 = Sz Sy Dx,  V3[i][j] = sum_q w_q V(q) N_i(q) N_j(q),
// unknown (iz, iy, ix) at row (iz Ny + iy) Nx + ix.  A row of V3 couples the
// (2p+1)^3 neighbours j = i + (dz, dy, dx), |d*| <= p.  V3 is symmetric, so
// only the offsets from the centre onwards in (dz, dy, dx) lexicographic
// order are stored ((w^3 + 1) / 2 of them, w = 2p + 1), one plane of N rows
// per offset; V3[i][i - d] is read as V3[i - d][i] from the plane of d at
// row i - d.
//
// Assembly is sum-factorised axis by axis over slabs of z quadrature
// points: A1[qz][qy][ix][dx] sums the x quadrature, A2[qz][iy][dy][ix][dx]
// the y quadrature, and the z sum adds the slab into V3, so an entry costs
// O(p nq) per axis instead of O((p nq)^3).
//
// The step loop, the COCG kernels and the MFMA per-axis contractions are
// those of the 2D path (tdsez_krylov.hpp).  The preconditioner is the exact
// inverse of the separable part S3 + i a T3: with T Q = S Q Lambda per axis,
//   P^-1 R = (Qz Qy Qx) [ (Qz^T Qy^T Qx^T R) / (1 + i a (lx + my + nz)) ],
// six contractions (x; y per z plane; z with the scaling fused; and back).
#include <cmath>
#include <cstring>
#include <vector>

#include "tdsez_krylov.hpp"

namespace tdsez {
namespace {

// ------------------------------------------------------------------ stencil
// Number of stored offsets of the half stencil and the index of an offset.
__host__ __device__ inline int half3_count(int p) {
    const int w = 2 * p + 1;
    return (w * w * w + 1) / 2;
}
__host__ __device__ inline int full3_index(int p, int dz, int dy, int dx) {
    const int w = 2 * p + 1;
    return ((dz + p) * w + (dy + p)) * w + (dx + p);
}

// Overlapping spans of global B-splines ga, gb (support spans g - p .. g) on
// nel spans, clipped to [lo, hi]; empty when e0 > e1.
__device__ inline void span_overlap(int ga, int gb, int p, int nel, int lo, int hi, int* e0, int* e1) {
    const int gh = ga > gb ? ga : gb, gl = ga > gb ? gb : ga;
    int a = gh - p, b = gl;
    if (a < 0) a = 0;
    if (b > nel - 1) b = nel - 1;
    if (a < lo) a = lo;
    if (b > hi) b = hi;
    *e0 = a;
    *e1 = b;
}

// A1[lz][qy][ix][kx] = sum over x quadrature of w N_ix N_(ix+dx) V, for the
// slab's z quadrature points qz0 + lz (dx = kx - p; zero for a neighbour
// outside the grid).  Global B-spline index = unknown + 1.
__global__ void v3_a1_kernel(int Nx, int p, int nq, int nelx, int NQy, int qz0, int nqz,
                             const double* __restrict__ brx, const double* __restrict__ gw,
                             const double* __restrict__ Bx, const double* __restrict__ Vq,
                             double* __restrict__ A1) {
    const int w = 2 * p + 1;
    const long long NQx = (long long)nelx * nq;
    const long long total = (long long)nqz * NQy * Nx * w;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int kx = (int)(e % w);
        long long t = e / w;
        const int ix = (int)(t % Nx);
        t /= Nx;
        const int qy = (int)(t % NQy);
        const int lz = (int)(t / NQy);
        const int jx = ix + kx - p;
        double sum = 0.0;
        if (jx >= 0 && jx < Nx) {
            const int ga = ix + 1, gb = jx + 1;
            int e0, e1;
            span_overlap(ga, gb, p, nelx, 0, nelx - 1, &e0, &e1);
            const double* __restrict__ vrow = Vq + ((long long)(qz0 + lz) * NQy + qy) * NQx;
            for (int ex = e0; ex <= e1; ++ex) {
                const double hx = 0.5 * (brx[ex + 1] - brx[ex]);
                for (int q = 0; q < nq; ++q) {
                    const long long iq = (long long)ex * nq + q;
                    sum += gw[q] * hx * Bx[iq * (p + 1) + (ga - ex)] * Bx[iq * (p + 1) + (gb - ex)] * vrow[iq];
                }
            }
        }
        A1[e] = sum;
    }
}

// A2[lz][iy][ky][ix][kx] = sum over y quadrature of w N_iy N_(iy+dy) A1.
__global__ void v3_a2_kernel(int Nx, int Ny, int p, int nq, int nely, int nqz, const double* __restrict__ bry,
                             const double* __restrict__ gw, const double* __restrict__ By,
                             const double* __restrict__ A1, double* __restrict__ A2) {
    const int w = 2 * p + 1;
    const long long NQy = (long long)nely * nq;
    const long long total = (long long)nqz * Ny * w * Nx * w;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int kx = (int)(e % w);
        long long t = e / w;
        const int ix = (int)(t % Nx);
        t /= Nx;
        const int ky = (int)(t % w);
        t /= w;
        const int iy = (int)(t % Ny);
        const int lz = (int)(t / Ny);
        const int jy = iy + ky - p;
        double sum = 0.0;
        if (jy >= 0 && jy < Ny) {
            const int ga = iy + 1, gb = jy + 1;
            int e0, e1;
            span_overlap(ga, gb, p, nely, 0, nely - 1, &e0, &e1);
            for (int ey = e0; ey <= e1; ++ey) {
                const double hy = 0.5 * (bry[ey + 1] - bry[ey]);
                for (int q = 0; q < nq; ++q) {
                    const long long iq = (long long)ey * nq + q;
                    const double wy = gw[q] * hy * By[iq * (p + 1) + (ga - ey)] * By[iq * (p + 1) + (gb - ey)];
                    sum += wy * A1[(((long long)lz * NQy + iq) * Nx + ix) * w + kx];
                }
            }
        }
        A2[e] = sum;
    }
}

// V3h[h][row] += sum over the slab's z quadrature (spans es0..es1) of
// w N_iz N_(iz+dz) A2, for rows with iz in iz0..iz1 and every stored offset
// h.  The slabs are added in order, so the result does not depend on the
// launch configuration.
__global__ void v3_z_kernel(int Nx, int Ny, int Nz, int p, int nq, int nelz, int es0, int es1, int iz0, int iz1,
                            const double* __restrict__ brz, const double* __restrict__ gw,
                            const double* __restrict__ Bz, const double* __restrict__ A2,
                            double* __restrict__ V3h, long long vstride) {
    const int w = 2 * p + 1;
    const int lc = (w * w * w - 1) / 2;
    const int nh = half3_count(p);
    const long long plane = (long long)Nx * Ny;
    const long long nrow = (long long)(iz1 - iz0 + 1) * plane;
    const long long total = nrow * nh;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int h = (int)(e / nrow);
        const long long row = (long long)iz0 * plane + e % nrow;
        const int iz = (int)(row / plane);
        const int iy = (int)((row / Nx) % Ny);
        const int ix = (int)(row % Nx);
        const int l = h + lc;
        const int kx = l % w, ky = (l / w) % w, kz = l / (w * w);
        const int jz = iz + kz - p, jy = iy + ky - p, jx = ix + kx - p;
        if (jz < 0 || jz >= Nz || jy < 0 || jy >= Ny || jx < 0 || jx >= Nx) continue;
        int e0, e1;
        span_overlap(iz + 1, jz + 1, p, nelz, es0, es1, &e0, &e1);
        double sum = 0.0;
        for (int ez = e0; ez <= e1; ++ez) {
            const double hz = 0.5 * (brz[ez + 1] - brz[ez]);
            for (int q = 0; q < nq; ++q) {
                const long long iq = (long long)ez * nq + q;
                const double wz = gw[q] * hz * Bz[iq * (p + 1) + (iz + 1 - ez)] * Bz[iq * (p + 1) + (jz + 1 - ez)];
                const long long lz = iq - (long long)es0 * nq;
                sum += wz * A2[((((lz * Ny + iy) * w + ky) * Nx + ix) * w) + kx];
            }
        }
        V3h[(long long)h * vstride + row] += sum;
    }
}

// ------------------------------------------------------------------ operator
// Tile of outputs: a tile row is one 128-byte line of a plane (16 FP64 or
// 32 FP32 values), 256 outputs per tile.
template <typename FT>
struct Tile3 {
    static constexpr int TX = 128 / (int)sizeof(FT);
    static constexpr int TY = 4;
    static constexpr int TZ = 256 / (TX * TY);
};
template <typename FT>
struct Cplx2;
template <>
struct Cplx2<double> {
    typedef double2 type;
};
template <>
struct Cplx2<float> {
    typedef float2 type;
};
template <typename FT>
dim3 stencil3_grid(int Nx, int Ny, int Nz) {
    return dim3((Nx + Tile3<FT>::TX - 1) / Tile3<FT>::TX, (Ny + Tile3<FT>::TY - 1) / Tile3<FT>::TY,
                (Nz + Tile3<FT>::TZ - 1) / Tile3<FT>::TZ);
}
// Tiles are launched on a 1D grid of 8 ceil(tiles / 8) workgroups.
// Workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8), so
// tile = (b mod 8) ceil(tiles / 8) + b / 8 gives each XCD a contiguous run of
// tiles, i.e. a slab of z planes: the halo of the input, and the mirrored
// potential rows of the offsets below the centre, are then mostly in that
// XCD's own L2.
inline unsigned stencil3_launch(dim3 tiles) {
    const unsigned nb = tiles.x * tiles.y * tiles.z;
    return 8 * ((nb + 7) / 8);
}

// out = w y + a S3 c + b (T3 + V3 + Ebar D3) c (planar complex; y may be
// null) for one tile, the input tile with its p-wide halo in LDS.  One pass
// over the (2p+1)^3 neighbours reads each neighbour once: along every
// (dz, dy) line the x sums Sx c, (Tx + Ebar Dx) c (and Dx c for the
// observables) are formed and weighted with the y and z factors, and the
// neighbour's potential coefficient is taken from this row's plane (stored
// offsets) or from the mirrored row's plane (the others).  OBS: per-block
// partial sums of Re c^H S3 c and Re c^H D3 c (FP64).
template <int PP, typename FT, bool OBS>
__global__ __launch_bounds__(256, 2) void apply3_kernel(
    int Nx, int Ny, int Nz, dim3 tiles, const FT* __restrict__ Sxb, const FT* __restrict__ Txb, const FT* __restrict__ Dxb,
    const FT* __restrict__ Syb, const FT* __restrict__ Tyb, const FT* __restrict__ Szb, const FT* __restrict__ Tzb,
    const FT* __restrict__ V3h, long long vstride, const FT* __restrict__ cre, const FT* __restrict__ cim,
    const FT* __restrict__ yre, const FT* __restrict__ yim, FT wre, FT wim, FT are, FT aim, FT bre, FT bim, FT Ebar,
    FT* __restrict__ ore, FT* __restrict__ oim, double* __restrict__ obs, const double* __restrict__ flag,
    double* __restrict__ dotp) {
    if (flag && *flag != 0.0) return;  // the solve has converged
    constexpr int TX = Tile3<FT>::TX, TY = Tile3<FT>::TY, TZ = Tile3<FT>::TZ;
    constexpr int K = 2 * PP + 1;
    constexpr int WX = TX + 2 * PP, WY = TY + 2 * PP, WZ = TZ + 2 * PP;
    constexpr int LC = (K * K * K - 1) / 2;
    typedef typename Cplx2<FT>::type C2;
    __shared__ C2 tc[WZ][WY][WX];  // the input tile, (re, im) pairs
    const int nb = (int)(tiles.x * tiles.y * tiles.z);
    const int tile = (int)(blockIdx.x % 8) * ((nb + 7) / 8) + (int)(blockIdx.x / 8);
    if (tile >= nb) return;  // padding of the launch to a multiple of 8
    const int bx = tile % (int)tiles.x, by = (tile / (int)tiles.x) % (int)tiles.y,
              bz = tile / (int)(tiles.x * tiles.y);
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int ix = x0 + tx, iy = y0 + ty, iz = z0 + tz;
    const long long plane = (long long)Nx * Ny;
    for (int t = threadIdx.x; t < WX * WY * WZ; t += 256) {
        const int lz = t / (WX * WY), ly = (t / WX) % WY, lx = t % WX;
        const int gz = z0 + lz - PP, gy = y0 + ly - PP, gx = x0 + lx - PP;
        FT vr = 0, vi = 0;
        if (gz >= 0 && gz < Nz && gy >= 0 && gy < Ny && gx >= 0 && gx < Nx) {
            const long long at = ((long long)gz * Ny + gy) * Nx + gx;
            vr = cre[at];
            vi = cim[at];
        }
        tc[lz][ly][lx] = C2{vr, vi};
    }
    const int ixc = ix < Nx ? ix : Nx - 1, iyc = iy < Ny ? iy : Ny - 1, izc = iz < Nz ? iz : Nz - 1;
    const long long row = ((long long)izc * Ny + iyc) * Nx + ixc;
    const unsigned urow = (unsigned)row;  // N < 2^31
    // x factors of the thread's column; y and z factors of the tile's rows
    // and planes in LDS (read once per line instead of a global load)
    __shared__ FT fy[2][TY][K], fz[2][TZ][K];
    if (threadIdx.x < TY * K) {
        const int r = threadIdx.x / K, k = threadIdx.x % K;
        const int gy = y0 + r < Ny ? y0 + r : Ny - 1;
        fy[0][r][k] = band_at(Syb, PP, Ny, gy, gy + k - PP);
        fy[1][r][k] = band_at(Tyb, PP, Ny, gy, gy + k - PP);
    } else if (threadIdx.x >= 64 && threadIdx.x < 64 + TZ * K) {
        const int r = (threadIdx.x - 64) / K, k = (threadIdx.x - 64) % K;
        const int gz = z0 + r < Nz ? z0 + r : Nz - 1;
        fz[0][r][k] = band_at(Szb, PP, Nz, gz, gz + k - PP);
        fz[1][r][k] = band_at(Tzb, PP, Nz, gz, gz + k - PP);
    }
    FT sx[K], hx[K], dxv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int jx = ixc + k - PP;
        sx[k] = band_at(Sxb, PP, Nx, ixc, jx);
        dxv[k] = band_at(Dxb, PP, Nx, ixc, jx);
        hx[k] = band_at(Txb, PP, Nx, ixc, jx) + Ebar * dxv[k];
    }
    __syncthreads();
    constexpr int CL = (K * K - 1) / 2;  // the line (dz, dy) = (0, 0)
    // (global address space: plain loads rather than flat ones, whose
    // completion the LDS waits would also wait for)
    typedef const __attribute__((address_space(1))) FT* gptr;
    FT Sr = 0, Si = 0, Hr = 0, Hi = 0, Dr = 0, Di = 0, Vr = 0, Vi = 0;
    // One (dz, dy) line of x sums, weighted by its y and z factors.
    auto line_sums = [&](int kz, int ky, FT usr, FT usi, FT uhr, FT uhi, FT udr, FT udi) {
        const FT sz = fz[0][tz][kz], tzv = fz[1][tz][kz];
        const FT sy = fy[0][ty][ky], tyv = fy[1][ty][ky];
        const FT szy = sz * sy, hzy = sz * tyv + tzv * sy;
        Sr += szy * usr;
        Si += szy * usi;
        Hr += szy * uhr + hzy * usr;
        Hi += szy * uhi + hzy * usi;
        if constexpr (OBS) {
            Dr += szy * udr;
            Di += szy * udi;
        }
    };
    // Lines after the centre line, each with its mirror line: the stored
    // offset d = (dz, dy, dx) of a line gives this row's V3[i][i+d] from row
    // i of plane d, and V3[i][i-d] = V3[i-d][i] from row i-d of the same
    // plane, read in the same step (row i-d is mostly another row of this
    // tile, or of a neighbouring tile working at the same time, so the
    // second read is served by the cache).  Rows i-d off the grid stay
    // inside the plane's margins and meet a zero input.
#pragma unroll 1
    for (int li = CL + 1; li < K * K; ++li) {
        const int kz = li / K, ky = li % K;        // direct line
        const int mz = K - 1 - kz, my = K - 1 - ky;  // its mirror
        const long long fline = ((long long)(kz - PP) * Ny + (ky - PP)) * Nx;
        const FT* __restrict__ p0 = V3h + (long long)(li * K - LC) * vstride;
        FT a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;  // direct line: S, H, D sums
        FT b0 = 0, b1 = 0, b2 = 0, b3 = 0, b4 = 0, b5 = 0;  // mirror line
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
            const gptr pd = (gptr)(p0 + (long long)kx * vstride);
            const gptr pm = (gptr)(p0 + (long long)kx * vstride - fline - (kx - PP));
            const FT vd = pd[urow], vm = pm[urow];
            const C2 zd = tc[tz + kz][ty + ky][tx + kx];
            const C2 zm = tc[tz + mz][ty + my][tx + K - 1 - kx];
            Vr += vd * zd.x + vm * zm.x;
            Vi += vd * zd.y + vm * zm.y;
            a0 += sx[kx] * zd.x;
            a1 += sx[kx] * zd.y;
            a2 += hx[kx] * zd.x;
            a3 += hx[kx] * zd.y;
            b0 += sx[K - 1 - kx] * zm.x;
            b1 += sx[K - 1 - kx] * zm.y;
            b2 += hx[K - 1 - kx] * zm.x;
            b3 += hx[K - 1 - kx] * zm.y;
            if constexpr (OBS) {
                a4 += dxv[kx] * zd.x;
                a5 += dxv[kx] * zd.y;
                b4 += dxv[K - 1 - kx] * zm.x;
                b5 += dxv[K - 1 - kx] * zm.y;
            }
        }
        line_sums(kz, ky, a0, a1, a2, a3, a4, a5);
        line_sums(mz, my, b0, b1, b2, b3, b4, b5);
    }
    {
        // the centre line: the diagonal, and dx > 0 with its mirror -dx
        FT a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
        const FT* __restrict__ p0 = V3h;
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
            const C2 z = tc[tz + PP][ty + PP][tx + kx];
            a0 += sx[kx] * z.x;
            a1 += sx[kx] * z.y;
            a2 += hx[kx] * z.x;
            a3 += hx[kx] * z.y;
            if constexpr (OBS) {
                a4 += dxv[kx] * z.x;
                a5 += dxv[kx] * z.y;
            }
        }
        const FT v0 = ((gptr)p0)[urow];
        const C2 z0 = tc[tz + PP][ty + PP][tx + PP];
        Vr += v0 * z0.x;
        Vi += v0 * z0.y;
#pragma unroll
        for (int e = 1; e <= PP; ++e) {
            const gptr pd = (gptr)(p0 + (long long)e * vstride);
            const FT vd = pd[urow], vm = (pd - e)[urow];
            const C2 zd = tc[tz + PP][ty + PP][tx + PP + e], zm = tc[tz + PP][ty + PP][tx + PP - e];
            Vr += vd * zd.x + vm * zm.x;
            Vi += vd * zd.y + vm * zm.y;
        }
        line_sums(PP, PP, a0, a1, a2, a3, a4, a5);
    }
    double nu = 0.0, dip = 0.0;
    if (ix < Nx && iy < Ny && iz < Nz) {
        const FT gr = Hr + Vr, gi = Hi + Vi;
        FT accr = are * Sr - aim * Si + bre * gr - bim * gi;
        FT acci = are * Si + aim * Sr + bre * gi + bim * gr;
        if (yre) {
            const FT yr = yre[row], yi = yim[row];
            accr += wre * yr - wim * yi;
            acci += wre * yi + wim * yr;
        }
        ore[row] = accr;
        oim[row] = acci;
        const C2 c0 = tc[tz + PP][ty + PP][tx + PP];
        const double c0r = c0.x, c0i = c0.y;
        if constexpr (OBS) {
            nu = c0r * (double)Sr + c0i * (double)Si;
            dip = c0r * (double)Dr + c0i * (double)Di;
        } else if (dotp) {
            // c^T (A c), unconjugated (the Krylov step's p^T q)
            nu = c0r * (double)accr - c0i * (double)acci;
            dip = c0r * (double)acci + c0i * (double)accr;
        }
    }
    double* const red_out = OBS ? obs : dotp;
    if (red_out) {
        __shared__ double red[2][256];
        red[0][threadIdx.x] = nu;
        red[1][threadIdx.x] = dip;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                red[0][threadIdx.x] += red[0][threadIdx.x + s];
                red[1][threadIdx.x] += red[1][threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            red_out[2 * tile] = red[0][0];
            red_out[2 * tile + 1] = red[1][0];
        }
    }
}

}  // namespace
}  // namespace tdsez

using namespace tdsez;

struct tdsez_system3d_s {
    SystemData ax, ay, az;     // per-axis 1D matrices (V = 0, m = 1)
    int Nx = 0, Ny = 0, Nz = 0, p = 0, order = 0, nq = 0;
    double* d_V3h = nullptr;   // half stencil, [offset][margin + row + margin]
    long long v3_margin = 0;   // p (Ny Nx + Nx + 1): the largest row offset of a neighbour
    long long v3_stride = 0;   // N + 2 margin
    double* d_Qx = nullptr;    // per-axis generalised eigenvectors (column-major)
    double* d_Qy = nullptr;
    double* d_Qz = nullptr;
    double* d_lx = nullptr;    // and eigenvalues
    double* d_my = nullptr;
    double* d_nz = nullptr;
    double* d_work = nullptr;  // kNumVec64 planar FP64 vectors
    double* d_part = nullptr;
    double* d_obs_part = nullptr;
    double* d_dpart = nullptr;  // partial sums of the dot products fused into the operator and preconditioner
    double* d_sc = nullptr;
    int* d_status = nullptr;
    // FP32 copies for TDSEZ_FP32_REFINED, made by the first such call
    float* d_V3h32 = nullptr;
    float* d_bands32 = nullptr;  // Sx, Tx, Dx, Sy, Ty, Sz, Tz
    float* d_Qx32 = nullptr;
    float* d_Qy32 = nullptr;
    float* d_Qz32 = nullptr;
    float* d_work32 = nullptr;
    rocblas_handle blas = nullptr;
    CnStats stats;
};

namespace {

void free_axis(SystemData& a) {
    for (int m = 0; m < 6; ++m) (void)hipFree(a.d_band[m]);
    (void)hipFree(a.d_H0);
    (void)hipFree(a.d_K);
}

void free3d(tdsez_system3d_s* s) {
    free_axis(s->ax);
    free_axis(s->ay);
    free_axis(s->az);
    void* ptrs[] = {s->d_V3h, s->d_Qx, s->d_Qy, s->d_Qz, s->d_lx, s->d_my, s->d_nz, s->d_work, s->d_part,
                    s->d_obs_part, s->d_dpart, s->d_sc, s->d_status, s->d_V3h32, s->d_bands32, s->d_Qx32, s->d_Qy32,
                    s->d_Qz32, s->d_work32};
    for (void* q : ptrs) (void)hipFree(q);
    if (s->blas) rocblas_destroy_handle(s->blas);
}

// FP32 copies of the operator and preconditioner data (first
// TDSEZ_FP32_REFINED call; synchronous)
tdsez_status ensure_fp32_3d(tdsez_system3d_s* s) {
    if (s->d_work32) return TDSEZ_OK;
    const int Nx = s->Nx, Ny = s->Ny, Nz = s->Nz, p = s->p;
    const long long n = (long long)Nx * Ny * Nz;
    const long long nv = (long long)half3_count(p) * s->v3_stride;
    const long long bx = (long long)Nx * (p + 1), by = (long long)Ny * (p + 1), bz = (long long)Nz * (p + 1);
    float *v3 = nullptr, *bands = nullptr, *qx = nullptr, *qy = nullptr, *qz = nullptr, *work = nullptr;
    hipError_t he = hipSuccess;
    auto H = [&](hipError_t e) { if (he == hipSuccess) he = e; };
    H(hipMalloc(&v3, sizeof(float) * nv));
    H(hipMalloc(&bands, sizeof(float) * (3 * bx + 2 * by + 2 * bz)));
    H(hipMalloc(&qx, sizeof(float) * (size_t)Nx * Nx));
    H(hipMalloc(&qy, sizeof(float) * (size_t)Ny * Ny));
    H(hipMalloc(&qz, sizeof(float) * (size_t)Nz * Nz));
    H(hipMalloc(&work, sizeof(float) * (size_t)n * 2 * kNumVec32));
    if (he != hipSuccess) {
        (void)hipFree(v3); (void)hipFree(bands); (void)hipFree(qx); (void)hipFree(qy); (void)hipFree(qz);
        (void)hipFree(work);
        return fail(TDSEZ_ENOMEM, "3D FP32 workspace allocation failed");
    }
    to_fp32_kernel<<<grid_for(nv), 256>>>(nv, s->d_V3h, v3);
    float* o = bands;
    const double* src[7] = {s->ax.d_band[0], s->ax.d_band[1], s->ax.d_band[3], s->ay.d_band[0],
                            s->ay.d_band[1], s->az.d_band[0], s->az.d_band[1]};
    const long long len[7] = {bx, bx, bx, by, by, bz, bz};
    for (int k = 0; k < 7; ++k) {
        to_fp32_kernel<<<grid_for(len[k]), 256>>>(len[k], src[k], o);
        o += len[k];
    }
    to_fp32_kernel<<<grid_for((long long)Nx * Nx), 256>>>((long long)Nx * Nx, s->d_Qx, qx);
    to_fp32_kernel<<<grid_for((long long)Ny * Ny), 256>>>((long long)Ny * Ny, s->d_Qy, qy);
    to_fp32_kernel<<<grid_for((long long)Nz * Nz), 256>>>((long long)Nz * Nz, s->d_Qz, qz);
    H(hipGetLastError());
    H(hipDeviceSynchronize());
    s->d_V3h32 = v3;
    s->d_bands32 = bands;
    s->d_Qx32 = qx;
    s->d_Qy32 = qy;
    s->d_Qz32 = qz;
    s->d_work32 = work;
    if (he != hipSuccess) return fail(TDSEZ_EHIP, "3D FP32 copies: %s", hipGetErrorString(he));
    return TDSEZ_OK;
}

// The 3D operator and preconditioner for the shared step loop.
struct Op3D {
    tdsez_system3d_s* s;
    const CnWork& cw;
    double alpha;
    // the preconditioner inverts S3 + i alpha T3 (Crank-Nicolson), or
    // T3 - shift S3 when `shifted` (inverse iteration)
    bool shifted = false;
    double shift = 0.0;
    int nblk_apply(bool fp32) const {
        const dim3 t = fp32 ? stencil3_grid<float>(s->Nx, s->Ny, s->Nz) : stencil3_grid<double>(s->Nx, s->Ny, s->Nz);
        return (int)(t.x * t.y * t.z);
    }
    int nblk_precond() const {
        // the last contraction: x, over the rows of all planes
        return ((s->Nx + kGemmTile - 1) / kGemmTile) * ((s->Nz * s->Ny + kGemmTile - 1) / kGemmTile);
    }
    // no force stencil in 3D (the acceleration is not offered there)
    int accel(int, double*, hipStream_t) { return 0; }
    template <typename FT>
    void apply_t(const FT* const* b, const FT* V3pad, const FT* cr, const FT* ci, const FT* yr, const FT* yi, double wr,
                 double wi, double ar, double ai, double br, double bi, double Eb, FT* outr, FT* outi, double* obsp,
                 const double* flag, hipStream_t stream, double* dotp = nullptr) {
        const int Nx = s->Nx, Ny = s->Ny, Nz = s->Nz;
        const dim3 tiles = stencil3_grid<FT>(Nx, Ny, Nz);
        const unsigned grid = stencil3_launch(tiles);
        const bool ob = obsp != nullptr;
        switch (s->p * 2 + (ob ? 1 : 0)) {
#define TD3_CASE(PV_, OB_)                                                                                       \
    case PV_ * 2 + OB_:                                                                                          \
        apply3_kernel<PV_, FT, OB_><<<grid, 256, 0, stream>>>(Nx, Ny, Nz, tiles, b[0], b[1], b[2], b[3], b[4], b[5], \
                                                                b[6], V3pad + s->v3_margin, s->v3_stride, cr, ci, yr, yi, (FT)wr, (FT)wi, (FT)ar, \
                                                                (FT)ai, (FT)br, (FT)bi, (FT)Eb, outr, outi, obsp, \
                                                                flag, dotp);                                     \
        break;
            TD3_CASE(1, 0) TD3_CASE(1, 1) TD3_CASE(2, 0) TD3_CASE(2, 1) TD3_CASE(3, 0) TD3_CASE(3, 1)
            TD3_CASE(4, 0) TD3_CASE(4, 1)
#undef TD3_CASE
            default: break;
        }
    }
    void apply(int in, int yv, double wr, double wi, double ar, double ai, double br, double bi, double Eb, int outv,
               double* obsp, const double* flag, hipStream_t stream, double* dotp = nullptr) {
        const double* b[7] = {s->ax.d_band[0], s->ax.d_band[1], s->ax.d_band[3], s->ay.d_band[0],
                              s->ay.d_band[1], s->az.d_band[0], s->az.d_band[1]};
        apply_t<double>(b, s->d_V3h, cw.re(in), cw.im(in), yv >= 0 ? cw.re(yv) : nullptr,
                        yv >= 0 ? cw.im(yv) : nullptr, wr, wi, ar, ai, br, bi, Eb, cw.re(outv), cw.im(outv), obsp,
                        flag, stream, dotp);
    }
    void apply32(int in, double ar, double ai, double br, double bi, double Eb, int outv, const double* flag,
                 hipStream_t stream, double* dotp = nullptr) {
        const int p = s->p;
        const long long bx = (long long)s->Nx * (p + 1), by = (long long)s->Ny * (p + 1);
        const float* f = s->d_bands32;
        const float* b[7] = {f, f + bx, f + 2 * bx, f + 3 * bx, f + 3 * bx + by, f + 3 * bx + 2 * by,
                             f + 3 * bx + 2 * by + (long long)s->Nz * (p + 1)};
        apply_t<float>(b, s->d_V3h32, cw.re32(in), cw.im32(in), nullptr, nullptr, 0.0, 0.0, ar, ai, br, bi, Eb,
                       cw.re32(outv), cw.im32(outv), nullptr, flag, stream, dotp);
    }
    // z = P^-1 r, the planes of r as (Nz Ny) x Nx, per-plane Ny x Nx and
    // Nz x (Ny Nx) row-major matrices for the x, y and z contractions
    template <typename FT>
    void precond_t(const FT* Qx, const FT* Qy, const FT* Qz, const FT* rr, const FT* ri, FT* ar_, FT* ai_, FT* br_,
                   FT* bi_, FT* zr, FT* zi, const double* flag, hipStream_t stream, double* rzp) {
        const int Nx = s->Nx, Ny = s->Ny, Nz = s->Nz;
        const long long pl = (long long)Nx * Ny;
        const int T = kGemmTile;
        const FdmScale none{0, 0, 0, 0, nullptr, nullptr, nullptr, 1};
        const FdmScale cn = shifted ? FdmScale{-shift, 0.0, 1.0, 0.0, s->d_nz, s->d_lx, s->d_my, Nx}
                                    : FdmScale{1.0, 0.0, 0.0, alpha, s->d_nz, s->d_lx, s->d_my, Nx};
        const dim3 gx((Nx + T - 1) / T, (Nz * Ny + T - 1) / T, 1);
        const dim3 gy((Nx + T - 1) / T, (Ny + T - 1) / T, Nz);
        const dim3 gz((unsigned)((pl + T - 1) / T), (Nz + T - 1) / T, 1);
        // forward: x, y (per z plane), z with the scaling
        fdm_gemm_kernel<FT, false, false><<<gx, kGemmThreads, 0, stream>>>(Nz * Ny, Nx, Nx, Qx, 1, Nx, rr, ri, ar_,
                                                                           ai_, 0, 0, none, flag);
        fdm_gemm_kernel<FT, true, false><<<gy, kGemmThreads, 0, stream>>>(Ny, Nx, Ny, Qy, Ny, 1, ar_, ai_, br_, bi_, pl,
                                                                          pl, none, flag);
        fdm_gemm_kernel<FT, true, true><<<gz, kGemmThreads, 0, stream>>>(Nz, (int)pl, Nz, Qz, Nz, 1, br_, bi_, ar_,
                                                                         ai_, 0, 0, cn, flag);
        // back: z, y, x
        fdm_gemm_kernel<FT, true, false><<<gz, kGemmThreads, 0, stream>>>(Nz, (int)pl, Nz, Qz, 1, Nz, ar_, ai_, br_,
                                                                          bi_, 0, 0, none, flag);
        fdm_gemm_kernel<FT, true, false><<<gy, kGemmThreads, 0, stream>>>(Ny, Nx, Ny, Qy, 1, Ny, br_, bi_, ar_, ai_, pl,
                                                                          pl, none, flag);
        if (rzp)
            fdm_gemm_kernel<FT, false, false, true><<<gx, kGemmThreads, 0, stream>>>(
                Nz * Ny, Nx, Nx, Qx, Nx, 1, ar_, ai_, zr, zi, 0, 0, none, flag, rr, ri, rzp);
        else
            fdm_gemm_kernel<FT, false, false><<<gx, kGemmThreads, 0, stream>>>(Nz * Ny, Nx, Nx, Qx, Nx, 1, ar_, ai_, zr,
                                                                               zi, 0, 0, none, flag);
    }
    void precond(int rin, int zout, const double* flag, hipStream_t stream, double* rzp = nullptr) {
        precond_t<double>(s->d_Qx, s->d_Qy, s->d_Qz, cw.re(rin), cw.im(rin), cw.re(kT1), cw.im(kT1), cw.re(kT2),
                          cw.im(kT2), cw.re(zout), cw.im(zout), flag, stream, rzp);
    }
    void precond32(int rin, int zout, const double* flag, hipStream_t stream, double* rzp = nullptr) {
        precond_t<float>(s->d_Qx32, s->d_Qy32, s->d_Qz32, cw.re32(rin), cw.im32(rin), cw.re32(kT132),
                         cw.im32(kT132), cw.re32(kT232), cw.im32(kT232), cw.re32(zout), cw.im32(zout), flag, stream,
                         rzp);
    }
};

// Basis values of one axis at its quadrature points (device), and the
// breakpoints on the device.
tdsez_status axis_basis(const double* br, int nb, int p, int nq, const double* gx, double** d_br, double** d_B) {
    const long long nqa = (long long)(nb - 1) * nq;
    std::vector<double> xq(nqa);
    for (int e = 0; e + 1 < nb; ++e)
        for (int q = 0; q < nq; ++q)
            xq[(size_t)e * nq + q] = 0.5 * (br[e + 1] + br[e]) + 0.5 * (br[e + 1] - br[e]) * gx[q];
    double *dxq = nullptr, *ddB = nullptr;
    hipError_t he = hipSuccess;
    auto H = [&](hipError_t e) { if (he == hipSuccess) he = e; };
    H(hipMalloc(d_br, sizeof(double) * nb));
    H(hipMalloc(d_B, sizeof(double) * nqa * (p + 1)));
    H(hipMalloc(&dxq, sizeof(double) * nqa));
    H(hipMalloc(&ddB, sizeof(double) * nqa * (p + 1)));
    if (he == hipSuccess) {
        H(hipMemcpy(*d_br, br, sizeof(double) * nb, hipMemcpyHostToDevice));
        H(hipMemcpy(dxq, xq.data(), sizeof(double) * nqa, hipMemcpyHostToDevice));
    }
    if (he == hipSuccess) {
        basis_kernel<<<grid_for(nqa), 256>>>(*d_br, nb, p, nq, dxq, *d_B, ddB);
        H(hipGetLastError());
        H(hipDeviceSynchronize());
    }
    (void)hipFree(dxq);
    (void)hipFree(ddB);
    if (he != hipSuccess) return fail(TDSEZ_EHIP, "3D basis values: %s", hipGetErrorString(he));
    return TDSEZ_OK;
}

}  // namespace

extern "C" {

tdsez_status tdsez_assemble_3d(const double* breaks_x, int nbx, const double* breaks_y, int nby,
                               const double* breaks_z, int nbz, int order, int nq, const double* V_q,
                               tdsez_system3d* out) {
    if (!out) return fail(TDSEZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (!breaks_x || !breaks_y || !breaks_z || !V_q) return fail(TDSEZ_EINVAL, "NULL argument");
    if (order < 2) return fail(TDSEZ_EINVAL, "order must be >= 2");
    if (order - 1 > 4) return fail(TDSEZ_EUNSUPPORTED, "3D: order %d > 5", order);
    if (nq < 1 || nq > 32) return fail(TDSEZ_EINVAL, "nq must be in 1..32");
    const double* brs[3] = {breaks_x, breaks_y, breaks_z};
    const int nbs[3] = {nbx, nby, nbz};
    for (int a = 0; a < 3; ++a) {
        if (nbs[a] < 2) return fail(TDSEZ_EINVAL, "need at least 2 breakpoints per axis");
        for (int i = 0; i + 1 < nbs[a]; ++i)
            if (!(brs[a][i + 1] > brs[a][i]) || !std::isfinite(brs[a][i]) || !std::isfinite(brs[a][i + 1]))
                return fail(TDSEZ_EINVAL, "breakpoints must be finite and strictly increasing");
    }
    const int p = order - 1;
    const int Nx = nbx - 1 + p - 2, Ny = nby - 1 + p - 2, Nz = nbz - 1 + p - 2;
    if (Nx < 2 * p + 1 || Ny < 2 * p + 1 || Nz < 2 * p + 1)
        return fail(TDSEZ_EINVAL, "need at least 2p+1 unknowns per axis");
    const long long nqx = (long long)(nbx - 1) * nq, nqy = (long long)(nby - 1) * nq, nqz = (long long)(nbz - 1) * nq;
    const long long nV = nqx * nqy * nqz;
    for (long long i = 0; i < nV; ++i)
        if (!std::isfinite(V_q[i])) return fail(TDSEZ_EINVAL, "V_q[%lld] is not finite", i);
    auto* s = new tdsez_system3d_s();
    s->Nx = Nx;
    s->Ny = Ny;
    s->Nz = Nz;
    s->p = p;
    s->order = order;
    s->nq = nq;
    auto bail = [&](tdsez_status st) {
        free3d(s);
        delete s;
        return st;
    };
    tdsez_status st = assemble_device(breaks_x, nbx, order, nq, nullptr, nullptr, nullptr, &s->ax);
    if (!st) st = assemble_device(breaks_y, nby, order, nq, nullptr, nullptr, nullptr, &s->ay);
    if (!st) st = assemble_device(breaks_z, nbz, order, nq, nullptr, nullptr, nullptr, &s->az);
    if (st) return bail(st);
    if (rocblas_create_handle(&s->blas) != rocblas_status_success)
        return bail(fail(TDSEZ_EHIP, "rocblas_create_handle failed"));
    const long long n = (long long)Nx * Ny * Nz;
    const int w = 2 * p + 1;
    {
        double gx[32], gw[32];
        gauss_legendre_host(nq, gx, gw);
        double *dbx = nullptr, *dby = nullptr, *dbz = nullptr, *dBx = nullptr, *dBy = nullptr, *dBz = nullptr;
        double *dgw = nullptr, *dVq = nullptr, *dA1 = nullptr, *dA2 = nullptr;
        auto clean = [&]() {
            void* ptrs[] = {dbx, dby, dbz, dBx, dBy, dBz, dgw, dVq, dA1, dA2};
            for (void* q : ptrs) (void)hipFree(q);
        };
        st = axis_basis(breaks_x, nbx, p, nq, gx, &dbx, &dBx);
        if (!st) st = axis_basis(breaks_y, nby, p, nq, gx, &dby, &dBy);
        if (!st) st = axis_basis(breaks_z, nbz, p, nq, gx, &dbz, &dBz);
        if (st) {
            clean();
            return bail(st);
        }
        // z slabs: as many z spans as keep A2 near 64 M entries
        const long long per_qz = (long long)Ny * w * Nx * w;
        int slab = (int)std::max<long long>(1, (64ll << 20) / (per_qz * nq));
        slab = std::min(slab, nbz - 1);
        hipError_t he = hipSuccess;
        auto H = [&](hipError_t e) { if (he == hipSuccess) he = e; };
        H(hipMalloc(&dgw, sizeof(double) * nq));
        H(hipMalloc(&dVq, sizeof(double) * nV));
        H(hipMalloc(&dA1, sizeof(double) * (size_t)slab * nq * nqy * Nx * w));
        H(hipMalloc(&dA2, sizeof(double) * (size_t)slab * nq * per_qz));
        s->v3_margin = (long long)p * ((long long)Ny * Nx + Nx + 1);
        s->v3_stride = n + 2 * s->v3_margin;
        const long long nv3 = (long long)half3_count(p) * s->v3_stride;
        H(hipMalloc(&s->d_V3h, sizeof(double) * (size_t)nv3));
        if (he == hipSuccess) {
            H(hipMemcpy(dgw, gw, sizeof(double) * nq, hipMemcpyHostToDevice));
            H(hipMemcpy(dVq, V_q, sizeof(double) * nV, hipMemcpyHostToDevice));
        }
        if (he == hipSuccess) {
            copy_kernel<double><<<grid_for(nv3), 256>>>(nv3, nullptr, s->d_V3h, nullptr);
            const int nelz = nbz - 1;
            for (int es0 = 0; es0 < nelz && he == hipSuccess; es0 += slab) {
                const int es1 = std::min(es0 + slab, nelz) - 1;
                const int nqs = (es1 - es0 + 1) * nq;
                v3_a1_kernel<<<4096, 256>>>(Nx, p, nq, nbx - 1, (int)nqy, es0 * nq, nqs, dbx, dgw, dBx, dVq, dA1);
                v3_a2_kernel<<<4096, 256>>>(Nx, Ny, p, nq, nby - 1, nqs, dby, dgw, dBy, dA1, dA2);
                // rows whose z B-spline (global index iz + 1, spans iz + 1 - p .. iz + 1)
                // meets the slab
                const int iz0 = std::max(0, es0 - 1), iz1 = std::min(Nz - 1, es1 + p - 1);
                v3_z_kernel<<<4096, 256>>>(Nx, Ny, Nz, p, nq, nelz, es0, es1, iz0, iz1, dbz, dgw, dBz, dA2,
                                           s->d_V3h + s->v3_margin, s->v3_stride);
                H(hipGetLastError());
            }
            H(hipDeviceSynchronize());
        }
        clean();
        if (he != hipSuccess) return bail(fail(TDSEZ_EHIP, "3D assembly: %s", hipGetErrorString(he)));
    }
    st = axis_eigen(s->blas, s->ax, &s->d_Qx, &s->d_lx);
    if (!st) st = axis_eigen(s->blas, s->ay, &s->d_Qy, &s->d_my);
    if (!st) st = axis_eigen(s->blas, s->az, &s->d_Qz, &s->d_nz);
    if (st) return bail(st);
    const dim3 sg = stencil3_grid<double>(Nx, Ny, Nz);
    if (hipMalloc(&s->d_work, sizeof(double) * (size_t)n * 2 * kNumVec64) != hipSuccess ||
        hipMalloc(&s->d_part, sizeof(double) * 2 * kRedBlocks) != hipSuccess ||
        hipMalloc(&s->d_sc, sizeof(double) * 2 * kScBlock) != hipSuccess ||
        hipMalloc(&s->d_status, sizeof(int) * 4) != hipSuccess ||
        hipMalloc(&s->d_obs_part, sizeof(double) * 2 * (size_t)sg.x * sg.y * sg.z) != hipSuccess)
        return bail(fail(TDSEZ_ENOMEM, "3D workspace allocation failed"));
    {
        const dim3 s32 = stencil3_grid<float>(Nx, Ny, Nz);
        const size_t nb = std::max<size_t>({(size_t)sg.x * sg.y * sg.z, (size_t)s32.x * s32.y * s32.z,
                                            (size_t)((Nx + kGemmTile - 1) / kGemmTile) *
                                                ((Nz * Ny + kGemmTile - 1) / kGemmTile)});
        if (hipMalloc(&s->d_dpart, sizeof(double) * 2 * nb) != hipSuccess)
            return bail(fail(TDSEZ_ENOMEM, "3D workspace allocation failed"));
    }
    *out = s;
    return TDSEZ_OK;
}

tdsez_status tdsez_system3d_size(tdsez_system3d s, int* nx, int* ny, int* nz, int* halfbw) {
    if (!s) return fail(TDSEZ_EINVAL, "system is NULL");
    if (nx) *nx = s->Nx;
    if (ny) *ny = s->Ny;
    if (nz) *nz = s->Nz;
    if (halfbw) *halfbw = s->p;
    return TDSEZ_OK;
}

tdsez_status tdsez_get_v3_rows(tdsez_system3d s, const long* rows, int nrows, double* host_out) {
    if (!s || !rows || !host_out) return fail(TDSEZ_EINVAL, "NULL argument");
    if (nrows < 0) return fail(TDSEZ_EINVAL, "nrows < 0");
    const int p = s->p, w = 2 * p + 1, nh = half3_count(p), lc = (w * w * w - 1) / 2;
    const int Nx = s->Nx, Ny = s->Ny, Nz = s->Nz;
    const long long n = (long long)Nx * Ny * Nz;
    for (int r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= n) return fail(TDSEZ_EINVAL, "row %ld outside 0..%lld", rows[r], n - 1);
    // small systems: one copy of the whole half stencil; large ones: the
    // needed entries one by one (meant for a few sampled rows)
    std::vector<double> all;
    const long long M = s->v3_margin, vs = s->v3_stride;
    if ((long long)nh * vs <= (32ll << 20)) {
        all.resize((size_t)nh * vs);
        TDSEZ_HIP_TRY(hipMemcpy(all.data(), s->d_V3h, sizeof(double) * all.size(), hipMemcpyDeviceToHost));
    }
    for (int r = 0; r < nrows; ++r) {
        const long long row = rows[r];
        const int iz = (int)(row / ((long long)Nx * Ny)), iy = (int)((row / Nx) % Ny), ix = (int)(row % Nx);
        for (int l = 0; l < w * w * w; ++l) {
            const int dx = l % w - p, dy = (l / w) % w - p, dz = l / (w * w) - p;
            const int jz = iz + dz, jy = iy + dy, jx = ix + dx;
            double v = 0.0;
            if (jz >= 0 && jz < Nz && jy >= 0 && jy < Ny && jx >= 0 && jx < Nx) {
                const long long at = M + (l >= lc ? (long long)(l - lc) * vs + row
                                                  : (long long)(lc - l) * vs + ((long long)jz * Ny + jy) * Nx + jx);
                if (!all.empty())
                    v = all[(size_t)at];
                else
                    TDSEZ_HIP_TRY(hipMemcpy(&v, s->d_V3h + at, sizeof(double), hipMemcpyDeviceToHost));
            }
            host_out[(size_t)r * w * w * w + l] = v;
        }
    }
    return TDSEZ_OK;
}

tdsez_status tdsez_apply_3d(tdsez_system3d s, const double* c, double* out, double are, double aim, double bre,
                            double bim, double Ebar, void* stream_v) {
    if (!s || !c || !out) return fail(TDSEZ_EINVAL, "NULL argument");
    hipStream_t stream = (hipStream_t)stream_v;
    CnWork cw;
    cw.n = (long long)s->Nx * s->Ny * s->Nz;
    cw.w = s->d_work;
    const int g = grid_for(cw.n);
    to_planar_kernel<<<g, 256, 0, stream>>>(c, cw.n, cw.re(kC), cw.im(kC));
    Op3D op{s, cw, 0.0};
    op.apply(kC, -1, 0.0, 0.0, are, aim, bre, bim, Ebar, kB, nullptr, nullptr, stream);
    from_planar_kernel<<<g, 256, 0, stream>>>(cw.re(kB), cw.im(kB), cw.n, out);
    TDSEZ_HIP_TRY(hipGetLastError());
    return TDSEZ_OK;
}

tdsez_status tdsez_ground_state_3d(tdsez_system3d s, double sigma, double tol, int maxit, double* psi,
                                   double* energy) {
    if (!s || !psi || !energy) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!std::isfinite(sigma) || !(tol > 0.0) || maxit < 1)
        return fail(TDSEZ_EINVAL, "sigma must be finite, tol > 0 and maxit >= 1");
    const int Nx = s->Nx, Ny = s->Ny, Nz = s->Nz;
    CnWork cw;
    cw.n = (long long)Nx * Ny * Nz;
    cw.w = s->d_work;
    const long long n = cw.n;
    const int g = grid_for(n);
    // (H - sigma S) y = S x by preconditioned CG (the pencil is real and
    // H - sigma S positive definite for sigma below the lowest level); the
    // preconditioner is the exact inverse of T3 - sigma S3
    Op3D op{s, cw, 0.0};
    op.shifted = true;
    op.shift = sigma;
    enum { X = kC, Y = kX, R = kR, Z = kZ, P = kP, Q = kQ, B = kB };
    std::vector<double> part(2 * kRedBlocks);
    auto dot = [&](int u, int v, bool abs2) -> double {
        dot_kernel<double><<<kRedBlocks, kRedThreads>>>(n, cw.re(u), cw.im(u), cw.re(v), cw.im(v), abs2, s->d_part,
                                                        nullptr);
        if (hipMemcpy(part.data(), s->d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return std::nan("");
        double acc = 0.0;
        for (int k = 0; k < kRedBlocks; ++k) acc += part[2 * k];
        return acc;
    };
    // start: a smooth positive bump over the grid (nodal index space),
    // S-normalised
    {
        std::vector<double> h((size_t)2 * n, 0.0);
        for (int iz = 0; iz < Nz; ++iz)
            for (int iy = 0; iy < Ny; ++iy)
                for (int ix = 0; ix < Nx; ++ix) {
                    const double u = (ix - 0.5 * (Nx - 1)) / (0.125 * Nx), v = (iy - 0.5 * (Ny - 1)) / (0.125 * Ny),
                                 w = (iz - 0.5 * (Nz - 1)) / (0.125 * Nz);
                    h[((size_t)iz * Ny + iy) * Nx + ix] = std::exp(-(u * u + v * v + w * w));
                }
        TDSEZ_HIP_TRY(hipMemcpy(cw.re(X), h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
    }
    double* sc = s->d_sc;  // scratch scalars for the CG update kernels
    auto set_sc = [&](double a0, double a1, double a2, double a3, double a4, double a5) -> tdsez_status {
        double v[kScBlock] = {};
        v[0] = a0;
        v[1] = a1;
        v[2] = a2;
        v[3] = a3;
        v[4] = a4;
        v[5] = a5;
        TDSEZ_HIP_TRY(hipMemcpy(sc, v, sizeof(v), hipMemcpyHostToDevice));
        return TDSEZ_OK;
    };
    double E = 0.0, Eprev = 0.0, res = 1.0;
    int outer = 0;
    const int kInner = 400;
    for (outer = 0; outer < maxit; ++outer) {
        // B = S x; y = 0; r = B
        op.apply(X, -1, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, B, nullptr, nullptr, nullptr);
        copy_kernel<double><<<g, 256>>>(2 * n, nullptr, cw.re(Y), nullptr);
        copy_kernel<double><<<g, 256>>>(2 * n, cw.re(B), cw.re(R), nullptr);
        const double b2 = dot(B, B, true);
        op.precond(R, Z, nullptr, nullptr);
        copy_kernel<double><<<g, 256>>>(2 * n, cw.re(Z), cw.re(P), nullptr);
        double rho = dot(R, Z, false);
        const double itol = std::max(1e-3 * tol, 1e-15);
        for (int it = 0; it < kInner; ++it) {
            // q = (H - sigma S) p
            op.apply(P, -1, 0.0, 0.0, -sigma, 0.0, 1.0, 0.0, 0.0, Q, nullptr, nullptr, nullptr);
            const double pq = dot(P, Q, false);
            if (!(pq > 0.0)) return fail(TDSEZ_EINVAL, "3D ground state: H - sigma S is not positive definite "
                                                       "(sigma %g is not below the lowest level)", sigma);
            const double al = rho / pq;
            TDSEZ_HIP_TRY(set_sc(0.0, 0.0, al, 0.0, 0.0, 0.0) == TDSEZ_OK ? hipSuccess : hipErrorUnknown);
            cocg_xr_dev_kernel<double><<<g, 256>>>(n, sc, cw.re(P), cw.im(P), cw.re(Q), cw.im(Q), cw.re(Y),
                                                   cw.im(Y), cw.re(R), cw.im(R));
            const double r2 = dot(R, R, true);
            if (r2 <= itol * itol * b2) break;
            op.precond(R, Z, nullptr, nullptr);
            const double rz = dot(R, Z, false);
            const double be = rz / rho;
            rho = rz;
            TDSEZ_HIP_TRY(set_sc(0.0, 0.0, 0.0, 0.0, be, 0.0) == TDSEZ_OK ? hipSuccess : hipErrorUnknown);
            cocg_p_dev_kernel<double><<<g, 256>>>(n, sc, cw.re(Z), cw.im(Z), cw.re(P), cw.im(P));
        }
        // x = y / |y|_S, E = x^T H x
        op.apply(Y, -1, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, B, nullptr, nullptr, nullptr);
        const double ny2 = dot(Y, B, false);
        if (!(ny2 > 0.0) || !std::isfinite(ny2)) return fail(TDSEZ_ENOCONV, "3D ground state: no progress");
        const double inv = 1.0 / std::sqrt(ny2);
        TDSEZ_HIP_TRY(set_sc(0.0, 0.0, 0.0, 0.0, inv, 0.0) == TDSEZ_OK ? hipSuccess : hipErrorUnknown);
        copy_kernel<double><<<g, 256>>>(2 * n, nullptr, cw.re(X), nullptr);
        cocg_p_dev_kernel<double><<<g, 256>>>(n, sc, cw.re(X), cw.im(X), cw.re(Y), cw.im(Y));  // y *= inv
        copy_kernel<double><<<g, 256>>>(2 * n, cw.re(Y), cw.re(X), nullptr);
        op.apply(X, -1, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, Q, nullptr, nullptr, nullptr);  // H x
        op.apply(X, -1, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, B, nullptr, nullptr, nullptr);  // S x
        Eprev = E;
        E = dot(X, Q, false);
        // residual |H x - E S x| / |S x|: r = Hx - E Sx via x += al p, r -= al q
        copy_kernel<double><<<g, 256>>>(2 * n, cw.re(Q), cw.re(R), nullptr);
        TDSEZ_HIP_TRY(set_sc(0.0, 0.0, E, 0.0, 0.0, 0.0) == TDSEZ_OK ? hipSuccess : hipErrorUnknown);
        copy_kernel<double><<<g, 256>>>(2 * n, nullptr, cw.re(Z), nullptr);
        cocg_xr_dev_kernel<double><<<g, 256>>>(n, sc, cw.re(B), cw.im(B), cw.re(B), cw.im(B), cw.re(Z), cw.im(Z),
                                               cw.re(R), cw.im(R));
        res = std::sqrt(dot(R, R, true) / dot(B, B, true));
        if (!std::isfinite(E) || !std::isfinite(res)) return fail(TDSEZ_ENONFINITE, "3D ground state: non-finite");
        if (outer > 0 && std::fabs(E - Eprev) <= tol * std::fabs(E) && res <= std::sqrt(tol)) break;
    }
    TDSEZ_HIP_TRY(hipGetLastError());
    from_planar_kernel<<<g, 256>>>(cw.re(X), cw.im(X), n, psi);
    TDSEZ_HIP_TRY(hipGetLastError());
    TDSEZ_HIP_TRY(hipDeviceSynchronize());
    *energy = E;
    if (outer >= maxit)
        return fail(TDSEZ_ENOCONV, "3D ground state: %d iterations, |dE| %g, residual %g", maxit,
                    std::fabs(E - Eprev), res);
    return TDSEZ_OK;
}

tdsez_status tdsez_time_apply_3d(tdsez_system3d s, tdsez_precision prec, int reps, void* stream_v, double* ms_out) {
    if (!s || !ms_out) return fail(TDSEZ_EINVAL, "NULL argument");
    if (reps < 1) return fail(TDSEZ_EINVAL, "reps must be >= 1");
    if (prec != TDSEZ_FP64 && prec != TDSEZ_FP32_REFINED) return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    const bool mixed = prec == TDSEZ_FP32_REFINED;
    if (mixed) {
        if (tdsez_status st = ensure_fp32_3d(s)) return st;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    CnWork cw;
    cw.n = (long long)s->Nx * s->Ny * s->Nz;
    cw.w = s->d_work;
    cw.w32 = s->d_work32;
    Op3D op{s, cw, 0.0};
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

tdsez_status tdsez_propagate_3d(tdsez_system3d s, double* psi, const double* E, double dt, int nsteps,
                                tdsez_precision prec, unsigned obs, double* obs_out, double tol, int maxit,
                                void* stream_v) {
    if (!s || !psi || !E) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TDSEZ_EINVAL, "dt must be > 0");
    if (nsteps < 0) return fail(TDSEZ_EINVAL, "nsteps < 0");
    if (obs & ~3u) return fail(TDSEZ_EINVAL, "3D observables: TDSEZ_OBS_NORM and TDSEZ_OBS_DIPOLE only");
    if (obs && !obs_out) return fail(TDSEZ_EINVAL, "obs requested but obs_out is NULL");
    if (prec != TDSEZ_FP64 && prec != TDSEZ_FP32_REFINED) return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    if (!(tol > 0.0) || maxit < 1) return fail(TDSEZ_EINVAL, "tol must be > 0 and maxit >= 1");
    const bool mixed = prec == TDSEZ_FP32_REFINED;
    if (mixed) {
        if (tdsez_status st = ensure_fp32_3d(s)) return st;
    }
    CnWork cw;
    cw.n = (long long)s->Nx * s->Ny * s->Nz;
    cw.w = s->d_work;
    cw.w32 = s->d_work32;
    cw.part = s->d_part;
    cw.sc = s->d_sc;
    cw.status = s->d_status;
    cw.obs_part = s->d_obs_part;
    cw.dpart = s->d_dpart;
    const dim3 sg = stencil3_grid<double>(s->Nx, s->Ny, s->Nz);
    cw.nblk_obs = (int)(sg.x * sg.y * sg.z);
    Op3D op{s, cw, 0.5 * dt};
    return cn_cocg_propagate(cw, op, psi, E, dt, nsteps, mixed, obs, obs_out, tol, maxit, (hipStream_t)stream_v,
                             &s->stats, "3D");
}

tdsez_status tdsez_system3d_stats(tdsez_system3d s, long* steps, long* iterations, int* max_iterations,
                                  long* sweeps) {
    if (!s) return fail(TDSEZ_EINVAL, "system is NULL");
    if (steps) *steps = (long)s->stats.steps_total;
    if (iterations) *iterations = (long)s->stats.iters_total;
    if (max_iterations) *max_iterations = s->stats.iters_max;
    if (sweeps) *sweeps = (long)s->stats.sweeps_total;
    s->stats = CnStats();
    return TDSEZ_OK;
}

void tdsez_system3d_destroy(tdsez_system3d s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    free3d(s);
    delete s;
}

}  // extern "C"
