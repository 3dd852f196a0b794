// Ground state and low-lying eigenpairs of H0 c = e S c (the paper's section
// II.C eq. gen_ev) on the GPU, in FP64.  Section V.C solves this problem by
// shift-and-invert; here the invert step is a banded LDL^T of K = H0 - sigma S
// (sigma below the spectrum, so K is symmetric positive definite), and the
// outer method is subspace iteration with Rayleigh-Ritz:
//   W <- K^-1 S V;  S-orthonormalise W (Cholesky-QR, twice);
//   Rayleigh-Ritz on span(W);  stop when every wanted pair has relative
//   residual |H0 v - e S v| / (|H0 v| + |e| |S v|) below tol.
// Small dense steps (Cholesky of the Gram matrix, Jacobi on the projected
// matrix) run in one GPU thread; everything of size N runs in parallel.
#include <cmath>
#include <vector>

#include "tdsez_internal.hpp"

namespace tdsez {

namespace {

constexpr int kMaxBlock = 36;

// y_j = M x_j for nb vectors (row-major V[j*N + i]); M lower half band by rows.
__global__ void band_mv_kernel(const double* __restrict__ M, int N, int p, int nb,
                               const double* __restrict__ X, double* __restrict__ Y) {
    long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)N * nb) return;
    int j = (int)(idx / N), i = (int)(idx % N);
    const double* x = X + (long long)j * N;
    double s = M[(long long)i * (p + 1)] * x[i];
    for (int d = 1; d <= p; ++d) {
        if (i - d >= 0) s += M[(long long)i * (p + 1) + d] * x[i - d];
        if (i + d < N) s += M[(long long)(i + d) * (p + 1) + d] * x[i + d];
    }
    Y[idx] = s;
}

// K = H0 - sigma S factorised as L D L^T in place (one thread; banded,
// right-looking).  Kf[i*(p+1) + d] = K[i][i-d] on input; on output d >= 1
// holds L[i][i-d] and d = 0 holds D_i.  flag[0] = 1 if a pivot is not > 0.
__global__ void ldlt_factor_kernel(const double* __restrict__ H0, const double* __restrict__ S,
                                   double sigma, int N, int p, double* __restrict__ Kf,
                                   int* __restrict__ flag) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (long long e = 0; e < (long long)N * (p + 1); ++e) Kf[e] = H0[e] - sigma * S[e];
    for (int j = 0; j < N; ++j) {
        double dj = Kf[(long long)j * (p + 1)];
        if (!(dj > 0.0)) { flag[0] = 1; return; }
        // column j of L: L[i][j] = K'[i][j] / D_j for i = j+1..j+p
        for (int i = j + 1; i <= j + p && i < N; ++i) {
            double lij = Kf[(long long)i * (p + 1) + (i - j)] / dj;
            // update the trailing window K'[i][i2] -= L[i][j] K'[i2][j] (j < i2 <= i)
            for (int i2 = j + 1; i2 <= i; ++i2)
                Kf[(long long)i * (p + 1) + (i - i2)] -= lij * Kf[(long long)i2 * (p + 1) + (i2 - j)];
        }
        // store the multipliers after the updates (they used K'[i2][j] unscaled)
        for (int i = j + 1; i <= j + p && i < N; ++i) Kf[(long long)i * (p + 1) + (i - j)] /= dj;
    }
}

// X_j <- K^-1 X_j, one thread per vector.
__global__ void ldlt_solve_kernel(const double* __restrict__ Kf, int N, int p, int nb,
                                  double* __restrict__ X) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    double* x = X + (long long)j * N;
    for (int i = 0; i < N; ++i) {
        double s = x[i];
        for (int d = 1; d <= p && i - d >= 0; ++d) s -= Kf[(long long)i * (p + 1) + d] * x[i - d];
        x[i] = s;
    }
    for (int i = 0; i < N; ++i) x[i] /= Kf[(long long)i * (p + 1)];
    for (int i = N - 1; i >= 0; --i) {
        double s = x[i];
        for (int d = 1; d <= p && i + d < N; ++d) s -= Kf[(long long)(i + d) * (p + 1) + d] * x[i + d];
        x[i] = s;
    }
}

// G[a][b] = sum_i A_a[i] B_b[i]; one block per (a, b), FP64 tree reduction.
__global__ void gram_kernel(const double* __restrict__ A, const double* __restrict__ B, int N, int nb,
                            double* __restrict__ G) {
    int a = blockIdx.x, b = blockIdx.y;
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) s += A[(long long)a * N + i] * B[(long long)b * N + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) G[a * nb + b] = red[0];
}

// Cholesky of the nb x nb Gram matrix and R^-1 (upper), one thread.
__global__ void chol_inv_kernel(double* __restrict__ G, int nb, double* __restrict__ Rinv,
                                int* __restrict__ flag) {
    if (threadIdx.x != 0) return;
    // symmetrise, factor G = R^T R (R upper)
    double R[kMaxBlock][kMaxBlock];
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) R[i][j] = 0.0;
    for (int j = 0; j < nb; ++j) {
        double s = 0.5 * (G[j * nb + j] + G[j * nb + j]);
        for (int k = 0; k < j; ++k) s -= R[k][j] * R[k][j];
        if (!(s > 0.0)) { flag[0] = 2; return; }
        R[j][j] = std::sqrt(s);
        for (int i = j + 1; i < nb; ++i) {
            double t = 0.5 * (G[j * nb + i] + G[i * nb + j]);
            for (int k = 0; k < j; ++k) t -= R[k][j] * R[k][i];
            R[j][i] = t / R[j][j];
        }
    }
    // Rinv (upper triangular)
    for (int j = 0; j < nb; ++j) {
        for (int i = 0; i < nb; ++i) Rinv[i * nb + j] = 0.0;
        Rinv[j * nb + j] = 1.0 / R[j][j];
        for (int i = j - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= j; ++k) s += R[i][k] * Rinv[k * nb + j];
            Rinv[i * nb + j] = -s / R[i][i];
        }
    }
}

// Y_j = sum_a X_a C[a][j]  (X, Y: nb x N row-major vectors; C nb x nb).
__global__ void combine_kernel(const double* __restrict__ X, const double* __restrict__ C, int N, int nb,
                               double* __restrict__ Y) {
    long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)N * nb) return;
    int j = (int)(idx / N), i = (int)(idx % N);
    double s = 0.0;
    for (int a = 0; a < nb; ++a) s += X[(long long)a * N + i] * C[a * nb + j];
    Y[idx] = s;
}

// Cyclic Jacobi on the projected matrix Hs (nb x nb, symmetrised), one
// thread; eigenvalues ascending to ev, eigenvectors to the columns of Y.
__global__ void jacobi_kernel(const double* __restrict__ Hs, int nb, double* __restrict__ ev,
                              double* __restrict__ Y) {
    if (threadIdx.x != 0) return;
    double A[kMaxBlock][kMaxBlock], V[kMaxBlock][kMaxBlock];
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
            A[i][j] = 0.5 * (Hs[i * nb + j] + Hs[j * nb + i]);
            V[i][j] = i == j ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, nrm = 0.0;
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) {
                nrm += A[i][j] * A[i][j];
                if (i != j) off += A[i][j] * A[i][j];
            }
        if (off <= 1e-32 * nrm) break;
        for (int p = 0; p < nb - 1; ++p)
            for (int q = p + 1; q < nb; ++q) {
                if (A[p][q] == 0.0) continue;
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < nb; ++k) {
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < nb; ++k) {
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < nb; ++k) {
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int order[kMaxBlock];
    for (int i = 0; i < nb; ++i) order[i] = i;
    for (int i = 0; i < nb; ++i)
        for (int j = i + 1; j < nb; ++j)
            if (A[order[j]][order[j]] < A[order[i]][order[i]]) {
                int t = order[i]; order[i] = order[j]; order[j] = t;
            }
    for (int j = 0; j < nb; ++j) {
        ev[j] = A[order[j]][order[j]];
        for (int i = 0; i < nb; ++i) Y[i * nb + j] = V[i][order[j]];
    }
}

// relative residual of pair j: |H v - e S v| / (|H v| + |e| |S v|)
__global__ void residual_kernel(const double* __restrict__ HV, const double* __restrict__ SV,
                                const double* __restrict__ ev, int N, double* __restrict__ res) {
    int j = blockIdx.x;
    __shared__ double r2[256], h2[256], s2[256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double h = HV[(long long)j * N + i], s = SV[(long long)j * N + i];
        double r = h - ev[j] * s;
        a += r * r;
        b += h * h;
        c += s * s;
    }
    r2[threadIdx.x] = a;
    h2[threadIdx.x] = b;
    s2[threadIdx.x] = c;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r2[threadIdx.x] += r2[threadIdx.x + w];
            h2[threadIdx.x] += h2[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) res[j] = std::sqrt(r2[0]) / (std::sqrt(h2[0]) + std::fabs(ev[j]) * std::sqrt(s2[0]));
}

// deterministic start vectors: smooth envelopes with a pseudo-random
// perturbation from a 64-bit LCG (Knuth's MMIX constants)
__global__ void start_kernel(int N, int nb, double* __restrict__ V) {
    long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)N * nb) return;
    int j = (int)(idx / N), i = (int)(idx % N);
    unsigned long long z = 6364136223846793005ULL * (unsigned long long)(idx + 1) + 1442695040888963407ULL;
    z ^= z >> 29;
    double r = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    double x = (i + 1.0) / (N + 1.0);
    V[idx] = std::sin(3.14159265358979323846 * (j + 1) * x) + 0.05 * r;
}

}  // namespace

tdsez_status ground_state_device(SystemData* sys, int nev, double sigma, double tol, int maxit,
                                 double* eps_out, double* c_out) {
    const int N = sys->N, p = sys->p;
    if (nev < 1 || nev > N) return fail(TDSEZ_EINVAL, "nev=%d must be in 1..N=%d", nev, N);
    int nb = 2 * nev + 4;
    if (nb > N) nb = N;
    if (nb > kMaxBlock) return fail(TDSEZ_EUNSUPPORTED, "nev=%d too large (max %d)", nev, (kMaxBlock - 4) / 2);
    if (sigma >= 1e300) sigma = sys->minV - 1e-3 * (std::fabs(sys->minV) + 1.0);
    const double* S = sys->d_band[0];
    const double* H = sys->d_H0;
    double *Kf = nullptr, *V = nullptr, *W = nullptr, *HV = nullptr, *SV = nullptr;
    double *G = nullptr, *C = nullptr, *ev = nullptr, *res = nullptr;
    int* flag = nullptr;
    size_t vb = sizeof(double) * (size_t)N * nb;
    auto cleanup = [&]() {
        (void)hipFree(Kf); (void)hipFree(V); (void)hipFree(W); (void)hipFree(HV); (void)hipFree(SV);
        (void)hipFree(G); (void)hipFree(C); (void)hipFree(ev); (void)hipFree(res); (void)hipFree(flag);
    };
#define EIG_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            cleanup();                                                                  \
            return fail(TDSEZ_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
        }                                                                               \
    } while (0)
    EIG_TRY(hipMalloc(&Kf, sizeof(double) * (size_t)N * (p + 1)));
    EIG_TRY(hipMalloc(&V, vb));
    EIG_TRY(hipMalloc(&W, vb));
    EIG_TRY(hipMalloc(&HV, vb));
    EIG_TRY(hipMalloc(&SV, vb));
    EIG_TRY(hipMalloc(&G, sizeof(double) * nb * nb));
    EIG_TRY(hipMalloc(&C, sizeof(double) * nb * nb));
    EIG_TRY(hipMalloc(&ev, sizeof(double) * nb));
    EIG_TRY(hipMalloc(&res, sizeof(double) * nb));
    EIG_TRY(hipMalloc(&flag, sizeof(int)));
    EIG_TRY(hipMemset(flag, 0, sizeof(int)));
    const int th = 256;
    const int nbl = (int)(((long long)N * nb + th - 1) / th);
    ldlt_factor_kernel<<<1, 64>>>(H, S, sigma, N, p, Kf, flag);
    start_kernel<<<nbl, th>>>(N, nb, V);
    EIG_TRY(hipGetLastError());
    int hflag = 0;
    EIG_TRY(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
    if (hflag) {
        cleanup();
        return fail(TDSEZ_EINVAL, "H0 - sigma S is not positive definite for sigma=%g; choose sigma below "
                                  "the lowest eigenvalue", sigma);
    }
    std::vector<double> hres(nb), hev(nb);
    double best = 1e300;
    tdsez_status st = TDSEZ_ENOCONV;
    for (int it = 0; it < maxit; ++it) {
        band_mv_kernel<<<nbl, th>>>(S, N, p, nb, V, W);
        ldlt_solve_kernel<<<1, 64>>>(Kf, N, p, nb, W);
        for (int pass = 0; pass < 2; ++pass) {
            band_mv_kernel<<<nbl, th>>>(S, N, p, nb, W, SV);
            gram_kernel<<<dim3(nb, nb), 256>>>(W, SV, N, nb, G);
            chol_inv_kernel<<<1, 1>>>(G, nb, C, flag);
            combine_kernel<<<nbl, th>>>(W, C, N, nb, V);
            std::swap(V, W);
        }
        // W holds the S-orthonormal basis; Rayleigh-Ritz
        band_mv_kernel<<<nbl, th>>>(H, N, p, nb, W, HV);
        gram_kernel<<<dim3(nb, nb), 256>>>(W, HV, N, nb, G);
        jacobi_kernel<<<1, 1>>>(G, nb, ev, C);
        combine_kernel<<<nbl, th>>>(W, C, N, nb, V);
        band_mv_kernel<<<nbl, th>>>(H, N, p, nb, V, HV);
        band_mv_kernel<<<nbl, th>>>(S, N, p, nb, V, SV);
        residual_kernel<<<nev, 256>>>(HV, SV, ev, N, res);
        EIG_TRY(hipGetLastError());
        EIG_TRY(hipMemcpy(hres.data(), res, sizeof(double) * nev, hipMemcpyDeviceToHost));
        EIG_TRY(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
        if (hflag) {
            cleanup();
            return fail(TDSEZ_ENOCONV, "subspace lost rank (Gram matrix not positive definite)");
        }
        double r = 0.0;
        for (int j = 0; j < nev; ++j) r = std::max(r, hres[j]);
        if (r < tol) { st = TDSEZ_OK; break; }
        if (it % 25 == 24) {
            if (r < 1e-11 && r > 0.5 * best) { st = TDSEZ_OK; break; }  // round-off floor
            best = r;
        }
    }
    if (st != TDSEZ_OK) {
        cleanup();
        return fail(TDSEZ_ENOCONV, "ground state: no convergence to tol=%g in %d iterations", tol, maxit);
    }
    EIG_TRY(hipMemcpy(hev.data(), ev, sizeof(double) * nb, hipMemcpyDeviceToHost));
    std::vector<double> hv((size_t)N * nev);
    EIG_TRY(hipMemcpy(hv.data(), V, sizeof(double) * (size_t)N * nev, hipMemcpyDeviceToHost));
#undef EIG_TRY
    cleanup();
    for (int j = 0; j < nev; ++j) {
        eps_out[j] = hev[j];
        double* c = hv.data() + (size_t)j * N;
        int im = 0;
        for (int i = 1; i < N; ++i)
            if (std::fabs(c[i]) > std::fabs(c[im])) im = i;
        double sg = c[im] < 0.0 ? -1.0 : 1.0;
        for (int i = 0; i < N; ++i) c_out[(size_t)j * N + i] = sg * c[i];
    }
    return TDSEZ_OK;
}

}  // namespace tdsez

// ----------------------------------------------------------------------------
// Batched ground states: one workgroup per system, all systems in one launch.
// Shift-and-invert power iteration on the lowest eigenpair of H0 c = e S c:
//   K = H0 - sigma S = L D L^T (banded, factorised by one lane, FP64);
//   repeat  z = K^-1 S x;  x = z / sqrt(z^T S z);  e = x^T H0 x
//   until |H0 x - e S x| / (|H0 x| + |e| |S x|) < tol (checked every 4 steps).
// The matrix-vector products and reductions use the whole workgroup; the
// banded triangular solves are serial in one lane (the systems run in
// parallel across workgroups).
namespace tdsez {
namespace {

struct GsDesc {
    const double* S;
    const double* H0;
    double* work;      // (p+1)*N factor + 5*N vectors
    long long psi_off; // complex elements into the packed state buffer
    int N, p;
    double sigma;
};

__device__ double block_sum(double v, double* red) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;
}

__device__ void band_mv(const double* __restrict__ M, int N, int p, const double* __restrict__ x,
                        double* __restrict__ y) {
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double s = M[(long long)i * (p + 1)] * x[i];
        for (int d = 1; d <= p; ++d) {
            if (i - d >= 0) s += M[(long long)i * (p + 1) + d] * x[i - d];
            if (i + d < N) s += M[(long long)(i + d) * (p + 1) + d] * x[i + d];
        }
        y[i] = s;
    }
}

// K^-1 y for the banded LDL^T factor K (one thread: the rows are serial)
__device__ void ldl_solve_serial(const double* __restrict__ Kf, int N, int p, const double* __restrict__ y,
                                 double* __restrict__ z) {
    for (int i = 0; i < N; ++i) {
        double s = y[i];
        for (int d = 1; d <= p && i - d >= 0; ++d) s -= Kf[(long long)i * (p + 1) + d] * z[i - d];
        z[i] = s;
    }
    for (int i = 0; i < N; ++i) z[i] /= Kf[(long long)i * (p + 1)];
    for (int i = N - 1; i >= 0; --i) {
        double s = z[i];
        for (int d = 1; d <= p && i + d < N; ++d) s -= Kf[(long long)(i + d) * (p + 1) + d] * z[i + d];
        z[i] = s;
    }
}

// One system per workgroup: the lowest eigenpair of H0 c = e S c by
// shift-and-invert subspace iteration on two vectors with a 2 x 2
// Rayleigh-Ritz step: Z = K^-1 S X (K = H0 - sigma S, factorised once), then
// the Ritz pairs of (Z^T H0 Z, Z^T S Z) give the next X (S-orthonormal).
// The lowest Ritz value converges with the ratio (e0 - sigma)/(e2 - sigma),
// so a near-degenerate lowest pair (a double well's doublet) costs no more
// than a well separated level.
__global__ __launch_bounds__(256) void ground_batched_kernel(const GsDesc* __restrict__ descs, double tol,
                                                             int maxit, double* __restrict__ psi,
                                                             double* __restrict__ eps_out,
                                                             int* __restrict__ status) {
    const GsDesc g = descs[blockIdx.x];
    const int N = g.N, p = g.p;
    double* Kf = g.work;
    double* x1 = Kf + (long long)N * (p + 1);
    double* x2 = x1 + N;
    double* y = x2 + N;
    double* z1 = y + N;
    double* z2 = z1 + N;
    __shared__ double red[4];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    for (long long e = threadIdx.x; e < (long long)N * (p + 1); e += blockDim.x)
        Kf[e] = g.H0[e] - g.sigma * g.S[e];
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double t = (i + 1.0) / (N + 1.0);
        x1[i] = t * (1.0 - t);                // positive, smooth: not orthogonal to the ground state
        x2[i] = t * (1.0 - t) * (t - 0.5);    // odd about the middle: the partner of a symmetric doublet
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < N && !bad; ++j) {
            double dj = Kf[(long long)j * (p + 1)];
            if (!(dj > 0.0)) { bad = 1; break; }
            for (int i = j + 1; i <= j + p && i < N; ++i) {
                double lij = Kf[(long long)i * (p + 1) + (i - j)] / dj;
                for (int i2 = j + 1; i2 <= i; ++i2)
                    Kf[(long long)i * (p + 1) + (i - i2)] -= lij * Kf[(long long)i2 * (p + 1) + (i2 - j)];
            }
            for (int i = j + 1; i <= j + p && i < N; ++i) Kf[(long long)i * (p + 1) + (i - j)] /= dj;
        }
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) status[blockIdx.x] = 1;
        return;
    }
    // u^T M v for a band matrix M (y is scratch)
    auto form = [&](const double* M, const double* u, const double* v) {
        band_mv(M, N, p, v, y);
        __syncthreads();
        double a = 0.0;
        for (int i = threadIdx.x; i < N; i += blockDim.x) a += u[i] * y[i];
        a = block_sum(a, red);
        __syncthreads();
        return a;
    };
    double e = 0.0;
    int it = 0, converged = 0;
    for (; it < maxit && !converged; ++it) {
        // Z = K^-1 S X
        band_mv(g.S, N, p, x1, y);
        __syncthreads();
        if (threadIdx.x == 0) ldl_solve_serial(Kf, N, p, y, z1);
        __syncthreads();
        band_mv(g.S, N, p, x2, y);
        __syncthreads();
        if (threadIdx.x == 0) ldl_solve_serial(Kf, N, p, y, z2);
        __syncthreads();
        // Rayleigh-Ritz on span(z1, z2): A = Z^T H0 Z, B = Z^T S Z
        const double a11 = form(g.H0, z1, z1), a12 = form(g.H0, z1, z2), a22 = form(g.H0, z2, z2);
        const double b11 = form(g.S, z1, z1), b12 = form(g.S, z1, z2), b22 = form(g.S, z2, z2);
        // det(A - l B) = 0: qa l^2 + qb l + qc = 0, qa = det B > 0
        const double qa = b11 * b22 - b12 * b12;
        const double qb = -(a11 * b22 + a22 * b11 - 2.0 * a12 * b12);
        const double qc = a11 * a22 - a12 * a12;
        double l0, u1, u2, w1, w2;
        if (qa > 1e-30 * b11 * b22) {
            const double disc = sqrt(fmax(qb * qb - 4.0 * qa * qc, 0.0));
            // the two roots without cancellation
            const double q = -0.5 * (qb + (qb < 0.0 ? -disc : disc));
            const double r1 = q / qa, r2 = qc / q;
            l0 = fmin(r1, r2);
            const double l1 = fmax(r1, r2);
            // (A - l B) u = 0 from the better-conditioned row
            auto vec = [&](double l, double* v1, double* v2) {
                const double m11 = a11 - l * b11, m12 = a12 - l * b12, m22 = a22 - l * b22;
                if (fabs(m11) + fabs(m12) >= fabs(m12) + fabs(m22)) { *v1 = -m12; *v2 = m11; }
                else { *v1 = m22; *v2 = -m12; }
                const double nn = (*v1) * (*v1) * b11 + 2.0 * (*v1) * (*v2) * b12 + (*v2) * (*v2) * b22;
                const double sc = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
                *v1 *= sc;
                *v2 *= sc;
            };
            vec(l0, &u1, &u2);
            vec(l1, &w1, &w2);
            // the pair is B-orthogonal up to rounding; make it exact for the second
            const double o = u1 * w1 * b11 + (u1 * w2 + u2 * w1) * b12 + u2 * w2 * b22;
            w1 -= o * u1;
            w2 -= o * u2;
            const double nn = w1 * w1 * b11 + 2.0 * w1 * w2 * b12 + w2 * w2 * b22;
            const double sc = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
            w1 *= sc;
            w2 *= sc;
        } else {
            // z2 has no component left outside z1 (a one-dimensional
            // subspace): plain power step on z1, restart z2 from the odd start
            l0 = a11 / b11;
            u1 = 1.0 / sqrt(b11);
            u2 = 0.0;
            w1 = 0.0;
            w2 = 0.0;
        }
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            const double v1 = z1[i], v2 = z2[i];
            x1[i] = u1 * v1 + u2 * v2;
            if (w1 != 0.0 || w2 != 0.0) x2[i] = w1 * v1 + w2 * v2;
            else {
                const double t = (i + 1.0) / (N + 1.0);
                x2[i] = t * (1.0 - t) * (t - 0.5);
            }
        }
        __syncthreads();
        // 1/(l0) is the Ritz value of K^-1 S; the eigenvalue of the pencil
        // is the Rayleigh quotient of x1, checked with its residual
        if ((it & 3) == 3 || it == maxit - 1) {
            band_mv(g.H0, N, p, x1, y);  // y = H0 x1
            band_mv(g.S, N, p, x1, z1);  // z1 = S x1
            __syncthreads();
            double ev = 0.0;
            for (int i = threadIdx.x; i < N; i += blockDim.x) ev += x1[i] * y[i];
            ev = block_sum(ev, red);
            double r2 = 0.0, h2 = 0.0, s2 = 0.0;
            for (int i = threadIdx.x; i < N; i += blockDim.x) {
                double r = y[i] - ev * z1[i];
                r2 += r * r;
                h2 += y[i] * y[i];
                s2 += z1[i] * z1[i];
            }
            r2 = block_sum(r2, red);
            h2 = block_sum(h2, red);
            s2 = block_sum(s2, red);
            e = ev;
            if (sqrt(r2) < tol * (sqrt(h2) + fabs(ev) * sqrt(s2))) converged = 1;
            __syncthreads();
        }
        (void)l0;
    }
    // sign convention: largest-magnitude component positive (lowest index on ties)
    double best = 0.0;
    int bi = 0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < N; ++i)
            if (fabs(x1[i]) > best) { best = fabs(x1[i]); bi = i; }
        red[0] = x1[bi] < 0.0 ? -1.0 : 1.0;
        eps_out[blockIdx.x] = e;
        status[blockIdx.x] = converged ? 0 : 2;
    }
    __syncthreads();
    const double sg = red[0];
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        psi[2 * (g.psi_off + i)] = sg * x1[i];
        psi[2 * (g.psi_off + i) + 1] = 0.0;
    }
}

}  // namespace

tdsez_status ground_state_batched_device(BatchData* b, double sigma, double tol, int maxit, double* eps_out,
                                         double* psi, const long* psi_off) {
    const int nsys = (int)b->sys.size();
    std::vector<GsDesc> hd(nsys);
    long long wtot = 0;
    for (int s = 0; s < nsys; ++s) wtot += (long long)b->sys[s]->N * (b->sys[s]->p + 6);
    double* work = nullptr;
    GsDesc* dd = nullptr;
    double* dev_eps = nullptr;
    int* dstat = nullptr;
    auto cleanup = [&]() { (void)hipFree(work); (void)hipFree(dd); (void)hipFree(dev_eps); (void)hipFree(dstat); };
#define GB_TRY(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            cleanup();                                                                  \
            return fail(TDSEZ_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
        }                                                                               \
    } while (0)
    GB_TRY(hipMalloc(&work, sizeof(double) * (size_t)wtot));
    long long woff = 0;
    for (int s = 0; s < nsys; ++s) {
        SystemData* sy = b->sys[s];
        double sg = sigma >= 1e300 ? sy->minV - 1e-3 * (std::fabs(sy->minV) + 1.0) : sigma;
        hd[s] = GsDesc{sy->d_band[0], sy->d_H0, work + woff, (long long)psi_off[s], sy->N, sy->p, sg};
        woff += (long long)sy->N * (sy->p + 6);
    }
    GB_TRY(hipMalloc(&dd, sizeof(GsDesc) * nsys));
    GB_TRY(hipMalloc(&dev_eps, sizeof(double) * nsys));
    GB_TRY(hipMalloc(&dstat, sizeof(int) * nsys));
    GB_TRY(hipMemcpy(dd, hd.data(), sizeof(GsDesc) * nsys, hipMemcpyHostToDevice));
    ground_batched_kernel<<<nsys, 256>>>(dd, tol, maxit, psi, dev_eps, dstat);
    GB_TRY(hipGetLastError());
    std::vector<int> hs(nsys);
    GB_TRY(hipMemcpy(eps_out, dev_eps, sizeof(double) * nsys, hipMemcpyDeviceToHost));
    GB_TRY(hipMemcpy(hs.data(), dstat, sizeof(int) * nsys, hipMemcpyDeviceToHost));
#undef GB_TRY
    cleanup();
    for (int s = 0; s < nsys; ++s) {
        if (hs[s] == 1)
            return fail(TDSEZ_EINVAL, "system %d: H0 - sigma S not positive definite (choose sigma below the spectrum)", s);
        if (hs[s] == 2) return fail(TDSEZ_ENOCONV, "system %d: no convergence to tol=%g in %d iterations", s, tol, maxit);
    }
    return TDSEZ_OK;
}

}  // namespace tdsez
