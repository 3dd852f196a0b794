// Galerkin assembly of the B-spline matrices on the GPU.
//
// The element formulas are those of the paper's section V.A (overlap matrix,
// BenDaniel-Duke kinetic matrix with m^-1 sampled at the quadrature points,
// potential and dipole matrices) together with the two matrices that turn
// the Ehrenfest acceleration of section IV.A (eq. pdm_acceleration, without
// the a_Q term) into quadratic forms: G = <B| m^-1 V' |B>, Mi = <B| m^-1 |B>.
// Quadrature is Gauss-Legendre per knot span (section II.C).
//
// Two kernels: (1) one thread per quadrature point evaluates the order-k
// B-splines that are non-zero on its span and their derivatives; (2) one
// thread per band entry (row, diagonal) sums the span contributions in a
// fixed order, so assembly is deterministic (no atomics).
#include <cmath>

#include "tdsez_internal.hpp"

namespace tdsez {

// Gauss-Legendre nodes/weights on [-1,1]: Newton iteration on P_n started
// from the asymptotic root estimate; P_n and P_n' from the three-term
// recurrence.  Nodes ascending.
int gauss_legendre_host(int n, double* x, double* w) {
    if (n < 1 || n > 32) return 1;
    const double pi = 3.14159265358979323846;
    for (int k = 1; k <= n; ++k) {
        // k-th largest root, estimate cos(pi (k - 1/4) / (n + 1/2))
        double z = std::cos(pi * (k - 0.25) / (n + 0.5));
        double pn = 0.0, dpn = 1.0;
        for (int iter = 0; iter < 60; ++iter) {
            double p0 = 1.0, p1 = z;
            for (int l = 2; l <= n; ++l) {
                double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 1) ? z : p1;
            double pm1 = (n == 1) ? 1.0 : p0;
            dpn = n * (pm1 - z * pn) / (1.0 - z * z);
            double step = pn / dpn;
            z -= step;
            if (std::fabs(step) <= 4e-17) break;
        }
        // final derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int l = 2; l <= n; ++l) {
            double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
            p0 = p1;
            p1 = p2;
        }
        double pm1 = (n == 1) ? 1.0 : p0;
        double pcur = (n == 1) ? z : p1;
        dpn = n * (pm1 - z * pcur) / (1.0 - z * z);
        x[n - k] = z;
        w[n - k] = 2.0 / ((1.0 - z * z) * dpn * dpn);
    }
    return 0;
}

// Knot t_i of the open knot vector (end breakpoints repeated p+1 times).
__device__ inline double knot(const double* br, int nbr, int p, int i) {
    int j = i - p;
    j = j < 0 ? 0 : (j > nbr - 1 ? nbr - 1 : j);
    return br[j];
}

// One thread per quadrature point (span e, point q).  Writes the values and
// first derivatives of B_{e}, ..., B_{e+p} (global indices) at x_q.
// Order-(j+1) values come from order j by the left/right-difference form of
// the Cox-de Boor recursion (de Boor, BSPLVB).
__global__ void basis_kernel(const double* __restrict__ br, int nbr, int p, int nq,
                             const double* __restrict__ xq, double* __restrict__ Bv,
                             double* __restrict__ dB) {
    int nel = nbr - 1;
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nel * nq) return;
    int e = idx / nq;
    int mu = p + e;  // t_mu = br[e], t_{mu+1} = br[e+1]
    double x = xq[idx];
    double b[kMaxP + 1], bprev[kMaxP + 1];
    double left[kMaxP + 1], right[kMaxP + 1];
    b[0] = 1.0;
    bprev[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        if (j == p)
            for (int r = 0; r < p; ++r) bprev[r] = b[r];
        left[j] = x - knot(br, nbr, p, mu + 1 - j);
        right[j] = knot(br, nbr, p, mu + j) - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double den = right[r + 1] + left[j - r];
            double temp = b[r] / den;
            b[r] = saved + right[r + 1] * temp;
            saved = left[j - r] * temp;
        }
        b[j] = saved;
    }
    // derivative of order-(p+1) B_i: p [B_{i,p}/(t_{i+p}-t_i) - B_{i+1,p}/(t_{i+p+1}-t_{i+1})]
    // with bprev[a] = B_{mu-p+1+a, p} for a = 0..p-1
    for (int a = 0; a <= p; ++a) {
        int i = mu - p + a;
        double d = 0.0;
        if (p >= 1) {
            if (a >= 1) {
                double den = knot(br, nbr, p, i + p) - knot(br, nbr, p, i);
                if (den > 0.0) d += bprev[a - 1] / den;
            }
            if (a <= p - 1) {
                double den = knot(br, nbr, p, i + p + 1) - knot(br, nbr, p, i + 1);
                if (den > 0.0) d -= bprev[a] / den;
            }
            d *= p;
        }
        Bv[(size_t)idx * (p + 1) + a] = b[a];
        dB[(size_t)idx * (p + 1) + a] = d;
    }
}

// One thread per lower band entry M[j][j-d] (unknown indices, Dirichlet ends
// removed: unknown j is global B-spline j+1).  Sums over the knot spans shared
// by the two B-splines, then over the quadrature points of each span.
__global__ void band_kernel(const double* __restrict__ br, int nbr, int p, int nq, int N,
                            const double* __restrict__ gw, const double* __restrict__ xq,
                            const double* __restrict__ Bv, const double* __restrict__ dB,
                            const double* __restrict__ minv_q, const double* __restrict__ V_q,
                            const double* __restrict__ dV_q, double* __restrict__ S,
                            double* __restrict__ T, double* __restrict__ V, double* __restrict__ D,
                            double* __restrict__ G, double* __restrict__ Mi,
                            double* __restrict__ H0, double* __restrict__ K) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * (p + 1)) return;
    int j = idx / (p + 1), d = idx % (p + 1);
    double s = 0.0, t = 0.0, v = 0.0, dd = 0.0, g = 0.0, mi = 0.0, kv = 0.0;
    if (j - d >= 0) {
        int nel = nbr - 1;
        int g1 = j + 1, g2 = j + 1 - d;  // g1 >= g2
        int e0 = g1 - p > 0 ? g1 - p : 0;
        int e1 = g2 < nel - 1 ? g2 : nel - 1;
        for (int e = e0; e <= e1; ++e) {
            int a1 = g1 - e, a2 = g2 - e;
            double h = 0.5 * (br[e + 1] - br[e]);
            for (int q = 0; q < nq; ++q) {
                size_t iq = (size_t)e * nq + q;
                double w = gw[q] * h;
                double nn = w * Bv[iq * (p + 1) + a1] * Bv[iq * (p + 1) + a2];
                double mv = minv_q ? minv_q[iq] : 1.0;
                s += nn;
                t += 0.5 * w * mv * dB[iq * (p + 1) + a1] * dB[iq * (p + 1) + a2];
                v += nn * (V_q ? V_q[iq] : 0.0);
                dd += nn * xq[iq];
                g += nn * mv * (dV_q ? dV_q[iq] : 0.0);
                mi += nn * mv;
                // velocity (eq. vel_elem without its -i/2): row j, column j-d
                kv += w * mv * (Bv[iq * (p + 1) + a1] * dB[iq * (p + 1) + a2] -
                                dB[iq * (p + 1) + a1] * Bv[iq * (p + 1) + a2]);
            }
        }
    }
    S[idx] = s;
    T[idx] = t;
    V[idx] = v;
    D[idx] = dd;
    G[idx] = g;
    Mi[idx] = mi;
    H0[idx] = t + v;
    K[idx] = kv;
}

// Absorber weight W[j][j-d] = sum w eta N_j N_{j-d} (the CAP matrix of
// section V.A is -i W) when aq_form is false, or the a_Q form
// Q[j][j-d] = sum w (g N'_j N'_{j-d} / 2 - h N_j N_{j-d} / 4) with g = a_q,
// h = b_q: eq. aQ_definition expanded for a smooth inverse mass mu, with
// g = mu mu_1 and h = mu_1 mu_2 + mu mu_3 (mu_k the k-th derivative of mu).
// Same summation order as band_kernel.
__global__ void extra_band_kernel(const double* __restrict__ br, int nbr, int p, int nq, int N,
                                  const double* __restrict__ gw, const double* __restrict__ Bv,
                                  const double* __restrict__ dB, const double* __restrict__ a_q,
                                  const double* __restrict__ b_q, bool aq_form, double* __restrict__ out) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * (p + 1)) return;
    int j = idx / (p + 1), d = idx % (p + 1);
    double acc = 0.0;
    if (j - d >= 0) {
        int nel = nbr - 1;
        int g1 = j + 1, g2 = j + 1 - d;
        int e0 = g1 - p > 0 ? g1 - p : 0;
        int e1 = g2 < nel - 1 ? g2 : nel - 1;
        for (int e = e0; e <= e1; ++e) {
            int a1 = g1 - e, a2 = g2 - e;
            double h = 0.5 * (br[e + 1] - br[e]);
            for (int q = 0; q < nq; ++q) {
                size_t iq = (size_t)e * nq + q;
                double w = gw[q] * h;
                double nn = w * Bv[iq * (p + 1) + a1] * Bv[iq * (p + 1) + a2];
                if (aq_form) {
                    double gg = a_q ? a_q[iq] : 0.0, hh = b_q ? b_q[iq] : 0.0;
                    acc += 0.5 * w * gg * dB[iq * (p + 1) + a1] * dB[iq * (p + 1) + a2] - 0.25 * hh * nn;
                } else {
                    acc += nn * (a_q ? a_q[iq] : 0.0);
                }
            }
        }
    }
    out[idx] = acc;
}

// y = M x for the FP64 symmetric band M (lower rows M[j][j-d]) and nv real
// vectors x (natural order), one thread per output entry.
__global__ void symband_real_kernel(const double* __restrict__ M, int N, int p, int nv,
                                    const double* __restrict__ x, double* __restrict__ y) {
    long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)N * nv) return;
    int v = (int)(idx / N), i = (int)(idx % N);
    const double* xv = x + (size_t)v * N;
    double s = 0.0;
    for (int d = 0; d <= p; ++d) {
        if (i - d >= 0) s += M[(size_t)i * (p + 1) + d] * xv[i - d];
        if (d > 0 && i + d < N) s += M[(size_t)(i + d) * (p + 1) + d] * xv[i + d];
    }
    y[idx] = s;
}

tdsez_status assemble_device(const double* breaks, int nbreaks, int order, int nq,
                             const double* minv_q, const double* V_q, const double* dV_q,
                             SystemData* sys) {
    int p = order - 1, nel = nbreaks - 1;
    int N = nel + p - 2;
    size_t nqt = (size_t)nel * nq;
    double gx[32], gw[32];
    gauss_legendre_host(nq, gx, gw);
    std::vector<double> xq(nqt);
    for (int e = 0; e < nel; ++e) {
        double h = 0.5 * (breaks[e + 1] - breaks[e]), c = 0.5 * (breaks[e + 1] + breaks[e]);
        for (int q = 0; q < nq; ++q) xq[(size_t)e * nq + q] = c + h * gx[q];
    }
    double *d_br = nullptr, *d_gw = nullptr, *d_xq = nullptr, *d_Bv = nullptr, *d_dB = nullptr;
    double *d_minv = nullptr, *d_V = nullptr, *d_dV = nullptr;
    tdsez_status st = TDSEZ_OK;
    size_t bw = (size_t)N * (p + 1);
    auto cleanup = [&]() {
        (void)hipFree(d_br); (void)hipFree(d_gw); (void)hipFree(d_xq); (void)hipFree(d_Bv);
        (void)hipFree(d_dB); (void)hipFree(d_minv); (void)hipFree(d_V); (void)hipFree(d_dV);
    };
#define ASM_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            cleanup();                                                                  \
            return fail(TDSEZ_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
        }                                                                               \
    } while (0)
    ASM_TRY(hipMalloc(&d_br, sizeof(double) * nbreaks));
    ASM_TRY(hipMalloc(&d_gw, sizeof(double) * nq));
    ASM_TRY(hipMalloc(&d_xq, sizeof(double) * nqt));
    ASM_TRY(hipMalloc(&d_Bv, sizeof(double) * nqt * (p + 1)));
    ASM_TRY(hipMalloc(&d_dB, sizeof(double) * nqt * (p + 1)));
    ASM_TRY(hipMemcpy(d_br, breaks, sizeof(double) * nbreaks, hipMemcpyHostToDevice));
    ASM_TRY(hipMemcpy(d_gw, gw, sizeof(double) * nq, hipMemcpyHostToDevice));
    ASM_TRY(hipMemcpy(d_xq, xq.data(), sizeof(double) * nqt, hipMemcpyHostToDevice));
    if (minv_q) {
        ASM_TRY(hipMalloc(&d_minv, sizeof(double) * nqt));
        ASM_TRY(hipMemcpy(d_minv, minv_q, sizeof(double) * nqt, hipMemcpyHostToDevice));
    }
    if (V_q) {
        ASM_TRY(hipMalloc(&d_V, sizeof(double) * nqt));
        ASM_TRY(hipMemcpy(d_V, V_q, sizeof(double) * nqt, hipMemcpyHostToDevice));
    }
    if (dV_q) {
        ASM_TRY(hipMalloc(&d_dV, sizeof(double) * nqt));
        ASM_TRY(hipMemcpy(d_dV, dV_q, sizeof(double) * nqt, hipMemcpyHostToDevice));
    }
    for (int m = 0; m < 6; ++m) ASM_TRY(hipMalloc(&sys->d_band[m], sizeof(double) * bw));
    ASM_TRY(hipMalloc(&sys->d_H0, sizeof(double) * bw));
    ASM_TRY(hipMalloc(&sys->d_K, sizeof(double) * bw));
    {
        int th = 128;
        int nb = (int)((nqt + th - 1) / th);
        basis_kernel<<<nb, th>>>(d_br, nbreaks, p, nq, d_xq, d_Bv, d_dB);
        ASM_TRY(hipGetLastError());
        nb = (int)((bw + th - 1) / th);
        band_kernel<<<nb, th>>>(d_br, nbreaks, p, nq, N, d_gw, d_xq, d_Bv, d_dB, d_minv, d_V, d_dV,
                                sys->d_band[0], sys->d_band[1], sys->d_band[2], sys->d_band[3],
                                sys->d_band[4], sys->d_band[5], sys->d_H0, sys->d_K);
        ASM_TRY(hipGetLastError());
        ASM_TRY(hipDeviceSynchronize());
    }
#undef ASM_TRY
    cleanup();
    sys->N = N;
    sys->p = p;
    sys->order = order;
    sys->nq = nq;
    sys->nbreaks = nbreaks;
    sys->breaks.assign(breaks, breaks + nbreaks);
    double mv = 0.0;
    bool first = true;
    if (V_q)
        for (size_t i = 0; i < nqt; ++i)
            if (first || V_q[i] < mv) { mv = V_q[i]; first = false; }
    sys->minV = mv;
    sys->const_mass = true;
    if (minv_q)
        for (size_t i = 0; i < nqt; ++i)
            if (minv_q[i] != 1.0) { sys->const_mass = false; break; }
    return st;
}

tdsez_status assemble_extra_device(SystemData* sys, int which, const double* a_q, const double* b_q) {
    const int p = sys->p, nq = sys->nq, nbreaks = sys->nbreaks, nel = nbreaks - 1, N = sys->N;
    const size_t nqt = (size_t)nel * nq, bw = (size_t)N * (p + 1);
    double gx[32], gw[32];
    gauss_legendre_host(nq, gx, gw);
    std::vector<double> xq(nqt);
    for (int e = 0; e < nel; ++e) {
        double h = 0.5 * (sys->breaks[e + 1] - sys->breaks[e]), c = 0.5 * (sys->breaks[e + 1] + sys->breaks[e]);
        for (int q = 0; q < nq; ++q) xq[(size_t)e * nq + q] = c + h * gx[q];
    }
    double *d_br = nullptr, *d_gw = nullptr, *d_xq = nullptr, *d_Bv = nullptr, *d_dB = nullptr;
    double *d_a = nullptr, *d_b = nullptr, *d_out = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(d_br); (void)hipFree(d_gw); (void)hipFree(d_xq); (void)hipFree(d_Bv);
        (void)hipFree(d_dB); (void)hipFree(d_a); (void)hipFree(d_b); (void)hipFree(d_out);
    };
#define XT_TRY(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            cleanup();                                                                  \
            return fail(TDSEZ_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
        }                                                                               \
    } while (0)
    XT_TRY(hipMalloc(&d_br, sizeof(double) * nbreaks));
    XT_TRY(hipMalloc(&d_gw, sizeof(double) * nq));
    XT_TRY(hipMalloc(&d_xq, sizeof(double) * nqt));
    XT_TRY(hipMalloc(&d_Bv, sizeof(double) * nqt * (p + 1)));
    XT_TRY(hipMalloc(&d_dB, sizeof(double) * nqt * (p + 1)));
    XT_TRY(hipMalloc(&d_out, sizeof(double) * bw));
    XT_TRY(hipMemcpy(d_br, sys->breaks.data(), sizeof(double) * nbreaks, hipMemcpyHostToDevice));
    XT_TRY(hipMemcpy(d_gw, gw, sizeof(double) * nq, hipMemcpyHostToDevice));
    XT_TRY(hipMemcpy(d_xq, xq.data(), sizeof(double) * nqt, hipMemcpyHostToDevice));
    if (a_q) {
        XT_TRY(hipMalloc(&d_a, sizeof(double) * nqt));
        XT_TRY(hipMemcpy(d_a, a_q, sizeof(double) * nqt, hipMemcpyHostToDevice));
    }
    if (b_q) {
        XT_TRY(hipMalloc(&d_b, sizeof(double) * nqt));
        XT_TRY(hipMemcpy(d_b, b_q, sizeof(double) * nqt, hipMemcpyHostToDevice));
    }
    {
        int th = 128;
        int nb = (int)((nqt + th - 1) / th);
        basis_kernel<<<nb, th>>>(d_br, nbreaks, p, nq, d_xq, d_Bv, d_dB);
        XT_TRY(hipGetLastError());
        nb = (int)((bw + th - 1) / th);
        extra_band_kernel<<<nb, th>>>(d_br, nbreaks, p, nq, N, d_gw, d_Bv, d_dB, d_a, d_b, which == 1, d_out);
        XT_TRY(hipGetLastError());
        XT_TRY(hipDeviceSynchronize());
    }
#undef XT_TRY
    double*& slot = which == 1 ? sys->d_Q : sys->d_W;
    (void)hipFree(slot);
    slot = d_out;
    d_out = nullptr;
    cleanup();
    return TDSEZ_OK;
}

tdsez_status set_projectors_device(SystemData* sys, int npop, const double* phi) {
    const int N = sys->N, p = sys->p;
    (void)hipFree(sys->d_pops);
    sys->d_pops = nullptr;
    sys->npop = 0;
    if (npop == 0) return TDSEZ_OK;
    double* d_phi = nullptr;
    double* d_out = nullptr;
    const size_t n = (size_t)npop * N;
    if (hipMalloc(&d_phi, sizeof(double) * n) != hipSuccess || hipMalloc(&d_out, sizeof(double) * n) != hipSuccess) {
        (void)hipFree(d_phi);
        (void)hipFree(d_out);
        return fail(TDSEZ_ENOMEM, "projection states: device allocation failed");
    }
    hipError_t e = hipMemcpy(d_phi, phi, sizeof(double) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        symband_real_kernel<<<(int)((n + 127) / 128), 128>>>(sys->d_band[0], N, p, npop, d_phi, d_out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(d_phi);
    if (e != hipSuccess) {
        (void)hipFree(d_out);
        return fail(TDSEZ_EHIP, "projection states: %s", hipGetErrorString(e));
    }
    sys->d_pops = d_out;
    sys->npop = npop;
    return TDSEZ_OK;
}

}  // namespace tdsez

