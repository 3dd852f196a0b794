// C ABI of libtdsez (declared in include/tdsez.h): argument checking, handle
// management and error reporting around the device code of tdsez_*.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "tdsez_internal.hpp"

namespace tdsez {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

tdsez_status fail(tdsez_status st, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

static tdsez_status check_breaks(const double* breaks, int nbreaks) {
    if (!breaks) return fail(TDSEZ_EINVAL, "breaks is NULL");
    if (nbreaks < 2) return fail(TDSEZ_EINVAL, "nbreaks=%d < 2", nbreaks);
    for (int i = 0; i + 1 < nbreaks; ++i)
        if (!(breaks[i + 1] > breaks[i]) || !std::isfinite(breaks[i]) || !std::isfinite(breaks[i + 1]))
            return fail(TDSEZ_EINVAL, "breaks must be finite and strictly increasing (index %d)", i);
    return TDSEZ_OK;
}

static void free_batch_device(BatchData* b) {
    (void)hipFree(b->d_band64);
    (void)hipFree(b->d_band32);
    (void)hipFree(b->d_bandlo);
    (void)hipFree(b->d_state);
    (void)hipFree(b->d_dtot);
    (void)hipFree(b->d_rhs);
    (void)hipFree(b->d_lam);
    (void)hipFree(b->d_wsol);
    (void)hipFree(b->d_ckpt);
    (void)hipFree(b->d_seg);
    (void)hipFree(b->d_fac_seg);
    (void)hipFree(b->d_red_seg);
    b->d_lam = b->d_wsol = b->d_ckpt = b->d_seg = nullptr;
    b->d_fac_seg = b->d_red_seg = nullptr;
    b->ckpt_elems = b->seg_elems = 0;
    b->fac_seg_elems = b->red_seg_elems = 0;
    (void)hipFree(b->d_fac);
    (void)hipFree(b->d_red);
    (void)hipFree(b->d_desc);
    (void)hipFree(b->d_order);
    b->d_order = nullptr;
    (void)hipFree(b->d_status);
    (void)hipFree(b->d_prof);
    b->d_prof = nullptr;
    (void)hipFree(b->d_proj);
    (void)hipFree(b->d_c0);
    b->d_proj = nullptr;
    b->d_c0 = nullptr;
    b->d_band64 = nullptr;
    b->d_band32 = nullptr;
    b->d_bandlo = nullptr;
    b->d_state = nullptr;
    b->d_dtot = nullptr;
    b->d_rhs = nullptr;
    b->d_fac = nullptr;
    b->d_red = nullptr;
    b->d_desc = nullptr;
    b->desc_on_device.clear();
    b->d_status = nullptr;
    (void)hipFree(b->d_xch);
    (void)hipFree(b->d_gfac);
    (void)hipFree(b->d_obs_part);
    b->d_xch = b->d_gfac = nullptr;
    b->d_obs_part = nullptr;
    b->obs_part_elems = 0;
}

}  // namespace tdsez

using namespace tdsez;


extern "C" {

const char* tdsez_last_error(void) { return g_last_error.c_str(); }

int tdsez_version(void) { return 100; }

tdsez_status tdsez_gauss_legendre(int nq, double* x_out, double* w_out) {
    if (!x_out || !w_out) return fail(TDSEZ_EINVAL, "NULL output");
    if (nq < 1 || nq > 32) return fail(TDSEZ_EINVAL, "nq=%d outside 1..32", nq);
    gauss_legendre_host(nq, x_out, w_out);
    return TDSEZ_OK;
}

tdsez_status tdsez_quad_points(const double* breaks, int nbreaks, int nq, double* x_out) {
    tdsez_status st = check_breaks(breaks, nbreaks);
    if (st) return st;
    if (!x_out) return fail(TDSEZ_EINVAL, "x_out is NULL");
    if (nq < 1 || nq > 32) return fail(TDSEZ_EINVAL, "nq=%d outside 1..32", nq);
    double gx[32], gw[32];
    gauss_legendre_host(nq, gx, gw);
    for (int e = 0; e + 1 < nbreaks; ++e) {
        double h = 0.5 * (breaks[e + 1] - breaks[e]), c = 0.5 * (breaks[e + 1] + breaks[e]);
        for (int q = 0; q < nq; ++q) x_out[(size_t)e * nq + q] = c + h * gx[q];
    }
    return TDSEZ_OK;
}

tdsez_status tdsez_assemble(const double* breaks, int nbreaks, int order, int nq,
                            const double* minv_q, const double* V_q, const double* dV_q,
                            tdsez_system* out) {
    if (!out) return fail(TDSEZ_EINVAL, "out is NULL");
    *out = nullptr;
    tdsez_status st = check_breaks(breaks, nbreaks);
    if (st) return st;
    if (order < 2) return fail(TDSEZ_EINVAL, "order=%d < 2", order);
    if (order > kMaxP + 1) return fail(TDSEZ_EUNSUPPORTED, "order=%d > %d", order, kMaxP + 1);
    if (nq < 1 || nq > 32) return fail(TDSEZ_EINVAL, "nq=%d outside 1..32", nq);
    int N = (nbreaks - 1) + (order - 1) - 2;
    if (N < 1) return fail(TDSEZ_EINVAL, "no unknowns left after Dirichlet removal (N=%d)", N);
    size_t nqt = (size_t)(nbreaks - 1) * nq;
    const double* arrs[3] = {minv_q, V_q, dV_q};
    for (int a = 0; a < 3; ++a)
        if (arrs[a])
            for (size_t i = 0; i < nqt; ++i)
                if (!std::isfinite(arrs[a][i]))
                    return fail(TDSEZ_EINVAL, "non-finite sample %zu in input array %d", i, a);
    if (minv_q)
        for (size_t i = 0; i < nqt; ++i)
            if (!(minv_q[i] > 0.0)) return fail(TDSEZ_EINVAL, "m^-1 must be positive (sample %zu)", i);
    tdsez_system_s* s = new (std::nothrow) tdsez_system_s();
    if (!s) return fail(TDSEZ_ENOMEM, "host allocation failed");
    st = assemble_device(breaks, nbreaks, order, nq, minv_q, V_q, dV_q, &s->d);
    if (st) {
        tdsez_system_destroy(s);
        return st;
    }
    *out = s;
    return TDSEZ_OK;
}

tdsez_status tdsez_system_size(tdsez_system sys, int* ndof, int* halfbw) {
    if (!sys) return fail(TDSEZ_EINVAL, "sys is NULL");
    if (ndof) *ndof = sys->d.N;
    if (halfbw) *halfbw = sys->d.p;
    return TDSEZ_OK;
}

tdsez_status tdsez_get_band(tdsez_system sys, int which, double* host_out) {
    if (!sys || !host_out) return fail(TDSEZ_EINVAL, "NULL argument");
    const int N = sys->d.N, p = sys->d.p;
    const double* src = nullptr;
    double sign = 1.0;
    if (which >= TDSEZ_BAND_S && which <= TDSEZ_BAND_MI) src = sys->d.d_band[which];
    else if (which == TDSEZ_BAND_H0) src = sys->d.d_H0;
    else if (which == TDSEZ_BAND_K) {
        src = sys->d.d_K;
        sign = -1.0;  // antisymmetric: K[i][i+d] = -K[i+d][i]
    } else if (which == TDSEZ_BAND_W) src = sys->d.d_W;
    else if (which == TDSEZ_BAND_Q) src = sys->d.d_Q;
    else return fail(TDSEZ_EINVAL, "unknown band selector %d", which);
    if (!src) return fail(TDSEZ_EINVAL, "band %d is not set for this system", which);
    std::vector<double> rows((size_t)N * (p + 1));
    TDSEZ_HIP_TRY(hipMemcpy(rows.data(), src, sizeof(double) * rows.size(), hipMemcpyDeviceToHost));
    // rows[j*(p+1)+d] = M[j][j-d]  ->  band[d*N + i] = M[i][i+d] = M[i+d][i]
    for (int d = 0; d <= p; ++d)
        for (int i = 0; i < N; ++i)
            host_out[(size_t)d * N + i] = (i + d < N) ? sign * rows[(size_t)(i + d) * (p + 1) + d] : 0.0;
    return TDSEZ_OK;
}

tdsez_status tdsez_ground_state(tdsez_system sys, int nev, double sigma, double tol, int maxit,
                                double* eps_out, double* c_out) {
    if (!sys || !eps_out || !c_out) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!(tol > 0.0)) return fail(TDSEZ_EINVAL, "tol must be > 0");
    if (maxit < 1) return fail(TDSEZ_EINVAL, "maxit must be >= 1");
    return ground_state_device(&sys->d, nev, sigma, tol, maxit, eps_out, c_out);
}

tdsez_status tdsez_ground_state_batched(tdsez_batch b, double sigma, double tol, int maxit, double* eps_out,
                                       double* psi_packed, const long* psi_off) {
    if (!b || !eps_out || !psi_packed || !psi_off) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!(tol > 0.0)) return fail(TDSEZ_EINVAL, "tol must be > 0");
    if (maxit < 1) return fail(TDSEZ_EINVAL, "maxit must be >= 1");
    for (size_t s = 0; s < b->d.sys.size(); ++s)
        if (psi_off[s] < 0) return fail(TDSEZ_EINVAL, "negative psi offset for system %zu", s);
    return ground_state_batched_device(&b->d, sigma, tol, maxit, eps_out, psi_packed, psi_off);
}

tdsez_status tdsez_batch_create(const tdsez_system* sys, int nsys, tdsez_batch* out) {
    if (!out) return fail(TDSEZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (!sys || nsys < 1) return fail(TDSEZ_EINVAL, "need at least one system");
    for (int s = 0; s < nsys; ++s)
        if (!sys[s]) return fail(TDSEZ_EINVAL, "system %d is NULL", s);
    tdsez_batch_s* b = new (std::nothrow) tdsez_batch_s();
    if (!b) return fail(TDSEZ_ENOMEM, "host allocation failed");
    for (int s = 0; s < nsys; ++s) b->d.sys.push_back(&sys[s]->d);
    tdsez_status st = pack_bands(&b->d);
    if (st) {
        tdsez_batch_destroy(b);
        return st;
    }
    *out = b;
    return TDSEZ_OK;
}

tdsez_status tdsez_batch_set(tdsez_batch b, const char* key, double value) {
    if (!b || !key) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!std::strcmp(key, "refine")) {
        if (!(value >= 0 && value <= 4) || value != (double)(int)value)
            return fail(TDSEZ_EINVAL, "refine must be an integer in 0..4");
        b->d.refine = (int)value;
        return TDSEZ_OK;
    }
    if (!std::strcmp(key, "refine_tol")) {
        if (!(value >= 0.0) || std::isnan(value)) return fail(TDSEZ_EINVAL, "refine_tol must be >= 0");
        b->d.refine_tol = value;
        return TDSEZ_OK;
    }
    if (!std::strcmp(key, "norm_tol")) {
        if (!(value >= 0.0)) return fail(TDSEZ_EINVAL, "norm_tol must be >= 0");
        b->d.norm_tol = value;
        return TDSEZ_OK;
    }
    if (!std::strcmp(key, "profile")) {
        if (value != 0.0 && !b->d.d_prof) {
            size_t bytes = sizeof(unsigned long long) * kProfSlots * b->d.sys.size();
            TDSEZ_HIP_TRY(hipMalloc(&b->d.d_prof, bytes));
            TDSEZ_HIP_TRY(hipMemset(b->d.d_prof, 0, bytes));
        } else if (value == 0.0 && b->d.d_prof) {
            (void)hipFree(b->d.d_prof);
            b->d.d_prof = nullptr;
        }
        return TDSEZ_OK;
    }
    if (!std::strcmp(key, "max_waves")) {
        if (value != 2.0 && value != 4.0) return fail(TDSEZ_EINVAL, "max_waves must be 2 or 4");
        bool prof = b->d.d_prof != nullptr;
        b->d.max_waves = (int)value;
        b->d.tuned_chunks.clear();
        free_batch_device(&b->d);
        tdsez_status st = pack_bands(&b->d);
        if (st == TDSEZ_OK && prof) return tdsez_batch_set(b, "profile", 1.0);
        return st;
    }
    if (!std::strcmp(key, "chunks")) {
        bool prof = b->d.d_prof != nullptr;
        if (value < 0 || value > kMaxChunks4 || value != std::floor(value))
            return fail(TDSEZ_EINVAL, "chunks must be an integer in 0..%d", kMaxChunks4);
        b->d.force_chunks = (int)value;
        b->d.tuned_chunks.clear();
        free_batch_device(&b->d);
        tdsez_status st = pack_bands(&b->d);
        if (st == TDSEZ_OK && prof) return tdsez_batch_set(b, "profile", 1.0);
        return st;
    }
    return fail(TDSEZ_EINVAL, "unknown key '%s'", key);
}

tdsez_status tdsez_propagate_batched(tdsez_batch b, double* psi_packed, const long* psi_off,
                                     const double* E_packed, const long* E_off, const double* dt,
                                     const int* nsteps, tdsez_precision prec, unsigned obs,
                                     double* obs_packed, const long* obs_off, void* stream) {
    return tdsez_propagate_batched_ext(b, psi_packed, psi_off, E_packed, E_off, dt, nsteps, prec, obs, obs_packed,
                                       obs_off, 0u, nullptr, nullptr, stream);
}

tdsez_status tdsez_propagate_batched_ext(tdsez_batch b, double* psi_packed, const long* psi_off,
                                         const double* E_packed, const long* E_off, const double* dt,
                                         const int* nsteps, tdsez_precision prec, unsigned obs,
                                         double* obs_packed, const long* obs_off, unsigned ext,
                                         double* ext_packed, const long* ext_off, void* stream) {
    if (!b || !psi_packed || !psi_off || !E_packed || !E_off || !dt || !nsteps)
        return fail(TDSEZ_EINVAL, "NULL argument");
    if (ext & ~(unsigned)TDSEZ_EXT_SERIES) return fail(TDSEZ_EINVAL, "unknown extended-series bits 0x%x", ext);
    if (ext && (!ext_packed || !ext_off)) return fail(TDSEZ_EINVAL, "extended series requested but buffer is NULL");
    if (prec != TDSEZ_FP64 && prec != TDSEZ_FP32_REFINED)
        return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    if (obs & ~7u) return fail(TDSEZ_EINVAL, "unknown observable bits 0x%x", obs);
    if (obs && (!obs_packed || !obs_off)) return fail(TDSEZ_EINVAL, "obs requested but obs buffer is NULL");
    BatchData* d = &b->d;
    const int nsys = (int)d->sys.size();
    for (int s = 0; s < nsys; ++s) {
        if (!(dt[s] > 0.0) || !std::isfinite(dt[s])) return fail(TDSEZ_EINVAL, "dt[%d] must be > 0", s);
        if (nsteps[s] < 0) return fail(TDSEZ_EINVAL, "nsteps[%d] < 0", s);
        if (psi_off[s] < 0 || E_off[s] < 0 || (obs && obs_off[s] < 0) || (ext && ext_off[s] < 0))
            return fail(TDSEZ_EINVAL, "negative offset for system %d", s);
        // eq. pdm_acceleration: with a position-dependent mass the
        // acceleration needs the a_Q term (tdsez_set_aq)
        if ((obs & TDSEZ_OBS_ACCEL) && !d->sys[s]->const_mass && !d->sys[s]->d_Q)
            return fail(TDSEZ_EUNSUPPORTED,
                        "system %d has a position-dependent mass: the acceleration needs its a_Q term "
                        "(tdsez_set_aq before tdsez_batch_create)", s);
        SysDesc& sd = d->desc[s];
        sd.nsteps = nsteps[s];
        sd.dt = dt[s];
        sd.psi_off = psi_off[s];
        sd.E_off = E_off[s];
        sd.obs_off = obs ? obs_off[s] : 0;
        sd.ext_off = ext ? ext_off[s] : 0;
    }
    return launch_propagate(d, psi_packed, E_packed, obs ? obs_packed : nullptr, prec, obs,
                            (hipStream_t)stream, false, ext ? ext_packed : nullptr);
}

tdsez_status tdsez_adjoint_batched(tdsez_batch b, const double* psi0_packed, const long* psi_off,
                                   const double* E_packed, const long* E_off, const double* dt,
                                   const int* nsteps, tdsez_precision prec, unsigned obs,
                                   const double* dJdobs_packed, const long* obs_off, double* dJdE_packed,
                                   double* dJdpsi0_packed, int ckpt_stride, void* stream) {
    if (!b || !psi0_packed || !psi_off || !E_packed || !E_off || !dt || !nsteps || !dJdobs_packed ||
        !obs_off || !dJdE_packed)
        return fail(TDSEZ_EINVAL, "NULL argument");
    if (b->d.any_cap)
        return fail(TDSEZ_EUNSUPPORTED, "the adjoint does not support an absorbing potential");
    for (size_t s = 0; s < b->d.sys.size(); ++s)
        if ((obs & TDSEZ_OBS_ACCEL) && !b->d.sys[s]->const_mass)
            return fail(TDSEZ_EUNSUPPORTED, "adjoint of the acceleration with a position-dependent mass (system %zu)",
                        s);
    if (prec == TDSEZ_FP32_REFINED)
        return fail(TDSEZ_EUNSUPPORTED, "the adjoint runs in FP64 only (use TDSEZ_FP64)");
    if (prec != TDSEZ_FP64) return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    if (obs & ~7u) return fail(TDSEZ_EINVAL, "unknown observable bits 0x%x", obs);
    if (ckpt_stride < 0) return fail(TDSEZ_EINVAL, "ckpt_stride must be >= 0");
    BatchData* d = &b->d;
    const int nsys = (int)d->sys.size();
    for (int s = 0; s < nsys; ++s) {
        if (!(dt[s] > 0.0) || !std::isfinite(dt[s])) return fail(TDSEZ_EINVAL, "dt[%d] must be > 0", s);
        if (nsteps[s] < 0) return fail(TDSEZ_EINVAL, "nsteps[%d] < 0", s);
        if (psi_off[s] < 0 || E_off[s] < 0 || obs_off[s] < 0)
            return fail(TDSEZ_EINVAL, "negative offset for system %d", s);
        SysDesc& sd = d->desc[s];
        sd.nsteps = nsteps[s];
        sd.dt = dt[s];
        sd.psi_off = psi_off[s];
        sd.E_off = E_off[s];
        sd.obs_off = obs_off[s];
    }
    return launch_adjoint(d, psi0_packed, E_packed, dJdobs_packed, obs, dJdE_packed, dJdpsi0_packed, ckpt_stride,
                          (hipStream_t)stream);
}

// The one-system plan of tdsez_propagate: a lone system has the device to
// itself, so up to four waves (multi_wave_plan), or several workgroups for a
// long chain (span_plan).
static tdsez_status ensure_solo(tdsez_system sys) {
    if (sys->d.solo) return TDSEZ_OK;
    tdsez_system one = sys;
    tdsez_status st = tdsez_batch_create(&one, 1, &sys->d.solo);
    if (st) return st;
    sys->d.solo->d.max_waves = 4;
    sys->d.solo->d.solo = true;
    int nsteps_one = 1;
    return tdsez_batch_split(sys->d.solo, &nsteps_one, 1);
}

tdsez_status tdsez_system_set(tdsez_system sys, const char* key, double value) {
    if (!sys || !key) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!std::strcmp(key, "workgroups")) {
        if (!(value >= 0.0 && value <= kMaxSpan) || value != std::floor(value))
            return fail(TDSEZ_EINVAL, "workgroups must be an integer in 0..%d", kMaxSpan);
        sys->d.span_G = (int)value;
    } else if (!std::strcmp(key, "chunks_per_workgroup")) {
        if (!(value == 0.0 || (value >= 2.0 && value <= kMaxChunks4)) || value != std::floor(value))
            return fail(TDSEZ_EINVAL, "chunks_per_workgroup must be 0 or an integer in 2..%d", kMaxChunks4);
        sys->d.span_Pl = (int)value;
    } else {
        return fail(TDSEZ_EINVAL, "unknown key '%s'", key);
    }
    if (sys->d.solo) {
        tdsez_batch_destroy(sys->d.solo);
        sys->d.solo = nullptr;
    }
    return TDSEZ_OK;
}

tdsez_status tdsez_system_workgroups(tdsez_system sys, int* workgroups, int* chunks) {
    if (!sys) return fail(TDSEZ_EINVAL, "sys is NULL");
    if (tdsez_status st = ensure_solo(sys)) return st;
    const BatchData& d = sys->d.solo->d;
    if (workgroups) *workgroups = d.span_G > 1 ? d.span_G : 1;
    if (chunks) *chunks = d.plan.empty() ? 0 : d.plan[0].P;
    return TDSEZ_OK;
}

tdsez_status tdsez_propagate(tdsez_system sys, double* psi, const double* E, double dt, int nsteps,
                             tdsez_precision prec, unsigned obs, double* obs_out, void* stream) {
    return tdsez_propagate_ext(sys, psi, E, dt, nsteps, prec, obs, obs_out, 0u, nullptr, stream);
}

tdsez_status tdsez_propagate_ext(tdsez_system sys, double* psi, const double* E, double dt, int nsteps,
                                 tdsez_precision prec, unsigned obs, double* obs_out, unsigned ext,
                                 double* ext_out, void* stream) {
    if (!sys) return fail(TDSEZ_EINVAL, "sys is NULL");
    if (tdsez_status st = ensure_solo(sys)) return st;
    long zero = 0;
    return tdsez_propagate_batched_ext(sys->d.solo, psi, &zero, E, &zero, &dt, &nsteps, prec, obs, obs_out, &zero,
                                       ext, ext_out, &zero, stream);
}

// Drop the one-system plan (it packs the bands, so it is rebuilt after a
// band of the system changes).
static void drop_solo(tdsez_system sys) {
    if (sys->d.solo) {
        tdsez_batch_destroy(sys->d.solo);
        sys->d.solo = nullptr;
    }
}

static tdsez_status check_samples(const double* a, size_t n, const char* what) {
    if (!a) return TDSEZ_OK;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return fail(TDSEZ_EINVAL, "non-finite %s sample %zu", what, i);
    return TDSEZ_OK;
}

tdsez_status tdsez_set_cap(tdsez_system sys, const double* eta_q) {
    if (!sys) return fail(TDSEZ_EINVAL, "sys is NULL");
    const size_t nqt = (size_t)(sys->d.nbreaks - 1) * sys->d.nq;
    drop_solo(sys);
    if (!eta_q) {
        (void)hipFree(sys->d.d_W);
        sys->d.d_W = nullptr;
        return TDSEZ_OK;
    }
    if (tdsez_status st = check_samples(eta_q, nqt, "eta")) return st;
    for (size_t i = 0; i < nqt; ++i)
        if (eta_q[i] < 0.0) return fail(TDSEZ_EINVAL, "the absorber mask must be >= 0 (sample %zu)", i);
    return assemble_extra_device(&sys->d, 0, eta_q, nullptr);
}

tdsez_status tdsez_set_aq(tdsez_system sys, const double* g_q, const double* h_q) {
    if (!sys) return fail(TDSEZ_EINVAL, "sys is NULL");
    const size_t nqt = (size_t)(sys->d.nbreaks - 1) * sys->d.nq;
    drop_solo(sys);
    if (!g_q && !h_q) {
        (void)hipFree(sys->d.d_Q);
        sys->d.d_Q = nullptr;
        return TDSEZ_OK;
    }
    if (tdsez_status st = check_samples(g_q, nqt, "g")) return st;
    if (tdsez_status st = check_samples(h_q, nqt, "h")) return st;
    return assemble_extra_device(&sys->d, 1, g_q, h_q);
}

tdsez_status tdsez_set_projectors(tdsez_system sys, int npop, const double* phi) {
    if (!sys) return fail(TDSEZ_EINVAL, "sys is NULL");
    if (npop < 0 || npop > kMaxPop) return fail(TDSEZ_EINVAL, "npop must be in 0..%d", kMaxPop);
    if (npop > 0 && !phi) return fail(TDSEZ_EINVAL, "phi is NULL");
    if (tdsez_status st = check_samples(phi, (size_t)npop * sys->d.N, "projection state")) return st;
    drop_solo(sys);
    return set_projectors_device(&sys->d, npop, phi);
}

tdsez_status tdsez_ext_columns(tdsez_system sys, int* ncols) {
    if (!sys || !ncols) return fail(TDSEZ_EINVAL, "NULL argument");
    *ncols = kExtFixed + sys->d.npop;
    return TDSEZ_OK;
}

// Partition autotuner.  The chunk count P of a system trades the lane-serial
// sweeps (about N / P rows each) against the serial separator chain (P
// blocks); the best balance depends on p, N, the precision and on how much
// of the device the rest of the batch occupies.  Each trial re-packs the
// whole batch with one rule for the chunk length, runs a short profiled
// propagation of all systems together (so every trial sees the batch's own
// contention), and every system keeps the chunk count of the trial with the
// fewest shader cycles per step.
tdsez_status tdsez_autotune(tdsez_batch b, tdsez_precision prec, double budget_ms) {
    if (!b) return fail(TDSEZ_EINVAL, "b is NULL");
    if (prec != TDSEZ_FP64 && prec != TDSEZ_FP32_REFINED)
        return fail(TDSEZ_EINVAL, "unknown precision %d", (int)prec);
    if (!(budget_ms > 0.0) || !std::isfinite(budget_ms)) return fail(TDSEZ_EINVAL, "budget_ms must be > 0");
    BatchData* d = &b->d;
    const int nsys = (int)d->sys.size();
    const auto t_start = std::chrono::steady_clock::now();
    auto elapsed_ms = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    };
    // chunk length rules L = sqrt(c N), the default rule (c = 0.6) first
    static const double kRule[] = {0.6, 0.3, 1.2, 0.15, 2.4};
    constexpr int kTrials = sizeof(kRule) / sizeof(kRule[0]);
    constexpr int kWarm = 4, kProbe = 16;
    // (systems that may run on more waves: half the constant, up to 128
    // chunks on two waves, a quarter and up to 256 on four)
    auto chunks_for = [&](int s, double c) {
        const int N = d->sys[s]->N, p = d->sys[s]->p;
        const bool req = s < (int)d->two_wave_req.size() && d->two_wave_req[s];
        const int mw = req ? d->max_waves : 1;
        double L = std::sqrt((mw >= 4 ? 0.25 : mw == 2 ? 0.5 : 1.0) * c * N);
        if (L < 2.0 * p + 2) L = 2.0 * p + 2;
        int P = (int)std::lround(N / L);
        return make_plan(N, p, P < 1 ? 1 : P, mw >= 4 ? kMaxChunks4 : mw == 2 ? kMaxChunks2 : kMaxChunks).P;
    };
    // scratch inputs: a smooth finite state, zero field (the timing does not
    // depend on the values)
    std::vector<long> psi_off(nsys), E_off(nsys), obs_off(nsys);
    long npsi = 0;
    for (int s = 0; s < nsys; ++s) {
        psi_off[s] = npsi;
        npsi += d->sys[s]->N;
        E_off[s] = (long)s * (kProbe + 1);
        obs_off[s] = (long)s * 3 * (kProbe + 1);
    }
    std::vector<double> psi_h(2 * (size_t)npsi, 0.0);
    for (int s = 0; s < nsys; ++s) {
        const int N = d->sys[s]->N;
        for (int j = 0; j < N; ++j) psi_h[2 * (size_t)(psi_off[s] + j)] = std::sin(3.141592653589793 * (j + 1.0) / (N + 1.0));
    }
    double *d_psi = nullptr, *d_E = nullptr, *d_obs = nullptr;
    auto release = [&]() {
        (void)hipFree(d_psi);
        (void)hipFree(d_E);
        (void)hipFree(d_obs);
    };
    if (hipMalloc(&d_psi, sizeof(double) * psi_h.size()) != hipSuccess ||
        hipMalloc(&d_E, sizeof(double) * (size_t)nsys * (kProbe + 1)) != hipSuccess ||
        hipMalloc(&d_obs, sizeof(double) * (size_t)nsys * 3 * (kProbe + 1)) != hipSuccess) {
        release();
        return fail(TDSEZ_ENOMEM, "autotune scratch allocation failed");
    }
    if (hipMemset(d_E, 0, sizeof(double) * (size_t)nsys * (kProbe + 1)) != hipSuccess) {
        release();
        return fail(TDSEZ_EHIP, "hipMemset failed");
    }
    const bool had_prof = d->d_prof != nullptr;
    const double norm_tol = d->norm_tol;
    d->norm_tol = 0.0;
    d->force_chunks = 0;
    std::vector<double> best_cyc(nsys, INFINITY);
    std::vector<int> best_P(nsys, 0);
    std::vector<double> prof(kProfSlots * (size_t)nsys);
    tdsez_status st = TDSEZ_OK;
    for (int t = 0; t < kTrials && st == TDSEZ_OK; ++t) {
        if (t > 0 && elapsed_ms() > budget_ms) break;
        d->tuned_chunks.resize(nsys);
        bool differs = (t == 0);
        for (int s = 0; s < nsys; ++s) {
            const int P = chunks_for(s, kRule[t]);
            differs = differs || (P != best_P[s]);
            d->tuned_chunks[s] = P;
        }
        if (!differs) continue;
        free_batch_device(d);
        if ((st = pack_bands(d)) != TDSEZ_OK) break;
        if ((st = tdsez_batch_set(b, "profile", 1.0)) != TDSEZ_OK) break;
        for (int rep = 0; rep < 2 && st == TDSEZ_OK; ++rep) {
            if (hipMemcpy(d_psi, psi_h.data(), sizeof(double) * psi_h.size(), hipMemcpyHostToDevice) !=
                hipSuccess) {
                st = fail(TDSEZ_EHIP, "hipMemcpy failed");
                break;
            }
            for (int s = 0; s < nsys; ++s) {
                SysDesc& sd = d->desc[s];
                sd.nsteps = rep == 0 ? kWarm : kProbe;
                sd.dt = 0.05;
                sd.psi_off = psi_off[s];
                sd.E_off = E_off[s];
                sd.obs_off = obs_off[s];
            }
            st = launch_propagate(d, d_psi, d_E, d_obs, prec, TDSEZ_OBS_NORM | TDSEZ_OBS_DIPOLE | TDSEZ_OBS_ACCEL,
                                  nullptr, true);
        }
        if (st != TDSEZ_OK) break;
        if ((st = tdsez_batch_profile(b, nullptr, prof.data())) != TDSEZ_OK) break;
        for (int s = 0; s < nsys; ++s) {
            double cyc = 0.0;
            for (int k = 0; k < 8; ++k) cyc += prof[kProfSlots * (size_t)s + k];
            if (cyc < best_cyc[s]) {
                best_cyc[s] = cyc;
                best_P[s] = d->plan[s].P;
            }
        }
    }
    release();
    d->norm_tol = norm_tol;
    if (st == TDSEZ_OK) {
        int sys_fail = 0, step_fail = 0;
        st = tdsez_batch_status(b, nullptr, &sys_fail, &step_fail);
    }
    // keep the winners (or, after a failure, the rule) and re-pack
    if (st == TDSEZ_OK) d->tuned_chunks = best_P;
    else d->tuned_chunks.clear();
    free_batch_device(d);
    tdsez_status st2 = pack_bands(d);
    if (st2 == TDSEZ_OK && had_prof) st2 = tdsez_batch_set(b, "profile", 1.0);
    return st != TDSEZ_OK ? st : st2;
}

tdsez_status tdsez_batch_chunks(tdsez_batch b, int* chunks_out) {
    if (!b || !chunks_out) return fail(TDSEZ_EINVAL, "NULL argument");
    for (size_t s = 0; s < b->d.plan.size(); ++s) chunks_out[s] = b->d.plan[s].P;
    return TDSEZ_OK;
}

tdsez_status tdsez_batch_profile(tdsez_batch b, void* stream, double* out) {
    if (!b || !out) return fail(TDSEZ_EINVAL, "NULL argument");
    if (!b->d.d_prof) return fail(TDSEZ_EINVAL, "profiling is off (tdsez_batch_set(b, \"profile\", 1))");
    TDSEZ_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    const size_t n = b->d.sys.size();
    constexpr int K = kProfSlots;
    std::vector<unsigned long long> h(K * n);
    TDSEZ_HIP_TRY(hipMemcpy(h.data(), b->d.d_prof, sizeof(unsigned long long) * K * n, hipMemcpyDeviceToHost));
    for (size_t s = 0; s < n; ++s) {
        double ns = h[K * s + 8] > 0 ? (double)h[K * s + 8] : 1.0;
        for (int k = 0; k < 8; ++k) out[K * s + k] = (double)h[K * s + k] / ns;
        out[K * s + 8] = (double)b->d.plan[s].P;
        double worst;
        std::memcpy(&worst, &h[K * s + 9], sizeof(double));
        out[K * s + 9] = worst;
    }
    return TDSEZ_OK;
}

tdsez_status tdsez_batch_status(tdsez_batch b, void* stream, int* sys_out, int* step_out) {
    if (!b) return fail(TDSEZ_EINVAL, "b is NULL");
    TDSEZ_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int h[4] = {0, 0, 0, 0};
    TDSEZ_HIP_TRY(hipMemcpy(h, b->d.d_status, sizeof(int) * 4, hipMemcpyDeviceToHost));
    TDSEZ_HIP_TRY(hipMemset(b->d.d_status, 0, sizeof(int) * 4));
    if (sys_out) *sys_out = h[1];
    if (step_out) *step_out = h[2];
    if (h[0] == TDSEZ_ENONFINITE) return fail(TDSEZ_ENONFINITE, "non-finite state in system %d at step %d", h[1], h[2]);
    if (h[0] == TDSEZ_ENORMDRIFT) return fail(TDSEZ_ENORMDRIFT, "norm drift beyond tolerance in system %d at step %d", h[1], h[2]);
    if (h[0] == TDSEZ_ENOCONV)
        return fail(TDSEZ_ENOCONV, "refinement residual above refine_tol in system %d (first at step %d)", h[1], h[2]);
    if (h[0] != 0) return fail((tdsez_status)h[0], "device error %d in system %d at step %d", h[0], h[1], h[2]);
    return TDSEZ_OK;
}

tdsez_status tdsez_system_status(tdsez_system sys, void* stream, int* step_out) {
    if (!sys) return fail(TDSEZ_EINVAL, "sys is NULL");
    if (!sys->d.solo) return TDSEZ_OK;
    return tdsez_batch_status(sys->d.solo, stream, nullptr, step_out);
}

void tdsez_batch_destroy(tdsez_batch b) {
    if (!b) return;
    free_batch_device(&b->d);
    if (b->d.side) (void)hipStreamDestroy(b->d.side);
    if (b->d.side2) (void)hipStreamDestroy(b->d.side2);
    if (b->d.ev_fork) (void)hipEventDestroy(b->d.ev_fork);
    if (b->d.ev_join) (void)hipEventDestroy(b->d.ev_join);
    if (b->d.ev_join2) (void)hipEventDestroy(b->d.ev_join2);
    delete b;
}

tdsez_status tdsez_batch_split(tdsez_batch b, const int* nsteps, int count) {
    if (!b) return fail(TDSEZ_EINVAL, "b is NULL");
    BatchData* d = &b->d;
    const int nsys = (int)d->sys.size();
    if (count == TDSEZ_SPLIT_AUTO) {
        int dev = 0, cus = 0;
        TDSEZ_HIP_TRY(hipGetDevice(&dev));
        TDSEZ_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const int waves = (int)std::floor(1.16 * 4.0 * cus);
        count = std::max(0, std::min(nsys, waves - nsys));
    }
    if (count < 0 || count > nsys) return fail(TDSEZ_EINVAL, "count must be in 0..%d", nsys);
    if (count > 0 && !nsteps) return fail(TDSEZ_EINVAL, "nsteps is NULL");
    for (int s = 0; count > 0 && s < nsys; ++s)
        if (nsteps[s] < 0) return fail(TDSEZ_EINVAL, "nsteps[%d] < 0", s);
    std::vector<int> idx(nsys);
    for (int s = 0; s < nsys; ++s) idx[s] = s;
    auto cost = [&](int s) { return (double)d->sys[s]->N * (d->sys[s]->p + 1) * (double)nsteps[s]; };
    if (count > 0)
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return cost(x) > cost(y); });
    d->two_wave_req.assign(nsys, 0);
    for (int r = 0; r < count; ++r) d->two_wave_req[idx[r]] = 1;
    const bool prof = d->d_prof != nullptr;
    d->tuned_chunks.clear();
    free_batch_device(d);
    tdsez_status st = pack_bands(d);
    if (st == TDSEZ_OK && prof) return tdsez_batch_set(b, "profile", 1.0);
    return st;
}

tdsez_status tdsez_batch_two_wave(tdsez_batch b, int* flags_out) {
    if (!b || !flags_out) return fail(TDSEZ_EINVAL, "NULL argument");
    for (size_t s = 0; s < b->d.sys.size(); ++s)
        flags_out[s] = s < b->d.waves.size() && b->d.waves[s] > 1 ? 1 : 0;
    return TDSEZ_OK;
}

tdsez_status tdsez_batch_waves(tdsez_batch b, int* waves_out) {
    if (!b || !waves_out) return fail(TDSEZ_EINVAL, "NULL argument");
    for (size_t s = 0; s < b->d.sys.size(); ++s) waves_out[s] = s < b->d.waves.size() ? (int)b->d.waves[s] : 1;
    return TDSEZ_OK;
}

void tdsez_system_destroy(tdsez_system sys) {
    if (!sys) return;
    if (sys->d.solo) tdsez_batch_destroy(sys->d.solo);
    for (int m = 0; m < 6; ++m) (void)hipFree(sys->d.d_band[m]);
    (void)hipFree(sys->d.d_H0);
    (void)hipFree(sys->d.d_K);
    (void)hipFree(sys->d.d_W);
    (void)hipFree(sys->d.d_Q);
    (void)hipFree(sys->d.d_pops);
    delete sys;
}

}  // extern "C"
