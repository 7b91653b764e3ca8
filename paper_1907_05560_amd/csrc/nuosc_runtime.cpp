// Host runtime and C ABI of libnuosc (see include/nuosc.h).
//
// The runtime validates a parameter set, builds the per-energy tables in FP64
// (spectra eq 4.1-4.2, vacuum Hamiltonian eq 3.5-3.6), lays each run out in
// one device region, and drives the kernels on a stream.  The step controller
// runs on the device, so stepping needs no host round trip; the host reads a
// run's control block only when a call returns.
//
// A run (RunState) is served either by a handle of its own (nuosc_create) or
// as one slot of a batch (nuosc_batch_create), whose runs share every launch
// and whose device memory comes from one arena with a first-fit allocator.
#include "../../include/nuosc.h"
#include "nuosc_internal.hpp"

#include <algorithm>
#include <mutex>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

using nuosc::Control;
using nuosc::RunConst;

namespace {

thread_local std::string g_create_error;

constexpr double kHbarcEvKm = 1.973269804e-10;       // hbar c = 197.3269804 MeV fm
constexpr double kLumRefErgS = 1e51;                 // reference number luminosity:
constexpr double kEnergyRefMev = 11.0;               //   1e51 erg/s at 11 MeV

// ---------------------------------------------------------------- spectra
// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_m.
void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w)
{
    x.resize(m);
    w.resize(m);
    for (int i = 0; i < m; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = m * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // recompute the derivative at the converged node
                p0 = 1.0; p1 = z;
                for (int k = 2; k <= m; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = m * (z * p1 - p0) / (z * z - 1.0);
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
        }
    }
}

// F_k(eta) = int_0^inf x^k / (e^{x - eta} + 1) dx (eq 4.2) by 16-point
// Gauss-Legendre panels of width 1/4 on [0, max(eta, 0) + 90].
double fermi_integral(int k, double eta)
{
    static std::vector<double> gx, gw;
    if (gx.empty()) gauss_legendre(16, gx, gw);
    const double top = std::max(eta, 0.0) + 90.0;
    const double width = 0.25;
    const int panels = (int)std::ceil(top / width);
    double total = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double a = p * width, half = 0.5 * width;
        double s = 0.0;
        for (size_t i = 0; i < gx.size(); ++i) {
            const double x = a + half * (1.0 + gx[i]);
            s += gw[i] * std::pow(x, k) / (std::exp(x - eta) + 1.0);
        }
        total += half * s;
    }
    return total;
}

// Per-slot tables of one trajectory's 2 NE beam slots (slot k: neutrino of
// bin k; slot NE + k: antineutrino of bin k, whose amplitudes the device holds
// conjugated): signed inverse energy u and density weight.
struct Tables {
    std::vector<double> inv_e, g, gbar;
    std::vector<double> uinv64, wgt;
    std::vector<double> flux;   // number flux of the slot's birth flavor (nu_e or nubar_e) in its bin
    std::vector<float> uinv32;
    double vac[3][3][2];
};

bool build_tables(const nuosc_params& p, Tables& t)
{
    const int ne = p.n_energy, n = p.n_flavors;
    t.inv_e.resize(ne);
    t.g.resize(ne);
    t.gbar.resize(ne);
    t.uinv64.resize(2 * ne);
    t.uinv32.resize(2 * ne);
    t.wgt.resize(2 * ne);
    t.flux.resize(2 * ne);
    double temp[4], f2[4], nrel[4];
    for (int s = 0; s < 4; ++s) {
        f2[s] = fermi_integral(2, p.eta[s]);
        temp[s] = p.mean_e_mev[s] * f2[s] / fermi_integral(3, p.eta[s]);
        nrel[s] = (p.lum_erg_s[s] / kLumRefErgS) * (kEnergyRefMev / p.mean_e_mev[s]);
    }
    auto spectrum = [&](int s, double e) {  // eq 4.1 (denominator exp(E/T - eta) + 1)
        return e * e / (f2[s] * temp[s] * temp[s] * temp[s] * (std::exp(e / temp[s] - p.eta[s]) + 1.0));
    };
    const double de = (p.e_max_mev - p.e_min_mev) / ne;
    for (int k = 0; k < ne; ++k) {
        const double e = p.e_min_mev + (k + 0.5) * de;
        t.inv_e[k] = 1.0 / e;
        // nu_mu and nu_tau share the nu_x spectrum: the flavor sum of eq 3.8 reduces
        // to (n_e - n_x) rho_e up to the identity, which a traceless H drops.
        t.g[k] = de * (nrel[0] * spectrum(0, e) - nrel[2] * spectrum(2, e));
        t.gbar[k] = de * (nrel[1] * spectrum(1, e) - nrel[3] * spectrum(3, e));
        t.flux[k] = de * nrel[0] * spectrum(0, e);
        t.flux[ne + k] = de * nrel[1] * spectrum(1, e);
    }
    // Vacuum Hamiltonian H_vac(E) = vac / E, traceless, in km^-1 (E in MeV).
    const double kappa = 1.0 / (2.0e6 * kHbarcEvKm);
    std::memset(t.vac, 0, sizeof(t.vac));
    if (n == 2) {
        const double d = 0.5 * kappa * p.dm2_ev2;
        t.vac[0][0][0] = -d * std::cos(2 * p.theta);
        t.vac[1][1][0] = d * std::cos(2 * p.theta);
        t.vac[0][1][0] = t.vac[1][0][0] = d * std::sin(2 * p.theta);
    } else {
        using cd = std::complex<double>;
        const double c12 = std::cos(p.theta12), s12 = std::sin(p.theta12);
        const double c13 = std::cos(p.theta13), s13 = std::sin(p.theta13);
        const double c23 = std::cos(p.theta23), s23 = std::sin(p.theta23);
        const cd ed = std::polar(1.0, p.delta_cp);  // e^{i delta}
        // PMNS matrix (PDG parametrisation), rows e, mu, tau.
        const cd U[3][3] = {
            {c12 * c13, s12 * c13, s13 * std::conj(ed)},
            {-s12 * c23 - c12 * s23 * s13 * ed, c12 * c23 - s12 * s23 * s13 * ed, s23 * c13},
            {s12 * s23 - c12 * c23 * s13 * ed, -c12 * s23 - s12 * c23 * s13 * ed, c23 * c13}};
        const double m2[3] = {0.0, kappa * p.dm2_21_ev2, kappa * p.dm2_31_ev2};
        const double shift = (m2[1] + m2[2]) / 3.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                cd v = 0.0;
                for (int i = 0; i < 3; ++i) v += U[a][i] * m2[i] * std::conj(U[b][i]);
                if (a == b) v -= shift;
                t.vac[a][b][0] = v.real();
                t.vac[a][b][1] = v.imag();
            }
    }
    for (int k = 0; k < ne; ++k) {
        t.uinv64[k] = t.inv_e[k];
        t.uinv64[ne + k] = -t.inv_e[k];
        t.wgt[k] = t.g[k];
        t.wgt[ne + k] = -t.gbar[k];
    }
    for (int i = 0; i < 2 * ne; ++i) t.uinv32[i] = (float)t.uinv64[i];
    for (int k = 0; k < ne; ++k)
        if (!std::isfinite(t.g[k]) || !std::isfinite(t.gbar[k]) || !std::isfinite(t.flux[k]) ||
            !std::isfinite(t.flux[ne + k]))
            return false;
    return true;
}

// ---------------------------------------------------------------- layout
struct Layout {
    size_t psi[2], phase[2], uinv64, uinv32, wgt, jhist, partial, errpart, qbuf, dbuf, gbuf, ftab, xbuf, flux, azi,
        geo, zbuf, ctrl, prob, eavg, rconst, total;
    int64_t nb, nb_pad;
    int na, nblk, nblkf, nblkp, pstride;
    int nj;      // angle moments: 2 (bulb model), 4 (extended: azimuth)
    nuosc::PolySizes poly;  // Runge-Kutta per-trajectory tables (zero for the exponential stepper)
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

const char* validate(const nuosc_params* p)
{
    if (!p) return "params is NULL";
    if (p->n_flavors != 2 && p->n_flavors != 3) return "n_flavors must be 2 or 3";
    if (p->n_energy < 1) return "n_energy must be >= 1";
    if (p->n_angle < 0) return "n_angle must be >= 0";
    if (p->n_azimuth < 0) return "n_azimuth must be >= 0";
    if (p->n_azimuth > 1 && p->n_angle < 1) return "azimuth bins need emission-angle bins (n_angle >= 1)";
    if ((int64_t)std::max(p->n_angle, 1) * std::max(p->n_azimuth, 1) > (1 << 24)) return "too many trajectories";
    if (!(p->e_min_mev >= 0.0) || !(p->e_max_mev > p->e_min_mev)) return "need 0 <= e_min < e_max";
    for (int s = 0; s < 4; ++s) {
        if (!(p->mean_e_mev[s] > 0.0)) return "mean energies must be > 0";
        if (!(p->lum_erg_s[s] >= 0.0)) return "luminosities must be >= 0";
        if (!std::isfinite(p->eta[s])) return "eta must be finite";
    }
    if (!(p->r_nu_km > 0.0)) return "r_nu must be > 0";
    if (!(p->r_start_km >= p->r_nu_km)) return "r_start must be >= r_nu";
    if (!(p->r_end_km > p->r_start_km)) return "r_end must be > r_start";
    if (p->integrator != NUOSC_RK4_FIXED && p->integrator != NUOSC_RK_DP54 && p->integrator != NUOSC_EXP_STEPPER)
        return "unknown integrator";
    if (p->integrator == NUOSC_RK4_FIXED && p->n_fixed_steps < 1) return "n_fixed_steps must be >= 1";
    if (p->integrator == NUOSC_EXP_STEPPER) {
        if (p->frame != NUOSC_FRAME_LAB) return "the exponential stepper runs in the lab frame (frame = NUOSC_FRAME_LAB)";
        if (p->precision != NUOSC_FP64) return "the exponential stepper runs in FP64 (precision = NUOSC_FP64)";
        if (p->n_azimuth > 1) return "the exponential stepper runs the bulb model (n_azimuth <= 1)";
    }
    if (p->integrator != NUOSC_RK4_FIXED) {
        if (!(p->rtol > 0.0)) return "rtol must be > 0";
        if (!(p->dr_init_km > 0.0) || !(p->dr_max_km > 0.0)) return "dr_init and dr_max must be > 0";
        if (!(p->safety > 0.0 && p->safety <= 1.0)) return "safety must be in (0, 1]";
    }
    if (p->precision != NUOSC_FP64 && p->precision != NUOSC_FP32_AMP && p->precision != NUOSC_FP32_AMP_FP64_MATH)
        return "unknown precision";
    if (p->frame != NUOSC_FRAME_COROTATING && p->frame != NUOSC_FRAME_LAB) return "unknown frame";
    if (p->max_steps < 0 || p->max_wall_s < 0) return "limits must be >= 0";
    const int64_t na = (int64_t)std::max(p->n_angle, 1) * std::max(p->n_azimuth, 1);
    // each amplitude component array is addressed with 32-bit byte offsets
    const int64_t tsz = p->precision == NUOSC_FP64 ? 8 : 4;
    if ((2 * (int64_t)p->n_energy * na + 64) * tsz >= ((int64_t)1 << 32))
        return "too many beams (one amplitude component must stay below 4 GiB)";
    return nullptr;
}

Layout make_layout(const nuosc_params& p)
{
    Layout L{};
    const int n = p.n_flavors;
    L.na = std::max(p.n_angle, 1) * std::max(p.n_azimuth, 1);
    L.nj = p.n_azimuth > 1 ? 4 : 2;
    L.nb = 2 * (int64_t)p.n_energy * L.na;
    L.nb_pad = (int64_t)align_up((size_t)L.nb, 64);
    const size_t tsz = p.precision == NUOSC_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const bool rk = p.integrator != NUOSC_EXP_STEPPER;
    const int tpb = rk ? nuosc::kTrajPerBlock : nuosc::kExpTrajPerBlock;
    const int tpbf = rk ? nuosc::final_traj_per_block(p.precision) : nuosc::kExpTrajPerBlock;
    L.nblk = (L.na + tpb - 1) / tpb;
    L.nblkf = (L.na + tpbf - 1) / tpbf;
    // the power-moment launch writes its own count of partials (the exponential
    // stepper's launches all use nblk)
    L.nblkp = rk ? (L.na + nuosc::kPowerTrajPerBlock - 1) / nuosc::kPowerTrajPerBlock : L.nblk;
    L.pstride = std::max(L.nblk, L.nblkp);
    L.poly = rk ? nuosc::poly_sizes(n, p.integrator, p.precision) : nuosc::PolySizes{0, 0, 0};
    for (int b = 0; b < 2; ++b) L.psi[b] = take(2 * n * (size_t)L.nb_pad * tsz);
    for (int b = 0; b < 2; ++b) L.phase[b] = take((size_t)L.na * n * 8);
    L.uinv64 = take((size_t)2 * p.n_energy * 8);
    L.uinv32 = take((size_t)2 * p.n_energy * 4);
    L.wgt = take((size_t)2 * p.n_energy * 8);
    L.flux = take((size_t)2 * p.n_energy * 8);
    L.jhist = take((size_t)(nuosc::kMaxStages + 1) * L.nj * n * n * 8);
    L.partial = take((size_t)2 * L.nj * n * n * L.pstride * 8);  // two launches' partials (alternating)
    L.azi = take((size_t)2 * L.na * 8);
    L.geo = take((size_t)4 * L.na * 8);
    L.errpart = take((size_t)std::max(L.nblk, L.nblkf) * 8);
    L.qbuf = take((size_t)L.na * L.poly.qstride * 8);
    L.dbuf = take((size_t)L.na * L.poly.dstride * 8);
    L.gbuf = take(rk ? (size_t)L.na * nuosc::kMaxStages * n * 8 : 0);
    L.zbuf = take(rk ? (size_t)L.na * 8 * 8 : 0);
    L.ftab = take((size_t)L.na * L.poly.fstride);
    L.xbuf = take(p.integrator == NUOSC_EXP_STEPPER ? 2 * 2 * n * (size_t)L.nb_pad * 8 : 0);
    L.ctrl = take(2 * sizeof(Control));
    L.prob = take((size_t)L.nb * 8);
    L.eavg = take((size_t)2 * L.na * n * 8);
    L.rconst = take(sizeof(RunConst));
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- one run
// Host bookkeeping of one run and where its device data lives.
struct RunState {
    nuosc_params p{};
    RunConst rc{};               // host copy of the device constants
    Layout L{};
    int S = 0;
    char* base = nullptr;        // device region of the run (L.total bytes)
    RunConst* runs_dev = nullptr;  // device array the launches index
    int slot = 0;                // index of this run in runs_dev
    double* prob = nullptr;      // device [nb]
    double* eavg = nullptr;      // device [2][na][n]
    Control hctl{};              // host copy of ctrl[1]
};

// A launch list holding one run.
struct OneRun {
    int slot;
    const RunConst* rcp;
    nuosc::RunList list;
    explicit OneRun(const RunState& r) : slot(r.slot), rcp(&r.rc), list{r.runs_dev, 1, &slot, &rcp} {}
};

std::string hip_msg(hipError_t e, const char* what) { return std::string(what) + ": " + hipGetErrorString(e); }

#define HIP_CHECK(call, msg_out)                       \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) {                        \
            (msg_out) = hip_msg(e_, #call);            \
            return NUOSC_E_DEVICE;                     \
        }                                              \
    } while (0)

// The control block between attempts is ctrl[1]; the host writes both copies.
nuosc_status read_control(RunState& r, hipStream_t s, std::string& err)
{
    HIP_CHECK(hipMemcpyAsync(&r.hctl, r.rc.ctrl + 1, sizeof(Control), hipMemcpyDeviceToHost, s), err);
    HIP_CHECK(hipStreamSynchronize(s), err);
    return NUOSC_OK;
}

nuosc_status write_control(RunState& r, hipStream_t s, std::string& err)
{
    const Control two[2] = {r.hctl, r.hctl};
    HIP_CHECK(hipMemcpyAsync(r.rc.ctrl, two, sizeof(two), hipMemcpyHostToDevice, s), err);
    HIP_CHECK(hipStreamSynchronize(s), err);
    return NUOSC_OK;
}

nuosc_status status_of(const Control& c, std::string& err)
{
    switch (c.status) {
    case 0:
    case 1: return NUOSC_OK;
    case -4: err = "step error is not finite"; return NUOSC_E_NONFINITE;
    case -5: err = "adaptive step fell below 1e-14 r"; return NUOSC_E_STEP_UNDERFLOW;
    case -6: err = "max_steps reached"; return NUOSC_E_LIMIT;
    default: err = "corrupt control block"; return NUOSC_E_DEVICE;
    }
}

// Moments of the current state and the tables of stages 0 and 1 of the next
// attempt, for the control block on the device (after initialisation, a new
// state, or a host change of the step).
nuosc_status restart(RunState& r, hipStream_t s, std::string& err)
{
    OneRun one(r);
    if (r.rc.integrator == NUOSC_EXP_STEPPER) {
        HIP_CHECK(nuosc::launch_exp_stage(one.list, 0, s), err);
        return NUOSC_OK;
    }
    HIP_CHECK(nuosc::launch_stage(one.list, 0, s), err);
    return NUOSC_OK;
}

// Lays run r out at device address base (nuosc_footprint_bytes(p) bytes),
// uploads its tables, constants and control block (its constants go to
// runs_dev[slot]) and puts it in its initial state.  Synchronises s.
nuosc_status init_run(RunState& r, const nuosc_params* p, char* base, RunConst* runs_dev, int slot, hipStream_t s,
                      std::string& err)
{
    if (const char* why = validate(p)) {
        err = why;
        return NUOSC_E_INVALID;
    }
    Tables tab;
    if (!build_tables(*p, tab)) {
        err = "spectral tables are not finite";
        return NUOSC_E_INVALID;
    }
    r.p = *p;
    r.L = make_layout(*p);
    r.S = p->integrator == NUOSC_EXP_STEPPER ? nuosc::kExpLaunches : nuosc::num_stages(p->integrator);
    r.base = base;
    r.runs_dev = runs_dev;
    r.slot = slot;
    const Layout& L = r.L;
    RunConst& rc = r.rc;
    rc = RunConst{};
    rc.n = p->n_flavors;
    rc.ne = p->n_energy;
    rc.na = L.na;
    rc.ma = p->n_angle > 0;
    rc.nb = L.nb;
    rc.nb_pad = L.nb_pad;
    rc.nblk = L.nblk;
    rc.nblkf = L.nblkf;
    rc.nblkp = L.nblkp;
    rc.pstride = L.pstride;
    rc.qstride = L.poly.qstride;
    rc.dstride = L.poly.dstride;
    rc.fstride = L.poly.fstride;
    rc.np = std::max(p->n_azimuth, 1);
    rc.nth = L.na / rc.np;
    rc.nj = L.nj;
    rc.frame = p->frame;
    rc.precision = p->precision;
    rc.integrator = p->integrator;
    rc.r_nu = p->r_nu_km;
    rc.mu0 = p->mu0_km;
    rc.lambda0 = p->lambda0_km;
    rc.lambda_rref = p->lambda_rref_km;
    rc.lambda_power = p->lambda_power;
    rc.rtol = p->rtol;
    rc.safety = p->safety;
    rc.dr_max = p->dr_max_km;
    rc.r_start = p->r_start_km;
    rc.n_fixed = p->n_fixed_steps;
    rc.h_fixed = p->integrator == NUOSC_RK4_FIXED ? (p->r_end_km - p->r_start_km) / (double)p->n_fixed_steps : 0.0;
    rc.max_steps = p->max_steps;
    std::memcpy(rc.vac, tab.vac, sizeof(rc.vac));
    for (int b = 0; b < 2; ++b) {
        rc.psi[b] = base + L.psi[b];
        rc.phase[b] = (double*)(base + L.phase[b]);
    }
    rc.uinv64 = (const double*)(base + L.uinv64);
    rc.uinv32 = (const float*)(base + L.uinv32);
    rc.wgt = (const double*)(base + L.wgt);
    rc.flux = (const double*)(base + L.flux);
    rc.azi = (const double*)(base + L.azi);
    rc.geo = (const double*)(base + L.geo);
    rc.jhist = (double*)(base + L.jhist);
    rc.partial = (double*)(base + L.partial);
    rc.errpart = (double*)(base + L.errpart);
    rc.qbuf = (double*)(base + L.qbuf);
    rc.dbuf = (double*)(base + L.dbuf);
    rc.gbuf = (double*)(base + L.gbuf);
    rc.zbuf = (double*)(base + L.zbuf);
    rc.ftab = (void*)(base + L.ftab);
    rc.xbuf = (double*)(base + L.xbuf);
    rc.ctrl = (Control*)(base + L.ctrl);
    r.prob = (double*)(base + L.prob);
    r.eavg = (double*)(base + L.eavg);

    Control& c = r.hctl;
    std::memset(&c, 0, sizeof(c));
    c.r = p->r_start_km;
    c.r_end = p->r_end_km;
    if (p->integrator == NUOSC_RK4_FIXED) {
        c.h = c.h_prop = rc.h_fixed;
    } else {
        c.h_prop = std::min(p->dr_init_km, p->dr_max_km);
        c.h = std::min(c.h_prop, p->r_end_km - p->r_start_km);
    }
    const Control two[2] = {c, c};
    HIP_CHECK(hipMemcpyAsync((void*)rc.uinv64, tab.uinv64.data(), tab.uinv64.size() * 8, hipMemcpyHostToDevice, s), err);
    HIP_CHECK(hipMemcpyAsync((void*)rc.uinv32, tab.uinv32.data(), tab.uinv32.size() * 4, hipMemcpyHostToDevice, s), err);
    HIP_CHECK(hipMemcpyAsync((void*)rc.wgt, tab.wgt.data(), tab.wgt.size() * 8, hipMemcpyHostToDevice, s), err);
    HIP_CHECK(hipMemcpyAsync((void*)rc.flux, tab.flux.data(), tab.flux.size() * 8, hipMemcpyHostToDevice, s), err);
    // azimuth of every trajectory (extended model: midpoints of [0, 2 pi)): cos, sin
    std::vector<double> azi((size_t)2 * rc.na, 0.0);
    for (int j = 0; j < rc.na; ++j) {
        const double phi = rc.np > 1 ? 2.0 * M_PI * ((j % rc.np) + 0.5) / rc.np : 0.0;
        azi[2 * j] = std::cos(phi);
        azi[2 * j + 1] = std::sin(phi);
    }
    HIP_CHECK(hipMemcpyAsync((void*)rc.azi, azi.data(), azi.size() * 8, hipMemcpyHostToDevice, s), err);
    // per-trajectory constants of the multi-angle geometry (eq 3.14-3.15):
    // trajectory j in emission-angle bin j / np, cosine u at the bin's midpoint
    std::vector<double> geo((size_t)4 * rc.na, 0.0);
    if (rc.ma) {
        const double du = 1.0 / (double)rc.nth;
        for (int j = 0; j < rc.na; ++j) {
            const double u = ((double)(j / rc.np) + 0.5) * du;
            geo[4 * j] = u * u;
            geo[4 * j + 1] = 1.0 - u * u;
            geo[4 * j + 2] = u * du / (double)rc.np;
        }
    }
    HIP_CHECK(hipMemcpyAsync((void*)rc.geo, geo.data(), geo.size() * 8, hipMemcpyHostToDevice, s), err);
    HIP_CHECK(hipMemsetAsync(rc.jhist, 0, (size_t)(nuosc::kMaxStages + 1) * rc.nj * rc.n * rc.n * 8, s), err);
    HIP_CHECK(hipMemcpyAsync(rc.ctrl, two, sizeof(two), hipMemcpyHostToDevice, s), err);
    HIP_CHECK(hipMemcpyAsync(runs_dev + slot, &rc, sizeof(RunConst), hipMemcpyHostToDevice, s), err);
    OneRun one(r);
    HIP_CHECK(nuosc::launch_init_state(one.list, s), err);
    nuosc_status st = restart(r, s, err);
    if (st != NUOSC_OK) return st;
    HIP_CHECK(hipStreamSynchronize(s), err);
    return NUOSC_OK;
}

// Host state <-> device state: the device holds antineutrino amplitudes
// (beams NE*NA .. NB-1) complex-conjugated; psi is [2n][nb] (re/im rows).
void conjugate_antineutrinos(const RunConst& rc, double* psi)
{
    const int64_t half = rc.nb / 2;
    for (int a = 0; a < rc.n; ++a) {
        double* im = psi + (size_t)(2 * a + 1) * rc.nb;
        for (int64_t b = half; b < rc.nb; ++b) im[b] = -im[b];
    }
}

nuosc_status probabilities_of(RunState& r, double* p_out, hipStream_t s, std::string& err)
{
    OneRun one(r);
    HIP_CHECK(nuosc::launch_probabilities(one.list, r.prob, s), err);
    HIP_CHECK(hipMemcpyAsync(p_out, r.prob, (size_t)r.rc.nb * 8, hipMemcpyDeviceToHost, s), err);
    HIP_CHECK(hipStreamSynchronize(s), err);
    return NUOSC_OK;
}

}  // namespace

// ---------------------------------------------------------------- handles
struct nuosc_handle {
    RunState run;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* ws = nullptr;
    bool own_ws = false;
    size_t ws_bytes = 0;
    std::string err;
    // kernel timing: a pool of event triples, the stage of each used triple,
    // and per-stage sums of the harvested durations
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_stage;
    size_t ev_used = 0;
    double t_beam[nuosc::kMaxLaunches + 1] = {};
    double t_fin[nuosc::kMaxLaunches + 1] = {};
    int64_t t_count[nuosc::kMaxLaunches + 1] = {};
    // runs made by nuosc_create_static: the handle is a per-device slot and its
    // device memory the library's static array of that device
    bool is_static = false;
    int device = -1;
    // kGraphAttempts attempts of the run, captured on first use by the
    // synchronous step calls (the run's constants are fixed at creation)
    hipGraphExec_t graph = nullptr;
};

namespace {

static_assert(nuosc::kStaticScratchBytes == NUOSC_STATIC_SCRATCH_BYTES, "static scratch size");

// One handle slot per device for the static runs, and whether it is taken.
std::mutex g_static_mu;
nuosc_handle g_static_handle[nuosc::kMaxDevices];
bool g_static_busy[nuosc::kMaxDevices] = {};

nuosc_status fail(nuosc_handle* h, nuosc_status st, const std::string& msg)
{
    if (h) h->err = msg;
    else g_create_error = msg;
    return st;
}

nuosc_status checked(nuosc_handle* h, nuosc_status st, const std::string& msg)
{
    if (st != NUOSC_OK) h->err = msg;
    return st;
}

// Harvest every recorded event triple into the per-stage sums.
nuosc_status harvest_timing(nuosc_handle* h)
{
    if (h->ev_used == 0) return NUOSC_OK;
    std::string& err = h->err;
    HIP_CHECK(hipStreamSynchronize(h->stream), err);
    for (size_t i = 0; i < h->ev_used; ++i) {
        float a = 0.f, b = 0.f;
        HIP_CHECK(hipEventElapsedTime(&a, h->ev[3 * i], h->ev[3 * i + 1]), err);
        HIP_CHECK(hipEventElapsedTime(&b, h->ev[3 * i + 1], h->ev[3 * i + 2]), err);
        const int st = h->ev_stage[i];
        h->t_beam[st] += a;
        h->t_fin[st] += b;
        h->t_count[st] += 1;
    }
    h->ev_used = 0;
    return NUOSC_OK;
}

// One stage launch of the handle's run, timed when enabled.
nuosc_status stage(nuosc_handle* h, int st)
{
    hipEvent_t* ev = nullptr;
    if (h->timing) {
        if (h->ev_used * 3 == h->ev.size()) {
            nuosc_status s = harvest_timing(h);
            if (s != NUOSC_OK) return s;
        }
        ev = &h->ev[3 * h->ev_used];
        h->ev_stage[h->ev_used] = st;
        h->ev_used += 1;
    }
    OneRun one(h->run);
    if (h->run.rc.integrator == NUOSC_EXP_STEPPER)
        HIP_CHECK(nuosc::launch_exp_stage(one.list, st, h->stream, ev), h->err);
    else
        HIP_CHECK(nuosc::launch_stage(one.list, st, h->stream, ev), h->err);
    return NUOSC_OK;
}

nuosc_status enqueue(nuosc_handle* h, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        for (int st = 1; st <= h->run.S; ++st) {
            nuosc_status s = stage(h, st);
            if (s != NUOSC_OK) return s;
        }
    return NUOSC_OK;
}

// Attempts of the synchronous step calls: replays of a graph of
// kGraphAttempts attempts (one launch call instead of S + 2 per attempt, which
// bounds small runs), the rest launched directly.  Direct launches throughout
// while timing (events around each launch), for handles in the library's
// static memory (nothing is instantiated on their behalf) and on a stream that
// cannot be captured.
constexpr int64_t kGraphAttempts = 32;

nuosc_status enqueue_sync(nuosc_handle* h, int64_t n)
{
    if (h->timing || h->is_static || n < kGraphAttempts) return enqueue(h, n);
    if (!h->graph) {
        if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();  // (the null stream, for one, cannot be captured)
            return enqueue(h, n);
        }
        const nuosc_status s = enqueue(h, kGraphAttempts);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(h->stream, &g);
        if (s != NUOSC_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return s != NUOSC_OK ? s : fail(h, NUOSC_E_DEVICE, hip_msg(e, "capture of the attempts"));
        }
        hipGraphExec_t x = nullptr;
        const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return fail(h, NUOSC_E_DEVICE, hip_msg(ei, "hipGraphInstantiate"));
        h->graph = x;
    }
    int64_t i = 0;
    for (; i + kGraphAttempts <= n; i += kGraphAttempts) HIP_CHECK(hipGraphLaunch(h->graph, h->stream), h->err);
    return enqueue(h, n - i);
}

nuosc_status hread(nuosc_handle* h) { return read_control(h->run, h->stream, h->err); }
nuosc_status hwrite(nuosc_handle* h) { return write_control(h->run, h->stream, h->err); }
nuosc_status hstatus(nuosc_handle* h) { return checked(h, status_of(h->run.hctl, h->err), h->err); }

}  // namespace

extern "C" {

void nuosc_default_params(nuosc_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->n_flavors = 2;
    p->n_energy = 100;
    p->e_min_mev = 1.0;
    p->e_max_mev = 60.0;
    p->n_angle = 0;
    for (int s = 0; s < 4; ++s) { p->lum_erg_s[s] = 1e51; p->eta[s] = 0.0; }
    p->mean_e_mev[0] = 11.0; p->mean_e_mev[1] = 16.0; p->mean_e_mev[2] = 25.0; p->mean_e_mev[3] = 25.0;
    p->dm2_ev2 = -2.4e-3; p->theta = 0.1;
    p->dm2_21_ev2 = 7.5e-5; p->dm2_31_ev2 = -2.4e-3;
    p->theta12 = 0.59; p->theta13 = 0.15; p->theta23 = M_PI / 4; p->delta_cp = 0.0;
    p->lambda0_km = 1e4; p->lambda_rref_km = 10.0; p->lambda_power = 3.0;
    p->mu0_km = 1e5; p->r_nu_km = 10.0; p->r_start_km = 10.0; p->r_end_km = 250.0;
    p->integrator = NUOSC_RK4_FIXED; p->n_fixed_steps = 10000;
    p->rtol = 1e-9; p->dr_init_km = 1e-5; p->dr_max_km = 1.0; p->safety = 0.9;
    p->precision = NUOSC_FP64; p->frame = NUOSC_FRAME_COROTATING;
    p->n_azimuth = 0;
}

size_t nuosc_footprint_bytes(const nuosc_params* p)
{
    if (validate(p)) return 0;
    return make_layout(*p).total;
}

nuosc_status nuosc_create(const nuosc_params* p, void* hip_stream, void* device_workspace,
                          size_t workspace_bytes, nuosc_handle** out)
{
    if (!out) return fail(nullptr, NUOSC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (const char* why = validate(p)) return fail(nullptr, NUOSC_E_INVALID, why);
    const Layout L = make_layout(*p);
    if (device_workspace && workspace_bytes < L.total)
        return fail(nullptr, NUOSC_E_INVALID, "workspace smaller than nuosc_footprint_bytes");

    nuosc_handle* h = new (std::nothrow) nuosc_handle();
    if (!h) return fail(nullptr, NUOSC_E_NOMEM, "host allocation failed");
    auto bail = [&](nuosc_status st, const std::string& msg) {
        g_create_error = msg;
        nuosc_destroy(h);
        return st;
    };
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(NUOSC_E_DEVICE, hip_msg(e, "hipStreamCreate"));
        h->own_stream = true;
    }
    if (device_workspace) {
        h->ws = device_workspace;
        h->ws_bytes = workspace_bytes;
    } else {
        hipError_t e = hipMalloc(&h->ws, L.total);
        if (e != hipSuccess) return bail(NUOSC_E_NOMEM, hip_msg(e, "hipMalloc"));
        h->own_ws = true;
        h->ws_bytes = L.total;
    }
    char* base = (char*)h->ws;
    std::string err;
    nuosc_status st = init_run(h->run, p, base, (RunConst*)(base + L.rconst), 0, h->stream, err);
    if (st != NUOSC_OK) return bail(st, "initialisation: " + err);
    *out = h;
    return NUOSC_OK;
}

nuosc_status nuosc_create_static(const nuosc_params* p, void* hip_stream, nuosc_handle** out)
{
    if (!out) return fail(nullptr, NUOSC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (const char* why = validate(p)) return fail(nullptr, NUOSC_E_INVALID, why);
    const Layout L = make_layout(*p);
    if (L.total > NUOSC_STATIC_SCRATCH_BYTES)
        return fail(nullptr, NUOSC_E_INVALID,
                    "the run needs " + std::to_string(L.total) + " bytes of device memory, more than the " +
                        std::to_string(NUOSC_STATIC_SCRATCH_BYTES) + " bytes of the static scratch");
    int dev = -1;
    void* base = nullptr;
    hipError_t e = nuosc::static_scratch(&dev, &base);
    if (e != hipSuccess) return fail(nullptr, NUOSC_E_DEVICE, hip_msg(e, "address of the static scratch"));
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_busy[dev])
        return fail(nullptr, NUOSC_E_BUSY, "the static scratch of device " + std::to_string(dev) + " holds a live run");
    nuosc_handle* h = &g_static_handle[dev];
    *h = nuosc_handle();
    h->is_static = true;
    h->device = dev;
    h->stream = (hipStream_t)hip_stream;
    h->ws = base;
    h->ws_bytes = NUOSC_STATIC_SCRATCH_BYTES;
    std::string err;
    nuosc_status st = init_run(h->run, p, (char*)base, (RunConst*)((char*)base + L.rconst), 0, h->stream, err);
    if (st != NUOSC_OK) {
        *h = nuosc_handle();
        h->is_static = true;
        return fail(nullptr, st, "initialisation: " + err);
    }
    g_static_busy[dev] = true;
    *out = h;
    return NUOSC_OK;
}

nuosc_status nuosc_enqueue_steps(nuosc_handle* h, int64_t n_attempts)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    if (n_attempts < 0) return fail(h, NUOSC_E_INVALID, "n_attempts must be >= 0");
    return enqueue(h, n_attempts);
}

nuosc_status nuosc_enqueue_stage(nuosc_handle* h, int32_t stage)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    if (stage < 1 || stage > h->run.S) return fail(h, NUOSC_E_INVALID, "stage out of range");
    return ::stage(h, stage);
}

nuosc_status nuosc_timing_enable(nuosc_handle* h, int32_t on)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    HIP_CHECK(hipStreamSynchronize(h->stream), h->err);
    if (on && h->ev.empty()) {
        const size_t triples = 512;
        h->ev.resize(3 * triples, nullptr);
        h->ev_stage.resize(triples, 0);
        for (auto& x : h->ev) HIP_CHECK(hipEventCreate(&x), h->err);
    }
    h->timing = on != 0;
    h->ev_used = 0;
    for (int i = 0; i <= nuosc::kMaxLaunches; ++i) {
        h->t_beam[i] = h->t_fin[i] = 0.0;
        h->t_count[i] = 0;
    }
    return NUOSC_OK;
}

nuosc_status nuosc_timing_read(nuosc_handle* h, double* beam_ms, double* fin_ms, int64_t* count)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    nuosc_status st = harvest_timing(h);
    if (st != NUOSC_OK) return st;
    for (int i = 0; i <= h->run.S; ++i) {
        if (beam_ms) beam_ms[i] = h->t_beam[i];
        if (fin_ms) fin_ms[i] = h->t_fin[i];
        if (count) count[i] = h->t_count[i];
        h->t_beam[i] = h->t_fin[i] = 0.0;
        h->t_count[i] = 0;
    }
    return NUOSC_OK;
}

int32_t nuosc_num_stages(const nuosc_handle* h) { return h ? h->run.S : 0; }

nuosc_status nuosc_step(nuosc_handle* h, int64_t n_attempts, int64_t* n_accepted)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    if (n_attempts < 0) return fail(h, NUOSC_E_INVALID, "n_attempts must be >= 0");
    nuosc_status st = hread(h);
    if (st != NUOSC_OK) return st;
    const int64_t before = h->run.hctl.nacc;
    st = enqueue_sync(h, n_attempts);
    if (st != NUOSC_OK) return st;
    st = hread(h);
    if (st != NUOSC_OK) return st;
    if (n_accepted) *n_accepted = h->run.hctl.nacc - before;
    return hstatus(h);
}

nuosc_status nuosc_evolve(nuosc_handle* h, double r_target_km)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    nuosc_status st = hread(h);
    if (st != NUOSC_OK) return st;
    Control& c = h->run.hctl;
    if (c.status < 0) return hstatus(h);
    const double target = std::min(r_target_km, h->run.p.r_end_km);
    if (c.r >= target) return NUOSC_OK;
    // resume towards the new target
    c.r_end = target;
    c.status = 0;
    if (h->run.p.integrator != NUOSC_RK4_FIXED) c.h = std::min(c.h_prop, target - c.r);
    st = hwrite(h);
    if (st != NUOSC_OK) return st;
    st = checked(h, restart(h->run, h->stream, h->err), h->err);  // stage tables for the (possibly clipped) step
    if (st != NUOSC_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    int64_t batch = 8;
    for (;;) {
        st = enqueue_sync(h, batch);
        if (st != NUOSC_OK) return st;
        st = hread(h);
        if (st != NUOSC_OK) return st;
        if (c.status != 0) break;
        if (h->run.p.max_wall_s > 0) {
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el > h->run.p.max_wall_s) return fail(h, NUOSC_E_LIMIT, "max_wall_s reached");
        }
        batch = std::min<int64_t>(batch * 2, 2048);
    }
    return hstatus(h);
}

// Angle moments first, first + 1 of the current state (0, 1: J0, J1; 2, 3:
// the extended model's J2, J3, zero for the bulb model) as full complex
// matrices.
static nuosc_status moments_pair(nuosc_handle* h, int first, double* ja, double* jb, double* r_km)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    nuosc_status st = checked(h, restart(h->run, h->stream, h->err), h->err);
    if (st != NUOSC_OK) return st;
    const int n = h->run.rc.n, nm = n * n, nj = h->run.rc.nj;
    std::vector<double> J(4 * nm, 0.0);
    HIP_CHECK(hipMemcpyAsync(J.data(), h->run.rc.jhist, (size_t)nj * nm * 8, hipMemcpyDeviceToHost, h->stream),
              h->err);
    st = hread(h);
    if (st != NUOSC_OK) return st;
    for (int m = 0; m < 2; ++m) {
        double* out = m == 0 ? ja : jb;
        if (!out) continue;
        const double* src = J.data() + (first + m) * nm;
        for (int a = 0; a < n; ++a) {
            out[(a * n + a) * 2] = src[a];
            out[(a * n + a) * 2 + 1] = 0.0;
        }
        int u = 0;
        for (int a = 0; a < n; ++a)
            for (int b = a + 1; b < n; ++b, ++u) {
                const double re = src[n + 2 * u], im = src[n + 2 * u + 1];
                out[(a * n + b) * 2] = re;
                out[(a * n + b) * 2 + 1] = im;
                out[(b * n + a) * 2] = re;
                out[(b * n + a) * 2 + 1] = -im;
            }
    }
    if (r_km) *r_km = h->run.hctl.r;
    return NUOSC_OK;
}

nuosc_status nuosc_moments(nuosc_handle* h, double* j0, double* j1, double* r_km)
{
    return moments_pair(h, 0, j0, j1, r_km);
}

nuosc_status nuosc_moments_azimuth(nuosc_handle* h, double* j2, double* j3)
{
    return moments_pair(h, 2, j2, j3, nullptr);
}

nuosc_status nuosc_probabilities(nuosc_handle* h, double* p_out)
{
    if (!h || !p_out) return fail(h, NUOSC_E_INVALID, "NULL argument");
    return checked(h, probabilities_of(h->run, p_out, h->stream, h->err), h->err);
}

nuosc_status nuosc_energy_average(nuosc_handle* h, double* out)
{
    if (!h || !out) return fail(h, NUOSC_E_INVALID, "NULL argument");
    RunState& r = h->run;
    OneRun one(r);
    HIP_CHECK(nuosc::launch_energy_average(one.list, r.eavg, h->stream), h->err);
    HIP_CHECK(hipMemcpyAsync(out, r.eavg, (size_t)2 * r.rc.na * r.rc.n * 8, hipMemcpyDeviceToHost, h->stream),
              h->err);
    HIP_CHECK(hipStreamSynchronize(h->stream), h->err);
    return NUOSC_OK;
}

nuosc_status nuosc_enqueue_energy_average(nuosc_handle* h, double* out_device)
{
    if (!h || !out_device) return fail(h, NUOSC_E_INVALID, "NULL argument");
    OneRun one(h->run);
    HIP_CHECK(nuosc::launch_energy_average(one.list, out_device, h->stream), h->err);
    return NUOSC_OK;
}

nuosc_status nuosc_get_state(nuosc_handle* h, double* psi, double* phase)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    nuosc_status st = hread(h);
    if (st != NUOSC_OK) return st;
    const RunConst& rc = h->run.rc;
    const int cur = h->run.hctl.cur;
    const size_t rows = 2 * (size_t)rc.n;
    if (psi) {
        if (rc.precision == NUOSC_FP64) {
            HIP_CHECK(hipMemcpy2DAsync(psi, rc.nb * 8, rc.psi[cur], rc.nb_pad * 8, rc.nb * 8, rows,
                                       hipMemcpyDeviceToHost, h->stream), h->err);
            HIP_CHECK(hipStreamSynchronize(h->stream), h->err);
        } else {
            std::vector<float> tmp(rows * rc.nb);
            HIP_CHECK(hipMemcpy2DAsync(tmp.data(), rc.nb * 4, rc.psi[cur], rc.nb_pad * 4, rc.nb * 4, rows,
                                       hipMemcpyDeviceToHost, h->stream), h->err);
            HIP_CHECK(hipStreamSynchronize(h->stream), h->err);
            for (size_t i = 0; i < tmp.size(); ++i) psi[i] = tmp[i];
        }
        conjugate_antineutrinos(rc, psi);
    }
    if (phase)
        HIP_CHECK(hipMemcpyAsync(phase, rc.phase[cur], (size_t)rc.na * rc.n * 8, hipMemcpyDeviceToHost, h->stream),
                  h->err);
    HIP_CHECK(hipStreamSynchronize(h->stream), h->err);
    return NUOSC_OK;
}

nuosc_status nuosc_set_state(nuosc_handle* h, const double* psi, const double* phase, double r_km, double dr_km)
{
    if (!h || !psi) return fail(h, NUOSC_E_INVALID, "NULL argument");
    const nuosc_params& P = h->run.p;
    if (!(r_km >= P.r_nu_km) || !(r_km <= P.r_end_km)) return fail(h, NUOSC_E_INVALID, "radius out of range");
    nuosc_status st = hread(h);
    if (st != NUOSC_OK) return st;
    const RunConst& rc = h->run.rc;
    const int cur = h->run.hctl.cur;
    const size_t rows = 2 * (size_t)rc.n;
    std::vector<double> dev(psi, psi + rows * rc.nb);
    conjugate_antineutrinos(rc, dev.data());
    if (rc.precision == NUOSC_FP64) {
        HIP_CHECK(hipMemcpy2DAsync(rc.psi[cur], rc.nb_pad * 8, dev.data(), rc.nb * 8, rc.nb * 8, rows,
                                   hipMemcpyHostToDevice, h->stream), h->err);
        HIP_CHECK(hipStreamSynchronize(h->stream), h->err);
    } else {
        std::vector<float> tmp(rows * rc.nb);
        for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (float)dev[i];
        HIP_CHECK(hipMemcpy2DAsync(rc.psi[cur], rc.nb_pad * 4, tmp.data(), rc.nb * 4, rc.nb * 4, rows,
                                   hipMemcpyHostToDevice, h->stream), h->err);
        HIP_CHECK(hipStreamSynchronize(h->stream), h->err);
    }
    std::vector<double> ph((size_t)rc.na * rc.n, 0.0);
    if (phase) std::memcpy(ph.data(), phase, ph.size() * 8);
    HIP_CHECK(hipMemcpyAsync(rc.phase[cur], ph.data(), ph.size() * 8, hipMemcpyHostToDevice, h->stream), h->err);
    Control& c = h->run.hctl;
    c.nacc = c.nrej = c.attempts = 0;
    c.status = 0;
    c.last_rejected = 0;
    c.r_end = P.r_end_km;
    if (P.integrator == NUOSC_RK4_FIXED) {
        c.istep = (int64_t)std::llround((r_km - rc.r_start) / rc.h_fixed);
        c.r = rc.r_start + (double)c.istep * rc.h_fixed;
        c.h = c.h_prop = rc.h_fixed;
        if (c.istep >= rc.n_fixed) c.status = 1;
    } else {
        c.r = r_km;
        const double d = dr_km > 0 ? dr_km : P.dr_init_km;
        c.h_prop = std::min(d, P.dr_max_km);
        c.h = std::min(c.h_prop, P.r_end_km - r_km);
        if (c.r >= P.r_end_km) c.status = 1;
    }
    st = hwrite(h);
    if (st != NUOSC_OK) return st;
    st = checked(h, restart(h->run, h->stream, h->err), h->err);
    if (st != NUOSC_OK) return st;
    HIP_CHECK(hipStreamSynchronize(h->stream), h->err);
    return NUOSC_OK;
}

// ---------------------------------------------------------------- snapshots
// File layout (little-endian): the 8-byte tag, the header below, psi
// [n][2][nb] and phase [na][n] as FP64 in the host state layout, then a
// 64-bit FNV-1a hash of everything before it.
namespace {
constexpr char kSnapTag[8] = {'N', 'U', 'O', 'S', 'C', 'S', 'N', '1'};

uint64_t fnv1a(const void* data, size_t bytes, uint64_t h)
{
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < bytes; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}
constexpr uint64_t kFnvBasis = 14695981039346656037ull;

bool read_exact(std::FILE* f, void* dst, size_t bytes, uint64_t& hash)
{
    if (std::fread(dst, 1, bytes, f) != bytes) return false;
    hash = fnv1a(dst, bytes, hash);
    return true;
}

// Reads and checks the tag and header; on success the file is positioned at
// psi and hash covers everything read.
const char* read_snapshot_header(std::FILE* f, nuosc_snapshot_header& info, uint64_t& hash)
{
    char tag[8];
    hash = kFnvBasis;
    if (!read_exact(f, tag, sizeof(tag), hash) || std::memcmp(tag, kSnapTag, sizeof(tag)) != 0)
        return "not a snapshot file";
    if (!read_exact(f, &info, sizeof(info), hash)) return "truncated snapshot header";
    if ((info.n_flavors != 2 && info.n_flavors != 3) || info.n_energy < 1 || info.n_angle < 0 ||
        info.n_beams != 2 * (int64_t)info.n_energy * std::max(info.n_angle, 1) || info.n_beams > ((int64_t)1 << 40) ||
        (info.last_rejected != 0 && info.last_rejected != 1) || info.reserved != 0)
        return "inconsistent snapshot header";
    return nullptr;
}
}  // namespace

nuosc_status nuosc_snapshot_info(const char* path, nuosc_snapshot_header* info)
{
    if (!path || !info) return fail(nullptr, NUOSC_E_INVALID, "NULL argument");
    std::FILE* f = std::fopen(path, "rb");
    if (!f) return fail(nullptr, NUOSC_E_INVALID, std::string("cannot open ") + path);
    uint64_t hash;
    nuosc_snapshot_header hdr{};
    const char* e = read_snapshot_header(f, hdr, hash);
    if (!e) {
        // payload and hash
        const int64_t na = std::max(hdr.n_angle, 1);
        const size_t values = (size_t)hdr.n_flavors * 2 * hdr.n_beams + (size_t)na * hdr.n_flavors;
        std::vector<double> buf(1 << 16);
        size_t left = values;
        while (left && !e) {
            const size_t k = std::min(left, buf.size());
            if (!read_exact(f, buf.data(), k * 8, hash)) e = "truncated snapshot payload";
            left -= k;
        }
        uint64_t stored = 0;
        if (!e && std::fread(&stored, 8, 1, f) != 1) e = "truncated snapshot payload";
        if (!e && stored != hash) e = "snapshot checksum mismatch";
    }
    std::fclose(f);
    if (e) return fail(nullptr, NUOSC_E_INVALID, e);
    *info = hdr;
    return NUOSC_OK;
}

nuosc_status nuosc_snapshot_write(nuosc_handle* h, const char* path)
{
    if (!h || !path) return fail(h, NUOSC_E_INVALID, "NULL argument");
    const RunConst& rc = h->run.rc;
    const nuosc_params& P = h->run.p;
    std::vector<double> psi((size_t)rc.n * 2 * rc.nb), phase((size_t)rc.na * rc.n);
    nuosc_status st = nuosc_get_state(h, psi.data(), phase.data());
    if (st != NUOSC_OK) return st;
    const Control& c = h->run.hctl;
    nuosc_snapshot_header info{};
    info.n_flavors = rc.n;
    info.n_energy = rc.ne;
    info.n_angle = P.n_angle;
    info.precision = rc.precision;
    info.integrator = rc.integrator;
    info.frame = rc.frame;
    info.last_rejected = c.last_rejected;
    info.n_beams = rc.nb;
    info.r_km = c.r;
    info.dr_km = c.h_prop;
    info.accepted = c.nacc;
    info.rejected = c.nrej;
    std::FILE* f = std::fopen(path, "wb");
    if (!f) return fail(h, NUOSC_E_INVALID, std::string("cannot create ") + path);
    uint64_t hash = kFnvBasis;
    auto put = [&](const void* d, size_t bytes) {
        hash = fnv1a(d, bytes, hash);
        return std::fwrite(d, 1, bytes, f) == bytes;
    };
    bool ok = put(kSnapTag, sizeof(kSnapTag)) && put(&info, sizeof(info)) && put(psi.data(), psi.size() * 8) &&
              put(phase.data(), phase.size() * 8);
    ok = ok && std::fwrite(&hash, 8, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(h, NUOSC_E_INVALID, std::string("cannot write ") + path);
    return NUOSC_OK;
}

nuosc_status nuosc_snapshot_read(nuosc_handle* h, const char* path)
{
    if (!h || !path) return fail(h, NUOSC_E_INVALID, "NULL argument");
    const RunConst& rc = h->run.rc;
    const nuosc_params& P = h->run.p;
    std::FILE* f = std::fopen(path, "rb");
    if (!f) return fail(h, NUOSC_E_INVALID, std::string("cannot open ") + path);
    uint64_t hash;
    nuosc_snapshot_header info{};
    const char* e = read_snapshot_header(f, info, hash);
    if (!e && (info.n_flavors != rc.n || info.n_energy != rc.ne || info.n_angle != P.n_angle ||
               info.frame != rc.frame))
        e = "snapshot grid, flavors or frame differ from the run's";
    std::vector<double> psi, phase;
    if (!e) {
        psi.resize((size_t)rc.n * 2 * rc.nb);
        phase.resize((size_t)rc.na * rc.n);
        uint64_t stored = 0;
        if (!read_exact(f, psi.data(), psi.size() * 8, hash) || !read_exact(f, phase.data(), phase.size() * 8, hash) ||
            std::fread(&stored, 8, 1, f) != 1)
            e = "truncated snapshot payload";
        else if (stored != hash)
            e = "snapshot checksum mismatch";
    }
    std::fclose(f);
    if (e) return fail(h, NUOSC_E_INVALID, e);
    nuosc_status st = nuosc_set_state(h, psi.data(), phase.data(), info.r_km, info.dr_km);
    if (st != NUOSC_OK) return st;
    Control& c = h->run.hctl;
    c.nacc = info.accepted;
    c.nrej = info.rejected;
    c.attempts = info.accepted + info.rejected;
    c.last_rejected = info.last_rejected != 0;
    return hwrite(h);
}

nuosc_status nuosc_stats(nuosc_handle* h, int64_t* accepted, int64_t* rejected, double* r_km, double* dr_km)
{
    if (!h) return fail(nullptr, NUOSC_E_INVALID, "handle is NULL");
    nuosc_status st = hread(h);
    if (st != NUOSC_OK) return st;
    const Control& c = h->run.hctl;
    if (accepted) *accepted = c.nacc;
    if (rejected) *rejected = c.nrej;
    if (r_km) *r_km = c.r;
    if (dr_km) *dr_km = c.h_prop;
    return hstatus(h);
}

int64_t nuosc_num_beams(const nuosc_handle* h) { return h ? h->run.rc.nb : 0; }
int32_t nuosc_num_traj(const nuosc_handle* h) { return h ? h->run.rc.na : 0; }

const char* nuosc_last_error(const nuosc_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

void nuosc_destroy(nuosc_handle* h)
{
    if (!h) return;
    if (h->is_static) {
        // a slot of g_static_handle: wait for its work, then free the slot
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (h->device < 0) return;  // already released
        (void)hipStreamSynchronize(h->stream);
        for (auto& x : h->ev)
            if (x) (void)hipEventDestroy(x);
        g_static_busy[h->device] = false;
        *h = nuosc_handle();
        h->is_static = true;
        return;
    }
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto& x : h->ev)
        if (x) (void)hipEventDestroy(x);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
struct nuosc_batch {
    int32_t max_slots = 0, n = 0, precision = 0, integrator = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    bool own_arena = false;
    size_t runs_bytes = 0;                 // device RunConst array at the arena's front
    RunConst* runs_dev = nullptr;
    std::map<size_t, size_t> free_blocks;  // arena offset -> bytes, disjoint, coalesced
    std::vector<RunState> runs;
    std::vector<char> used;
    std::vector<size_t> off, bytes;        // arena block of each slot
    // the captured launch sequence of a batch step for one set of active runs;
    // a set is captured only when it is stepped a second time in a row
    hipGraphExec_t graph = nullptr;
    std::vector<int> graph_slots;
    int64_t graph_attempts = 0;
    std::vector<int> last_slots;
    int64_t last_attempts = 0;
    // batch steps that launched work: directly, by graph replay, and captures
    int64_t eager_steps = 0, graph_steps = 0, captures = 0;
    std::string err;
};

namespace {

thread_local std::string g_batch_create_error;

nuosc_status bfail(nuosc_batch* b, nuosc_status st, const std::string& msg)
{
    if (b) b->err = msg;
    else g_batch_create_error = msg;
    return st;
}

// First fit over the free blocks (offsets and sizes multiples of 256).
bool arena_alloc(nuosc_batch* b, size_t need, size_t& at)
{
    need = align_up(need, 256);
    for (auto it = b->free_blocks.begin(); it != b->free_blocks.end(); ++it) {
        if (it->second < need) continue;
        at = it->first;
        const size_t rest = it->second - need;
        b->free_blocks.erase(it);
        if (rest) b->free_blocks[at + need] = rest;
        return true;
    }
    return false;
}

void arena_free(nuosc_batch* b, size_t at, size_t bytes)
{
    bytes = align_up(bytes, 256);
    auto it = b->free_blocks.emplace(at, bytes).first;
    auto next = std::next(it);
    if (next != b->free_blocks.end() && it->first + it->second == next->first) {
        it->second += next->second;
        b->free_blocks.erase(next);
    }
    if (it != b->free_blocks.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            b->free_blocks.erase(it);
        }
    }
}

void drop_graph(nuosc_batch* b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_slots.clear();
    b->graph_attempts = 0;
}

// n attempts of every listed run, launched directly on the stream.
hipError_t launch_attempts(nuosc_batch* b, const nuosc::RunList& list, int64_t n)
{
    const int S = nuosc::num_stages(b->integrator);
    for (int64_t i = 0; i < n; ++i)
        for (int st = 1; st <= S; ++st) {
            hipError_t e = nuosc::launch_stage(list, st, b->stream);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

// Replays (capturing first if the active set or the count changed) the graph
// of n attempts of the listed runs.
nuosc_status graph_attempts(nuosc_batch* b, const std::vector<int>& slots, const nuosc::RunList& list, int64_t n)
{
    if (!b->graph || b->graph_slots != slots || b->graph_attempts != n) {
        drop_graph(b);
        HIP_CHECK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), b->err);
        hipError_t e = launch_attempts(b, list, n);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            b->err = hip_msg(e != hipSuccess ? e : e2, "capture of the batch step");
            return NUOSC_E_DEVICE;
        }
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->err = hip_msg(e, "hipGraphInstantiate");
            return NUOSC_E_DEVICE;
        }
        b->graph = x;
        b->graph_slots = slots;
        b->graph_attempts = n;
        b->captures += 1;
    }
    HIP_CHECK(hipGraphLaunch(b->graph, b->stream), b->err);
    return NUOSC_OK;
}

}  // namespace

extern "C" {

nuosc_status nuosc_batch_create(int32_t max_slots, int32_t n_flavors, int32_t precision, int32_t integrator,
                                size_t hbm_budget_bytes, void* hip_stream, void* device_arena, nuosc_batch** out)
{
    if (!out) return bfail(nullptr, NUOSC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 1024) return bfail(nullptr, NUOSC_E_INVALID, "max_slots must be in 1..1024");
    if (n_flavors != 2 && n_flavors != 3) return bfail(nullptr, NUOSC_E_INVALID, "n_flavors must be 2 or 3");
    if (precision != NUOSC_FP64 && precision != NUOSC_FP32_AMP && precision != NUOSC_FP32_AMP_FP64_MATH)
        return bfail(nullptr, NUOSC_E_INVALID, "unknown precision");
    if (integrator == NUOSC_EXP_STEPPER)
        return bfail(nullptr, NUOSC_E_INVALID, "the exponential stepper runs as single runs, not in batches");
    if (integrator != NUOSC_RK4_FIXED && integrator != NUOSC_RK_DP54)
        return bfail(nullptr, NUOSC_E_INVALID, "unknown integrator");
    const size_t runs_bytes = align_up((size_t)max_slots * sizeof(RunConst), 256);
    if (hbm_budget_bytes < runs_bytes + 256) return bfail(nullptr, NUOSC_E_INVALID, "hbm budget too small");
    nuosc_batch* b = new (std::nothrow) nuosc_batch();
    if (!b) return bfail(nullptr, NUOSC_E_NOMEM, "host allocation failed");
    auto bail = [&](nuosc_status st, const std::string& msg) {
        g_batch_create_error = msg;
        nuosc_batch_destroy(b);
        return st;
    };
    b->max_slots = max_slots;
    b->n = n_flavors;
    b->precision = precision;
    b->integrator = integrator;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(NUOSC_E_DEVICE, hip_msg(e, "hipStreamCreate"));
        b->own_stream = true;
    }
    if (device_arena) {
        b->arena = (char*)device_arena;
    } else {
        hipError_t e = hipMalloc((void**)&b->arena, hbm_budget_bytes);
        if (e != hipSuccess) return bail(NUOSC_E_NOMEM, hip_msg(e, "hipMalloc of the arena"));
        b->own_arena = true;
    }
    b->arena_bytes = hbm_budget_bytes;
    b->runs_bytes = runs_bytes;
    b->runs_dev = (RunConst*)b->arena;
    const size_t usable = (hbm_budget_bytes - runs_bytes) / 256 * 256;
    if (usable) b->free_blocks[runs_bytes] = usable;
    b->runs.resize(max_slots);
    b->used.assign(max_slots, 0);
    b->off.assign(max_slots, 0);
    b->bytes.assign(max_slots, 0);
    *out = b;
    return NUOSC_OK;
}

nuosc_status nuosc_batch_admit(nuosc_batch* b, const nuosc_params* p, int32_t* slot)
{
    if (!b || !slot) return bfail(b, NUOSC_E_INVALID, "NULL argument");
    if (const char* why = validate(p)) return bfail(b, NUOSC_E_INVALID, why);
    if (p->n_flavors != b->n || p->precision != b->precision || p->integrator != b->integrator)
        return bfail(b, NUOSC_E_INVALID, "n_flavors, precision and integrator must match the batch");
    if (p->n_azimuth > 1) return bfail(b, NUOSC_E_INVALID, "batches serve bulb-model runs (n_azimuth 0 or 1)");
    int free_slot = -1;
    for (int i = 0; i < b->max_slots; ++i)
        if (!b->used[i]) {
            free_slot = i;
            break;
        }
    if (free_slot < 0) return bfail(b, NUOSC_E_BUSY, "no free slot");
    const size_t need = make_layout(*p).total;
    size_t at = 0;
    if (!arena_alloc(b, need, at)) return bfail(b, NUOSC_E_BUSY, "no arena gap for the run's footprint");
    RunState& r = b->runs[free_slot];
    r = RunState{};
    nuosc_status st = init_run(r, p, b->arena + at, b->runs_dev, free_slot, b->stream, b->err);
    if (st != NUOSC_OK) {
        arena_free(b, at, need);
        return st;
    }
    b->used[free_slot] = 1;
    b->off[free_slot] = at;
    b->bytes[free_slot] = need;
    drop_graph(b);
    *slot = free_slot;
    return NUOSC_OK;
}

nuosc_status nuosc_batch_step(nuosc_batch* b, int64_t n_attempts, int32_t* n_finished)
{
    if (!b) return bfail(nullptr, NUOSC_E_INVALID, "batch is NULL");
    if (n_attempts < 0) return bfail(b, NUOSC_E_INVALID, "n_attempts must be >= 0");
    std::vector<int> slots;
    std::vector<const RunConst*> rcs;
    for (int i = 0; i < b->max_slots; ++i)
        if (b->used[i] && b->runs[i].hctl.status == 0) {
            slots.push_back(i);
            rcs.push_back(&b->runs[i].rc);
        }
    if (!slots.empty() && n_attempts > 0) {
        const nuosc::RunList list{b->runs_dev, (int)slots.size(), slots.data(), rcs.data()};
        const bool repeat = slots == b->last_slots && n_attempts == b->last_attempts;
        b->last_slots = slots;
        b->last_attempts = n_attempts;
        if (repeat) {
            nuosc_status st = graph_attempts(b, slots, list, n_attempts);
            if (st != NUOSC_OK) return st;
            b->graph_steps += 1;
        } else {
            HIP_CHECK(launch_attempts(b, list, n_attempts), b->err);
            b->eager_steps += 1;
        }
        for (int i : slots)
            HIP_CHECK(hipMemcpyAsync(&b->runs[i].hctl, b->runs[i].rc.ctrl + 1, sizeof(Control), hipMemcpyDeviceToHost,
                                     b->stream), b->err);
        HIP_CHECK(hipStreamSynchronize(b->stream), b->err);
    }
    int32_t fin = 0;
    for (int i = 0; i < b->max_slots; ++i)
        if (b->used[i] && b->runs[i].hctl.status != 0) ++fin;
    if (n_finished) *n_finished = fin;
    return NUOSC_OK;
}

nuosc_status nuosc_batch_query(nuosc_batch* b, int32_t slot, int64_t* accepted, int64_t* rejected, double* r_km,
                               int32_t* done, int32_t* run_status)
{
    if (!b) return bfail(nullptr, NUOSC_E_INVALID, "batch is NULL");
    if (slot < 0 || slot >= b->max_slots || !b->used[slot]) return bfail(b, NUOSC_E_INVALID, "slot is not occupied");
    const Control& c = b->runs[slot].hctl;
    if (accepted) *accepted = c.nacc;
    if (rejected) *rejected = c.nrej;
    if (r_km) *r_km = c.r;
    if (done) *done = c.status != 0 ? 1 : 0;
    std::string why;
    const nuosc_status st = status_of(c, why);
    if (run_status) *run_status = st;
    return NUOSC_OK;
}

int64_t nuosc_batch_num_beams(const nuosc_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->used[slot]) return 0;
    return b->runs[slot].rc.nb;
}

nuosc_status nuosc_batch_retire(nuosc_batch* b, int32_t slot, double* p_out)
{
    if (!b) return bfail(nullptr, NUOSC_E_INVALID, "batch is NULL");
    if (slot < 0 || slot >= b->max_slots || !b->used[slot]) return bfail(b, NUOSC_E_INVALID, "slot is not occupied");
    if (p_out) {
        nuosc_status st = probabilities_of(b->runs[slot], p_out, b->stream, b->err);
        if (st != NUOSC_OK) return st;
    }
    HIP_CHECK(hipStreamSynchronize(b->stream), b->err);
    arena_free(b, b->off[slot], b->bytes[slot]);
    b->used[slot] = 0;
    b->runs[slot] = RunState{};
    drop_graph(b);
    return NUOSC_OK;
}

nuosc_status nuosc_batch_graph_stats(const nuosc_batch* b, int64_t* eager_steps, int64_t* graph_steps,
                                     int64_t* captures)
{
    if (!b) return bfail(nullptr, NUOSC_E_INVALID, "batch is NULL");
    if (eager_steps) *eager_steps = b->eager_steps;
    if (graph_steps) *graph_steps = b->graph_steps;
    if (captures) *captures = b->captures;
    return NUOSC_OK;
}

int32_t nuosc_batch_occupied(const nuosc_batch* b)
{
    if (!b) return 0;
    int32_t k = 0;
    for (char u : b->used) k += u ? 1 : 0;
    return k;
}

const char* nuosc_batch_last_error(const nuosc_batch* b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

void nuosc_batch_destroy(nuosc_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->own_arena && b->arena) (void)hipFree(b->arena);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
