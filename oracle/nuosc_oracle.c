/*
 * Oracle for the bulb-model neutrino flavor evolution -- TEST INFRASTRUCTURE.
 *
 * Plain FP64 C written from the paper (Noormofidi, "Simulating Nonlinear
 * Neutrino Oscillations on Next-Generation Many-Core Architectures", arXiv
 * 1907.05560).  Only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  No blocking, fusion or reordering beyond what the
 * equations state; every sum runs in one fixed, documented order:
 *   - per-trajectory sums over energy ascending, all neutrinos first, then all
 *     antineutrinos;
 *   - angle moments over trajectories ascending, J0 and J1 in the same loop.
 * Build with -O2 -fno-fast-math -ffp-contract=off.
 *
 * Readings of the paper that this file takes (each is also stated where used):
 *   A  emission-angle bins at midpoints u_j = (j + 1/2)/N_A of cos(theta_0).
 *   B  Fermi-Dirac denominator exp(E/T - eta) + 1 (eq 4.1 is garbled).
 *   C  spectra normalised on (0, inf); beam weights divided by the fixed
 *      reference number luminosity 1e51 erg/s / 11 MeV.
 *   D  three flavors: PDG mixing matrix, matter term diag(lambda, 0, 0),
 *      antineutrinos use the complex conjugate vacuum Hamiltonian.
 *   E  every Hamiltonian is made traceless.
 *   F  density matrix rho = 2 psi psi^dagger (eq 3.9 up to its trace part).
 *   G  the coupling mu0 absorbs the prefactor eq 3.8 omits; the single-angle
 *      model multiplies it by D(r/R) (eq 3.16-3.17).
 *   H  evolution in the frame co-rotating with the flavor-diagonal part of
 *      the matter and self-interaction terms (see rhs()).
 *   I  embedded pair: Dormand-Prince 5(4), FSAL, advancing the 5th-order
 *      solution.
 *   J  step control: safety 0.9, growth factor in [0.2, 5], no growth right
 *      after a rejection, step capped at dr_max, last step clipped to r_end.
 *   K  step error: max over beams, components and re/im parts of
 *      |h sum_i e_i k_i| / rtol; the co-rotating phases are excluded.
 *   N  only nu_e-born and nubar_e-born beams are evolved; the nu_x flavors
 *      enter through the weights (unitarity of the flavor basis).
 *   Q  the paper's own stepper (eq 3.10-3.12 inside the half/full-step loop of
 *      Sections 4.2.3 and 5): which states are averaged and compared (see
 *      exp_attempt()); lab frame only.
 */
#include "nuosc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Built with -fopenmp (the timing variant liboracle_omp.so), the loops marked
 * OR_PARALLEL_FOR run their independent iterations (trajectories, beams or
 * state entries, each written by exactly one iteration) on several threads.
 * Every value is computed by the same code in the same order as in the serial
 * build; the sums over trajectories and the error maximum stay sequential or
 * exact, so both builds give bitwise the same results. */
#ifdef _OPENMP
#include <omp.h>
#define OR_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define OR_PARALLEL_FOR
#endif

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- complex */
typedef struct { double re, im; } cplx;

static cplx c_make(double re, double im) { cplx z; z.re = re; z.im = im; return z; }
static cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static cplx c_sub(cplx a, cplx b) { return c_make(a.re - b.re, a.im - b.im); }
static cplx c_mul(cplx a, cplx b) { return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static cplx c_conj(cplx a) { return c_make(a.re, -a.im); }
static cplx c_scale(cplx a, double s) { return c_make(a.re * s, a.im * s); }
static cplx c_expi(double phi) { return c_make(cos(phi), sin(phi)); }

/* ---------------------------------------------------------------- constants */
/* hbar*c = 197.3269804 MeV fm (CODATA 2018) = 1.973269804e-10 eV km.
 * Vacuum frequency (eq 3.6): Delta = dm2 / (2E), i.e. in km^-1 with E in MeV
 * and dm2 in eV^2: Delta = dm2 / (2 * 1e6 * E * hbar c[eV km]). */
static const double HBARC_EV_KM = 1.973269804e-10;
double or_vacuum_coefficient(void) { return 1.0 / (2.0e6 * HBARC_EV_KM); }

/* Reference number luminosity used to normalise the beam weights (reading C):
 * 1e51 erg/s carried at a mean energy of 11 MeV. */
static const double OR_PI = 3.14159265358979323846;
static const double LREF_ERG_S = 1e51;
static const double EREF_MEV = 11.0;

/* ---------------------------------------------------------------- run */
struct or_run {
    or_params p;
    int n;          /* flavors */
    int ne;         /* energy bins */
    int na;         /* trajectories: N_A (x N_phi azimuth bins), or 1 for the single-angle model */
    int nth;        /* emission (zenith) angle bins */
    int np;         /* azimuth bins per emission angle (1: the bulb model) */
    int ma;         /* 1 = multi-angle bulb model, 0 = single angle */
    int64_t nb;     /* beams = 2 * ne * na */
    int64_t ylen;   /* 2*n*nb amplitude reals followed by n*na phases */
    double* energy; /* [ne] */
    double* g;      /* [ne] neutrino weight */
    double* gbar;   /* [ne] antineutrino weight */
    cplx* hvac;     /* [ne][n][n] neutrino vacuum Hamiltonian */
    double* y;      /* state */
    double* k[7];   /* stage derivatives */
    double* ytmp;
    /* per-evaluation work */
    cplx* S;        /* [na][n][n] per-trajectory lab-frame sums */
    double* c;      /* [na] */
    double* w;      /* [na] */
    double* phi;    /* [na] azimuth angle of each trajectory */
    /* stepping */
    double r, h;
    int64_t istep;  /* RK4 steps taken */
    int64_t nacc, nrej;
    int last_rejected;
    int k1_valid;   /* Dormand-Prince first-same-as-last derivative held in k[0] */
    double last_err; /* scaled error of the last adaptive attempt */
    int done;
};

int64_t or_num_beams(const or_run* R) { return R->nb; }
int32_t or_num_traj(const or_run* R) { return R->na; }
int64_t or_state_len(const or_run* R) { return R->ylen; }

/* ------------------------------------------------------------ spectra (eq 4.1-4.2) */
/* F_k(eta) = int_0^inf x^k / (exp(x - eta) + 1) dx, composite Simpson rule on
 * [0, max(eta, 0) + 120]; the integrand is smooth and the tail is below 1e-50.
 * The 4e5 weighted samples are added with Kahan's compensated summation so that
 * rounding does not accumulate over the long sum. */
double or_fermi_integral(int k, double eta)
{
    const double X = (eta > 0.0 ? eta : 0.0) + 120.0;
    const int64_t N = 400000; /* even */
    const double h = X / (double)N;
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i <= N; ++i) {
        double x = h * (double)i;
        double f = pow(x, (double)k) / (exp(x - eta) + 1.0);
        double wgt = (i == 0 || i == N) ? 1.0 : ((i % 2) ? 4.0 : 2.0);
        double term = wgt * f - comp;
        double t = s + term;
        comp = (t - s) - term;
        s = t;
    }
    return s * h / 3.0;
}

/* <E> = T F3(eta) / F2(eta) for the spectrum of eq 4.1, so T = <E> F2 / F3. */
double or_temperature(double mean_e, double eta)
{
    return mean_e * or_fermi_integral(2, eta) / or_fermi_integral(3, eta);
}

/* Normalised Fermi-Dirac spectrum, eq 4.1 with reading B; f2 = F_2(eta). */
static double spectrum(double e, double t, double eta, double f2)
{
    return e * e / (f2 * t * t * t * (exp(e / t - eta) + 1.0));
}

double or_spectrum(double e, double t, double eta)
{
    return spectrum(e, t, eta, or_fermi_integral(2, eta));
}

/* ------------------------------------------------------------ geometry */
/* Single-angle geometric factor, eq 3.17: D(x) = 1/2 [1 - sqrt(1 - 1/x^2)]^2,
 * with 1 - 1/x^2 evaluated as (x - 1)(x + 1) / x^2 (exact subtraction near x = 1). */
double or_dilution(double x)
{
    double s = 1.0 - sqrt((x - 1.0) * (x + 1.0) / (x * x));
    return 0.5 * s * s;
}

/* Multi-angle: c_j(r) = cos(theta) at radius r of the trajectory emitted at
 * cos(theta_0) = u_j (eq 3.14), and the quadrature weight of d cos(theta') from
 * eq 3.15 with d cos^2(theta_0) = 2 u du: w_j = (R/r)^2 u_j du / c_j.
 * Eq 3.14 is evaluated in the equivalent form c^2 = u^2 + (1 - u^2)(1 - (R/r)^2)
 * with 1 - (R/r)^2 = (r - R)(r + R) / r^2: near the neutrinosphere the
 * literal 1 - (R/r)^2 (1 - u^2) cancels to a few digits for small u.
 * Single angle: the radial test ray, c = 1, and w[0] returns D(r/R). */
static void geometry(const or_run* R, double r, double* c, double* w)
{
    const double Rn = R->p.r_nu_km;
    if (!R->ma) {
        c[0] = 1.0;
        w[0] = or_dilution(r / Rn);
        return;
    }
    const double x = (Rn / r) * (Rn / r);
    const double y = (r - Rn) * (r + Rn) / (r * r);  /* 1 - (R/r)^2 */
    const double du = 1.0 / (double)R->nth;
    for (int j = 0; j < R->na; ++j) {
        /* trajectory j: emission angle bin j / N_phi, azimuth bin j % N_phi;
         * the azimuth bins share the emission-angle weight equally */
        double u = ((double)(j / R->np) + 0.5) * du; /* reading A */
        c[j] = sqrt(u * u + (1.0 - u * u) * y);
        w[j] = x * u * du / c[j] / (double)R->np;
    }
}

void or_geometry(const or_run* R, double r, double* c, double* w) { geometry(R, r, c, w); }

/* ------------------------------------------------------------ Hamiltonian pieces */
static double matter_potential(const or_run* R, double r)
{
    return R->p.lambda0_km * pow(R->p.lambda_rref_km / r, R->p.lambda_power);
}

/* Vacuum Hamiltonian of a neutrino of energy e (MeV), made traceless.
 * Two flavors, eq 3.5: (Delta/2) [[-cos 2theta, sin 2theta], [sin 2theta, cos 2theta]].
 * Three flavors (reading D): U diag(0, kappa dm21/E, kappa dm31/E) U^dagger
 * minus its trace, with U = R23 U13(delta) R12 (PDG). */
static void vacuum_hamiltonian(const or_params* p, double e, cplx* h)
{
    const double kappa = or_vacuum_coefficient();
    if (p->n_flavors == 2) {
        double d = kappa * p->dm2_ev2 / e;
        double c2 = cos(2.0 * p->theta), s2 = sin(2.0 * p->theta);
        h[0] = c_make(-0.5 * d * c2, 0.0);
        h[1] = c_make(0.5 * d * s2, 0.0);
        h[2] = c_make(0.5 * d * s2, 0.0);
        h[3] = c_make(0.5 * d * c2, 0.0);
        return;
    }
    double c12 = cos(p->theta12), s12 = sin(p->theta12);
    double c13 = cos(p->theta13), s13 = sin(p->theta13);
    double c23 = cos(p->theta23), s23 = sin(p->theta23);
    cplx r12[9] = {c_make(c12, 0), c_make(s12, 0), c_make(0, 0),
                   c_make(-s12, 0), c_make(c12, 0), c_make(0, 0),
                   c_make(0, 0), c_make(0, 0), c_make(1, 0)};
    cplx u13[9] = {c_make(c13, 0), c_make(0, 0), c_scale(c_expi(-p->delta_cp), s13),
                   c_make(0, 0), c_make(1, 0), c_make(0, 0),
                   c_scale(c_expi(p->delta_cp), -s13), c_make(0, 0), c_make(c13, 0)};
    cplx r23[9] = {c_make(1, 0), c_make(0, 0), c_make(0, 0),
                   c_make(0, 0), c_make(c23, 0), c_make(s23, 0),
                   c_make(0, 0), c_make(-s23, 0), c_make(c23, 0)};
    cplx t[9], U[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx s = c_make(0, 0);
            for (int m = 0; m < 3; ++m) s = c_add(s, c_mul(u13[a * 3 + m], r12[m * 3 + b]));
            t[a * 3 + b] = s;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx s = c_make(0, 0);
            for (int m = 0; m < 3; ++m) s = c_add(s, c_mul(r23[a * 3 + m], t[m * 3 + b]));
            U[a * 3 + b] = s;
        }
    double m[3] = {0.0, kappa * p->dm2_21_ev2 / e, kappa * p->dm2_31_ev2 / e};
    double tr3 = (m[0] + m[1] + m[2]) / 3.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx s = c_make(0, 0);
            for (int i = 0; i < 3; ++i)
                s = c_add(s, c_scale(c_mul(U[a * 3 + i], c_conj(U[b * 3 + i])), m[i]));
            if (a == b) s = c_sub(s, c_make(tr3, 0.0));
            h[a * 3 + b] = s;
        }
}

void or_tables(const or_run* R, double* energy, double* g, double* gbar, double* hvac)
{
    const int n = R->n;
    for (int k = 0; k < R->ne; ++k) {
        if (energy) energy[k] = R->energy[k];
        if (g) g[k] = R->g[k];
        if (gbar) gbar[k] = R->gbar[k];
        if (hvac)
            for (int i = 0; i < n * n; ++i) {
                hvac[(k * n * n + i) * 2 + 0] = R->hvac[k * n * n + i].re;
                hvac[(k * n * n + i) * 2 + 1] = R->hvac[k * n * n + i].im;
            }
    }
}

/* ------------------------------------------------------------ create / destroy */
or_run* or_create(const or_params* p)
{
    if (!p || (p->n_flavors != 2 && p->n_flavors != 3) || p->n_energy < 1 || p->n_angle < 0 ||
        p->n_azimuth < 0 || (p->n_azimuth > 1 && p->n_angle < 1))
        return NULL;
    or_run* R = (or_run*)calloc(1, sizeof(or_run));
    R->p = *p;
    R->n = p->n_flavors;
    R->ne = p->n_energy;
    R->ma = p->n_angle > 0;
    R->nth = R->ma ? p->n_angle : 1;
    R->np = p->n_azimuth > 1 ? p->n_azimuth : 1;
    R->na = R->nth * R->np;
    R->nb = 2 * (int64_t)R->ne * R->na;
    R->ylen = 2 * (int64_t)R->n * R->nb + (int64_t)R->n * R->na;
    const int n = R->n;

    R->energy = (double*)calloc(R->ne, sizeof(double));
    R->g = (double*)calloc(R->ne, sizeof(double));
    R->gbar = (double*)calloc(R->ne, sizeof(double));
    R->hvac = (cplx*)calloc((size_t)R->ne * n * n, sizeof(cplx));
    R->y = (double*)calloc(R->ylen, sizeof(double));
    for (int i = 0; i < 7; ++i) R->k[i] = (double*)calloc(R->ylen, sizeof(double));
    R->ytmp = (double*)calloc(R->ylen, sizeof(double));
    R->S = (cplx*)calloc((size_t)R->na * n * n, sizeof(cplx));
    R->c = (double*)calloc(R->na, sizeof(double));
    R->w = (double*)calloc(R->na, sizeof(double));
    R->phi = (double*)calloc(R->na, sizeof(double));
    /* Reading P: azimuth bins at the midpoints of [0, 2 pi). */
    if (R->np > 1)
        for (int j = 0; j < R->na; ++j) R->phi[j] = 2.0 * OR_PI * ((double)(j % R->np) + 0.5) / (double)R->np;

    /* Energy bins at midpoints of [E0, E1]. */
    const double de = (p->e_max_mev - p->e_min_mev) / (double)R->ne;
    double temp[4], f2[4];
    for (int s = 0; s < 4; ++s) {
        f2[s] = or_fermi_integral(2, p->eta[s]);
        temp[s] = p->mean_e_mev[s] * f2[s] / or_fermi_integral(3, p->eta[s]);
    }
    /* Number luminosity of species s relative to the reference (reading C). */
    double nrel[4];
    for (int s = 0; s < 4; ++s)
        nrel[s] = (p->lum_erg_s[s] / LREF_ERG_S) * (EREF_MEV / p->mean_e_mev[s]);
    for (int k = 0; k < R->ne; ++k) {
        double e = p->e_min_mev + ((double)k + 0.5) * de;
        R->energy[k] = e;
        /* Reading N: nu_mu and nu_tau both carry the nu_x spectrum, so the sum
         * of eq 3.8 over initial flavors reduces to (n_e - n_x) rho_e plus a
         * multiple of the identity, which drops out of the traceless H. */
        double fe = spectrum(e, temp[0], p->eta[0], f2[0]);
        double fx = spectrum(e, temp[2], p->eta[2], f2[2]);
        double fbe = spectrum(e, temp[1], p->eta[1], f2[1]);
        double fbx = spectrum(e, temp[3], p->eta[3], f2[3]);
        R->g[k] = de * (nrel[0] * fe - nrel[2] * fx);
        R->gbar[k] = de * (nrel[1] * fbe - nrel[3] * fbx);
        vacuum_hamiltonian(p, e, &R->hvac[(size_t)k * n * n]);
    }

    /* Initial state: every beam in its birth flavor (component 0), phases 0. */
    for (int64_t b = 0; b < R->nb; ++b) R->y[(b * n + 0) * 2 + 0] = 1.0;
    R->r = p->r_start_km;
    R->h = p->dr_init_km;
    if (R->h > p->dr_max_km) R->h = p->dr_max_km;
    if (R->r + R->h > p->r_end_km) R->h = p->r_end_km - R->r;
    return R;
}

void or_destroy(or_run* R)
{
    if (!R) return;
    free(R->energy); free(R->g); free(R->gbar); free(R->hvac); free(R->y);
    for (int i = 0; i < 7; ++i) free(R->k[i]);
    free(R->ytmp); free(R->S); free(R->c); free(R->w); free(R->phi);
    free(R);
}

/* ------------------------------------------------------------ state access */
int or_get_state(const or_run* R, double* psi, double* phase)
{
    const int n = R->n;
    if (psi)
        for (int a = 0; a < n; ++a)
            for (int64_t b = 0; b < R->nb; ++b) {
                psi[((int64_t)a * 2 + 0) * R->nb + b] = R->y[(b * n + a) * 2 + 0];
                psi[((int64_t)a * 2 + 1) * R->nb + b] = R->y[(b * n + a) * 2 + 1];
            }
    if (phase)
        memcpy(phase, R->y + 2 * (int64_t)n * R->nb, sizeof(double) * (size_t)n * R->na);
    return 0;
}

int or_set_state(or_run* R, const double* psi, const double* phase, double r_km)
{
    const int n = R->n;
    if (psi)
        for (int a = 0; a < n; ++a)
            for (int64_t b = 0; b < R->nb; ++b) {
                R->y[(b * n + a) * 2 + 0] = psi[((int64_t)a * 2 + 0) * R->nb + b];
                R->y[(b * n + a) * 2 + 1] = psi[((int64_t)a * 2 + 1) * R->nb + b];
            }
    if (phase)
        memcpy(R->y + 2 * (int64_t)n * R->nb, phase, sizeof(double) * (size_t)n * R->na);
    R->r = r_km;
    R->k1_valid = 0;
    R->done = 0;
    return 0;
}

/* ------------------------------------------------------------ physics */
/* Amplitude of flavor component a of beam b inside flat state y. */
static cplx amp(const or_run* R, const double* y, int64_t b, int a)
{
    return c_make(y[(b * R->n + a) * 2 + 0], y[(b * R->n + a) * 2 + 1]);
}

/* Angle moments (eq 3.13 factorised, eq 3.16 for the single-angle model).
 *
 * For every trajectory j, with beams in the co-rotating frame (reading H):
 * the lab-frame amplitude is psi = exp(-i sigma Phi_j) psi~ (sigma = +1 for
 * neutrinos, -1 for antineutrinos), so the lab-frame density matrix of
 * eq 3.9 (reading F: rho = 2 psi psi^dagger) has elements
 *   rho_ab = 2 exp(-i sigma (Phi_a - Phi_b)) psi~_a conj(psi~_b).
 * The integrand of eq 3.8 is rho_nu g - conj(rho_nubar) gbar, therefore
 *   S_j = 2 exp(-i (Phi_a - Phi_b)) sum_k [g_k psi~_a conj(psi~_b)
 *                                  - gbar_k conj(psibar~_a conj(psibar~_b))].
 * The kernel (1 - cos(theta) cos(theta')) of eq 3.13 splits into
 *   J0 = sum_j w_j S_j  and  J1 = sum_j w_j c_j S_j,
 * so that H_nunu on trajectory i is mu0 * traceless(J0 - c_i J1).
 * Single angle: J0 = D(r/R) S_0 and J1 = 0 (c = 1 for the radial ray). */
/* Neumaier's compensated summation: *s + *c carries the running sum. */
static void neu_add(double* s, double* c, double x)
{
    const double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

/* The density sum of trajectory j with the sum_mode order and kind (modes
 * 1-3; mode 0 is written out in moments_at). */
static void density_sum_mode(const or_run* R, const double* y, int j, cplx* acc)
{
    const int n = R->n, ne = R->ne, na = R->na;
    const int comp = R->p.sum_mode & 1, rev = (R->p.sum_mode >> 1) & 1;
    double sr[9], si[9], cr[9], ci[9];
    for (int i = 0; i < n * n; ++i) sr[i] = si[i] = cr[i] = ci[i] = 0.0;
    for (int step = 0; step < 2 * ne; ++step) {
        const int idx = rev ? 2 * ne - 1 - step : step;
        const int sp = idx / ne, k = idx - sp * ne;
        const int64_t b = (int64_t)(sp * na + j) * ne + k;
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c) {
                cplx rho = c_mul(amp(R, y, b, a), c_conj(amp(R, y, b, c)));
                cplx t = sp == 0 ? c_scale(rho, R->g[k]) : c_scale(c_conj(rho), -R->gbar[k]);
                const int i = a * n + c;
                if (comp) {
                    neu_add(&sr[i], &cr[i], t.re);
                    neu_add(&si[i], &ci[i], t.im);
                } else {
                    sr[i] += t.re;
                    si[i] += t.im;
                }
            }
    }
    for (int i = 0; i < n * n; ++i) acc[i] = c_make(sr[i] + cr[i], si[i] + ci[i]);
}

static void moments_at(const or_run* R, double r, const double* y, cplx* J0, cplx* J1, cplx* J2, cplx* J3)
{
    const int n = R->n, ne = R->ne, na = R->na;
    const double* phase = y + 2 * (int64_t)n * R->nb;
    geometry(R, r, R->c, R->w);
    if (R->p.sum_mode != 0) {
        OR_PARALLEL_FOR
        for (int j = 0; j < na; ++j) {
            cplx acc[9];
            density_sum_mode(R, y, j, acc);
            for (int a = 0; a < n; ++a)
                for (int c = 0; c < n; ++c) {
                    double dphi = phase[j * n + a] - phase[j * n + c];
                    R->S[(j * n + a) * n + c] = c_scale(c_mul(c_expi(-dphi), acc[a * n + c]), 2.0);
                }
        }
        for (int i = 0; i < n * n; ++i) {
            J0[i] = c_make(0, 0);
            J1[i] = c_make(0, 0);
            J2[i] = c_make(0, 0);
            J3[i] = c_make(0, 0);
        }
        if (!R->ma) {
            for (int i = 0; i < n * n; ++i) J0[i] = c_scale(R->S[i], R->w[0]);
            return;
        }
        const int comp = R->p.sum_mode & 1, rev = (R->p.sum_mode >> 1) & 1;
        const int nm = R->np > 1 ? 4 : 2;
        for (int i = 0; i < n * n; ++i) {
            double s[8] = {0}, c[8] = {0};
            for (int step = 0; step < na; ++step) {
                const int j = rev ? na - 1 - step : step;
                const double sn = sqrt((1.0 - R->c[j]) * (1.0 + R->c[j]));
                const double f[4] = {R->w[j], R->w[j] * R->c[j], R->w[j] * sn * cos(R->phi[j]),
                                     R->w[j] * sn * sin(R->phi[j])};
                for (int m = 0; m < nm; ++m) {
                    const cplx t = c_scale(R->S[j * n * n + i], f[m]);
                    if (comp) {
                        neu_add(&s[2 * m], &c[2 * m], t.re);
                        neu_add(&s[2 * m + 1], &c[2 * m + 1], t.im);
                    } else {
                        s[2 * m] += t.re;
                        s[2 * m + 1] += t.im;
                    }
                }
            }
            cplx* out[4] = {J0, J1, J2, J3};
            for (int m = 0; m < nm; ++m) out[m][i] = c_make(s[2 * m] + c[2 * m], s[2 * m + 1] + c[2 * m + 1]);
        }
        return;
    }
    OR_PARALLEL_FOR
    for (int j = 0; j < na; ++j) {
        cplx acc[9];
        for (int i = 0; i < n * n; ++i) acc[i] = c_make(0, 0);
        for (int k = 0; k < ne; ++k) {
            int64_t b = (int64_t)(0 * na + j) * ne + k;
            for (int a = 0; a < n; ++a)
                for (int c = 0; c < n; ++c) {
                    cplx rho = c_mul(amp(R, y, b, a), c_conj(amp(R, y, b, c)));
                    acc[a * n + c] = c_add(acc[a * n + c], c_scale(rho, R->g[k]));
                }
        }
        for (int k = 0; k < ne; ++k) {
            int64_t b = (int64_t)(1 * na + j) * ne + k;
            for (int a = 0; a < n; ++a)
                for (int c = 0; c < n; ++c) {
                    cplx rho = c_mul(amp(R, y, b, a), c_conj(amp(R, y, b, c)));
                    acc[a * n + c] = c_sub(acc[a * n + c], c_scale(c_conj(rho), R->gbar[k]));
                }
        }
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c) {
                double dphi = phase[j * n + a] - phase[j * n + c];
                R->S[(j * n + a) * n + c] = c_scale(c_mul(c_expi(-dphi), acc[a * n + c]), 2.0);
            }
    }
    for (int i = 0; i < n * n; ++i) {
        J0[i] = c_make(0, 0);
        J1[i] = c_make(0, 0);
        J2[i] = c_make(0, 0);
        J3[i] = c_make(0, 0);
    }
    if (!R->ma) {
        for (int i = 0; i < n * n; ++i) J0[i] = c_scale(R->S[i], R->w[0]);
        return;
    }
    for (int j = 0; j < na; ++j)
        for (int i = 0; i < n * n; ++i) {
            J0[i] = c_add(J0[i], c_scale(R->S[j * n * n + i], R->w[j]));
            J1[i] = c_add(J1[i], c_scale(R->S[j * n * n + i], R->w[j] * R->c[j]));
        }
    if (R->np == 1) return;
    /* Extended bulb model (eq 3.18): 1 - cos(gamma) = 1 - c c' - s s' cos(phi - phi')
     * = 1 - c c' - s cos(phi) s' cos(phi') - s sin(phi) s' sin(phi'), so two more
     * moments carry the azimuth dependence; s = sin(theta) = sqrt(1 - c^2). */
    for (int j = 0; j < na; ++j) {
        const double s = sqrt((1.0 - R->c[j]) * (1.0 + R->c[j]));
        for (int i = 0; i < n * n; ++i) {
            J2[i] = c_add(J2[i], c_scale(R->S[j * n * n + i], R->w[j] * s * cos(R->phi[j])));
            J3[i] = c_add(J3[i], c_scale(R->S[j * n * n + i], R->w[j] * s * sin(R->phi[j])));
        }
    }
}

/* H_nunu of trajectory j = mu0 * traceless(J0 - c J1)  (readings E, G); the
 * extended model subtracts s cos(phi) J2 + s sin(phi) J3 as well (eq 3.18). */
static void collective(const or_run* R, const cplx* J0, const cplx* J1, const cplx* J2, const cplx* J3, int j,
                       cplx* C)
{
    const int n = R->n;
    const double c = R->c[j];
    for (int i = 0; i < n * n; ++i) C[i] = c_sub(J0[i], c_scale(J1[i], c));
    if (R->np > 1) {
        const double s = sqrt((1.0 - c) * (1.0 + c));
        const double sc = s * cos(R->phi[j]), ss = s * sin(R->phi[j]);
        for (int i = 0; i < n * n; ++i) C[i] = c_sub(c_sub(C[i], c_scale(J2[i], sc)), c_scale(J3[i], ss));
    }
    double tr = 0.0;
    for (int a = 0; a < n; ++a) tr += C[a * n + a].re;
    for (int a = 0; a < n; ++a) C[a * n + a].re -= tr / (double)n;
    for (int i = 0; i < n * n; ++i) C[i] = c_scale(C[i], R->p.mu0_km);
}

/* Right-hand side of the flavor evolution (eq 3.2 with the bulb geometry).
 *
 * Along trajectory j the path length is l = r cos(theta) (eq 3.3), so
 * d psi / dr = -i H psi / c_j.  The Hamiltonian (readings D, E) is
 *   neutrino:      H  = H_vac(E) + H_m(r) + H_nunu
 *   antineutrino:  Hb = conj(H_vac(E)) - H_m(r) - conj(H_nunu)      (eq 3.4)
 * with H_m = lambda(r) * traceless(diag(1, 0[, 0])).
 *
 * Co-rotating frame (reading H).  Let G_j = diag(H_m + H_nunu) / c_j (real,
 * the same for every energy on trajectory j) and dPhi_j/dr = G_j.  Writing
 * psi = exp(-i sigma Phi_j) psi~ with sigma = +1 (nu), -1 (nubar), the
 * antineutrino diagonal is -(H_m + H_nunu)_aa, so both species evolve as
 *   d psi~ / dr = -i K~ psi~,
 *   K~_ab = exp(i sigma (Phi_a - Phi_b)) H_ab / c_j   (a != b),
 *   K~_aa = H_aa / c_j - sigma G_a = (H_vac)_aa / c_j.
 * The last equality is exact: the frame removes the matter and self-
 * interaction diagonal, which carries the large terms near the neutrinosphere.
 * In the lab frame Phi = G = 0 and K~ = H / c_j. */
static void rhs(const or_run* R, double r, const double* y, double* dy)
{
    const int n = R->n, ne = R->ne, na = R->na;
    const int corot = (R->p.frame == 0);
    const double* phase = y + 2 * (int64_t)n * R->nb;
    double* dphase = dy + 2 * (int64_t)n * R->nb;
    cplx J0[9], J1[9], J2[9], J3[9];
    moments_at(R, r, y, J0, J1, J2, J3); /* also leaves c_j, w_j in R->c, R->w */
    const double lam = matter_potential(R, r);

    OR_PARALLEL_FOR
    for (int j = 0; j < na; ++j) {
        const double cj = R->c[j];
        cplx C[9], Hm[9];
        collective(R, J0, J1, J2, J3, j, C);
        for (int i = 0; i < n * n; ++i) Hm[i] = c_make(0, 0);
        for (int a = 0; a < n; ++a) Hm[a * n + a] = c_make(lam * ((a == 0 ? 1.0 : 0.0) - 1.0 / (double)n), 0.0);
        double G[3] = {0, 0, 0};
        if (corot)
            for (int a = 0; a < n; ++a) G[a] = (Hm[a * n + a].re + C[a * n + a].re) / cj;
        for (int a = 0; a < n; ++a) dphase[j * n + a] = G[a];

        for (int s = 0; s < 2; ++s) {
            const double sigma = (s == 0) ? 1.0 : -1.0;
            cplx rot[9]; /* exp(i sigma (Phi_a - Phi_b)) */
            for (int a = 0; a < n; ++a)
                for (int c = 0; c < n; ++c)
                    rot[a * n + c] = c_expi(sigma * (phase[j * n + a] - phase[j * n + c]));
            for (int k = 0; k < ne; ++k) {
                const cplx* hv = &R->hvac[(size_t)k * n * n];
                cplx K[9];
                for (int a = 0; a < n; ++a)
                    for (int c = 0; c < n; ++c) {
                        cplx H;
                        if (s == 0)
                            H = c_add(c_add(hv[a * n + c], Hm[a * n + c]), C[a * n + c]);
                        else
                            H = c_sub(c_sub(c_conj(hv[a * n + c]), Hm[a * n + c]), c_conj(C[a * n + c]));
                        if (a != c)
                            K[a * n + c] = c_scale(c_mul(rot[a * n + c], H), 1.0 / cj);
                        else if (corot)
                            K[a * n + c] = c_make(hv[a * n + a].re / cj, 0.0);
                        else
                            K[a * n + c] = c_make(H.re / cj, 0.0);
                    }
                int64_t b = (int64_t)(s * na + j) * ne + k;
                for (int a = 0; a < n; ++a) {
                    cplx acc = c_make(0, 0);
                    for (int c = 0; c < n; ++c) acc = c_add(acc, c_mul(K[a * n + c], amp(R, y, b, c)));
                    /* -i * acc */
                    dy[(b * n + a) * 2 + 0] = acc.im;
                    dy[(b * n + a) * 2 + 1] = -acc.re;
                }
            }
        }
    }
}

void or_rhs(const or_run* R, double r, const double* y, double* dydr) { rhs(R, r, y, dydr); }

static void write_moments(const cplx* J, double* out, int n)
{
    for (int i = 0; i < n * n; ++i) { out[2 * i] = J[i].re; out[2 * i + 1] = J[i].im; }
}

void or_moments(const or_run* R, double* j0, double* j1)
{
    cplx J0[9], J1[9], J2[9], J3[9];
    moments_at(R, R->r, R->y, J0, J1, J2, J3);
    if (j0) write_moments(J0, j0, R->n);
    if (j1) write_moments(J1, j1, R->n);
}

void or_moments_azimuth(const or_run* R, double* j2, double* j3)
{
    cplx J0[9], J1[9], J2[9], J3[9];
    moments_at(R, R->r, R->y, J0, J1, J2, J3);
    if (j2) write_moments(J2, j2, R->n);
    if (j3) write_moments(J3, j3, R->n);
}

void or_azimuth(const or_run* R, double* phi)
{
    for (int j = 0; j < R->na; ++j) phi[j] = R->phi[j];
}

void or_collective(const or_run* R, double* out)
{
    const int n = R->n;
    cplx J0[9], J1[9], J2[9], J3[9];
    moments_at(R, R->r, R->y, J0, J1, J2, J3);
    for (int j = 0; j < R->na; ++j) {
        cplx C[9];
        collective(R, J0, J1, J2, J3, j, C);
        write_moments(C, out + (size_t)j * n * n * 2, n);
    }
}

/* ------------------------------------------------------------ integrators */
/* Optional projection of every beam back to unit norm |psi|^2 = 1 (the scheme
 * of the FP32-amplitude forms, which renormalise after each accepted step). */
static void renormalize(or_run* R)
{
    const int n = R->n;
    OR_PARALLEL_FOR
    for (int64_t b = 0; b < R->nb; ++b) {
        double s = 0.0;
        for (int a = 0; a < n; ++a) {
            cplx z = amp(R, R->y, b, a);
            s += z.re * z.re + z.im * z.im;
        }
        double f = 1.0 / sqrt(s);
        for (int a = 0; a < 2 * n; ++a) R->y[b * 2 * n + a] *= f;
    }
}

/* Y = y + h * sum_{i < m} a[i] k[i]  (coefficient sum first, ascending i). */
static void stage_state(const or_run* R, const double* y, double h, const double* a, int m, double* Y)
{
    OR_PARALLEL_FOR
    for (int64_t q = 0; q < R->ylen; ++q) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += a[i] * R->k[i][q];
        Y[q] = y[q] + h * acc;
    }
}

/* Classic fourth-order Runge-Kutta with N equal steps from r_start to r_end;
 * step n starts at r_start + n h, h = (r_end - r_start) / N. */
int or_step_rk4(or_run* R, int64_t nsteps)
{
    static const double A[4][3] = {{0, 0, 0}, {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 1.0}};
    static const double C[4] = {0.0, 0.5, 0.5, 1.0};
    static const double B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double h = (R->p.r_end_km - R->p.r_start_km) / (double)R->p.n_fixed_steps;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (R->istep >= R->p.n_fixed_steps) { R->done = 1; return OR_DONE; }
        const double r = R->p.r_start_km + (double)R->istep * h;
        for (int i = 0; i < 4; ++i) {
            stage_state(R, R->y, h, A[i], i, R->ytmp);
            rhs(R, r + C[i] * h, R->ytmp, R->k[i]);
        }
        stage_state(R, R->y, h, B, 4, R->ytmp);
        memcpy(R->y, R->ytmp, sizeof(double) * (size_t)R->ylen);
        if (R->p.renormalize) renormalize(R);
        R->istep += 1;
        R->nacc += 1;
        R->r = R->p.r_start_km + (double)R->istep * h;
        R->h = h;
        for (int64_t q = 0; q < R->ylen; ++q)
            if (!isfinite(R->y[q])) return OR_NONFINITE;
    }
    return OR_OK;
}

/* Dormand & Prince (1980) RK5(4)7M coefficients. */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
/* e = b(5th order) - b(4th order) */
static const double DP_E[7] = {71.0 / 57600.0, 0.0, -71.0 / 16695.0, 71.0 / 1920.0,
                               -17253.0 / 339200.0, 22.0 / 525.0, -1.0 / 40.0};

void or_dp54_tableau(double* c, double* a, double* e)
{
    for (int i = 0; i < 7; ++i) {
        c[i] = DP_C[i];
        e[i] = DP_E[i];
        for (int j = 0; j < 6; ++j) a[i * 6 + j] = DP_A[i][j];
    }
}

/* One attempt of the embedded pair with the controller of readings J and K. */
static int dp54_attempt(or_run* R)
{
    const int64_t namp = 2 * (int64_t)R->n * R->nb;
    const double r = R->r, h = R->h;
    if (!R->k1_valid) { rhs(R, r, R->y, R->k[0]); R->k1_valid = 1; }
    for (int i = 1; i < 7; ++i) {
        stage_state(R, R->y, h, DP_A[i], i, R->ytmp);
        rhs(R, r + DP_C[i] * h, R->ytmp, R->k[i]);
    }
    /* ytmp now holds stage 7 = the 5th-order solution (a_7j = b_j). */
    double err = 0.0;
    int finite = 1;
    /* (the maximum is exact, so a parallel reduction of it changes nothing) */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(max : err) reduction(& : finite)
#endif
    for (int64_t q = 0; q < namp; ++q) {
        double acc = 0.0;
        for (int i = 0; i < 7; ++i) acc += DP_E[i] * R->k[i][q];
        double d = fabs(h * acc) / R->p.rtol;
        if (!isfinite(d)) finite = 0;
        else if (d > err) err = d;
    }
    if (!finite) return OR_NONFINITE;
    R->last_err = err;

    const double fmin = 0.2, fmax = 5.0;
    double fac;
    if (err <= 1.0) {
        memcpy(R->y, R->ytmp, sizeof(double) * (size_t)R->ylen);
        memcpy(R->k[0], R->k[6], sizeof(double) * (size_t)R->ylen);
        if (R->p.renormalize) { renormalize(R); R->k1_valid = 0; }
        R->r = r + h;
        R->nacc += 1;
        fac = (err == 0.0) ? fmax : R->p.safety * pow(err, -0.2);
        if (fac > fmax) fac = fmax;
        if (fac < fmin) fac = fmin;
        if (R->last_rejected && fac > 1.0) fac = 1.0;
        R->last_rejected = 0;
    } else {
        R->nrej += 1;
        fac = R->p.safety * pow(err, -0.2);
        if (fac < fmin) fac = fmin;
        R->last_rejected = 1;
    }
    /* The underflow test applies to the controller's proposal; the clip to
     * r_end may legitimately leave a last step of any size. */
    double hn = h * fac;
    if (hn > R->p.dr_max_km) hn = R->p.dr_max_km;
    if (R->r >= R->p.r_end_km) { R->done = 1; R->h = hn; return OR_DONE; }
    if (hn < 1e-14 * R->r) { R->h = hn; return OR_UNDERFLOW; }
    if (R->r + hn > R->p.r_end_km) hn = R->p.r_end_km - R->r;
    R->h = hn;
    return OR_OK;
}

int or_step_dp54(or_run* R, int64_t nattempts)
{
    for (int64_t s = 0; s < nattempts; ++s) {
        if (R->done) return OR_DONE;
        int st = dp54_attempt(R);
        if (st != OR_OK) return st;
    }
    return OR_OK;
}

int or_evolve_dp54(or_run* R, double r_target, int64_t max_attempts)
{
    double save_end = R->p.r_end_km;
    if (r_target < save_end) R->p.r_end_km = r_target;
    if (R->r + R->h > R->p.r_end_km) R->h = R->p.r_end_km - R->r;
    int st = OR_OK;
    for (int64_t s = 0; (max_attempts <= 0 || s < max_attempts); ++s) {
        if (R->r >= R->p.r_end_km) { st = OR_DONE; break; }
        st = dp54_attempt(R);
        if (st != OR_OK) break;
    }
    R->p.r_end_km = save_end;
    if (R->r < save_end) R->done = 0;
    return st;
}

/* ------------------------------------------------------------ exponential stepper */
/* U = exp(-i K t) of a Hermitian n x n matrix K (row-major), taken from the
 * definition: the power series of exp(X), X = -i K t / 2^m, with m chosen so
 * that the 1-norm of X is at most 1/2, summed until a term no longer changes
 * the sum, then squared m times. */
static void expm_herm(int n, const cplx* K, double t, cplx* U)
{
    double norm = 0.0;
    for (int c = 0; c < n; ++c) {
        double col = 0.0;
        for (int a = 0; a < n; ++a) col += hypot(K[a * n + c].re, K[a * n + c].im);
        if (col > norm) norm = col;
    }
    norm *= fabs(t);
    int m = 0;
    while (norm > 0.5) { norm *= 0.5; ++m; }
    const double scale = ldexp(t, -m);
    cplx X[9], term[9], next[9];
    for (int i = 0; i < n * n; ++i) {
        X[i] = c_make(K[i].im * scale, -K[i].re * scale); /* -i K t / 2^m */
        term[i] = c_make(0, 0);
    }
    for (int a = 0; a < n; ++a) term[a * n + a] = c_make(1, 0);
    for (int i = 0; i < n * n; ++i) U[i] = term[i];
    for (int k = 1; k < 60; ++k) {
        double big = 0.0;
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c) {
                cplx acc = c_make(0, 0);
                for (int q = 0; q < n; ++q) acc = c_add(acc, c_mul(term[a * n + q], X[q * n + c]));
                next[a * n + c] = c_scale(acc, 1.0 / (double)k);
                double v = fabs(next[a * n + c].re) + fabs(next[a * n + c].im);
                if (v > big) big = v;
            }
        for (int i = 0; i < n * n; ++i) { term[i] = next[i]; U[i] = c_add(U[i], term[i]); }
        if (big < 1e-18) break;
    }
    for (int s = 0; s < m; ++s) {
        cplx sq[9];
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c) {
                cplx acc = c_make(0, 0);
                for (int q = 0; q < n; ++q) acc = c_add(acc, c_mul(U[a * n + q], U[q * n + c]));
                sq[a * n + c] = acc;
            }
        for (int i = 0; i < n * n; ++i) U[i] = sq[i];
    }
}

void or_expm_herm(int n, const double* k, double t, double* u)
{
    cplx K[9] = {{0, 0}}, U[9];
    if (n < 2 || n > 3) return;
    for (int i = 0; i < n * n; ++i) K[i] = c_make(k[2 * i], k[2 * i + 1]);
    expm_herm(n, K, t, U);
    for (int i = 0; i < n * n; ++i) { u[2 * i] = U[i].re; u[2 * i + 1] = U[i].im; }
}

/* One exponential step of every beam (eq 3.10-3.12, lab frame) of radial
 * length dr from radius r_from to r_to:
 *   out_b = exp(-i H_b dl_j) x_b,  dl_j = dr / ((c_j(r_from) + c_j(r_to)) / 2),
 * the path length of trajectory j across the step from the mean of its
 * cosines at the two ends (Appendix A.4.3; eq 3.3).  dr is the step itself,
 * not r_to - r_from, which loses digits when the step is small against r.  The Hamiltonian of beam
 * b is formed at radius r_h from the moments of state ymom (eq 3.13 and 3.4,
 * as in rhs() with Phi = 0):
 *   neutrino      H  = H_vac(E) + H_m(r_h) + H_nunu
 *   antineutrino  Hb = conj(H_vac(E)) - H_m(r_h) - conj(H_nunu).
 * The phase part of the flat state is copied from x unchanged (zero in the
 * lab frame). */
static void exp_step(const or_run* R, double r_h, const double* ymom, double r_from, double r_to, double dr,
                     const double* x, double* out)
{
    const int n = R->n, ne = R->ne, na = R->na;
    cplx J0[9], J1[9], J2[9], J3[9];
    double* cf = (double*)malloc(sizeof(double) * (size_t)na * 2);
    double* ct = cf + na;
    double* wtmp = (double*)malloc(sizeof(double) * (size_t)na);
    geometry(R, r_from, cf, wtmp);
    geometry(R, r_to, ct, wtmp);
    free(wtmp);
    moments_at(R, r_h, ymom, J0, J1, J2, J3); /* also leaves c_j(r_h), w_j(r_h) in R->c, R->w */
    const double lam = matter_potential(R, r_h);
    for (int j = 0; j < na; ++j) {
        const double dl = dr / (0.5 * (cf[j] + ct[j]));
        cplx C[9];
        collective(R, J0, J1, J2, J3, j, C);
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < ne; ++k) {
                const cplx* hv = &R->hvac[(size_t)k * n * n];
                cplx H[9], U[9];
                for (int a = 0; a < n; ++a)
                    for (int c = 0; c < n; ++c) {
                        const double hm = (a == c) ? lam * ((a == 0 ? 1.0 : 0.0) - 1.0 / (double)n) : 0.0;
                        if (s == 0)
                            H[a * n + c] = c_add(c_add(hv[a * n + c], c_make(hm, 0.0)), C[a * n + c]);
                        else
                            H[a * n + c] = c_sub(c_sub(c_conj(hv[a * n + c]), c_make(hm, 0.0)), c_conj(C[a * n + c]));
                    }
                expm_herm(n, H, dl, U);
                const int64_t b = (int64_t)(s * na + j) * ne + k;
                for (int a = 0; a < n; ++a) {
                    cplx acc = c_make(0, 0);
                    for (int c = 0; c < n; ++c) acc = c_add(acc, c_mul(U[a * n + c], amp(R, x, b, c)));
                    out[(b * n + a) * 2 + 0] = acc.re;
                    out[(b * n + a) * 2 + 1] = acc.im;
                }
            }
    }
    free(cf);
    for (int64_t q = 2 * (int64_t)n * R->nb; q < R->ylen; ++q) out[q] = x[q];
}

static void average(const or_run* R, const double* a, const double* b, double* out)
{
    for (int64_t q = 0; q < R->ylen; ++q) out[q] = 0.5 * (a[q] + b[q]);
}

/* One attempt of the paper's own stepper (Section 4.2.3 and the evolution
 * loop of Section 5; reading Q).  From psi0 at r with step h:
 *   H0 from psi0 at r;      psi1 = U(H0; r, r+h) psi0,  psi4 = U(H0; r, r+h/2) psi0
 *   H1 from psi1 at r+h;    H2 from psi4 at r+h/2
 *   psi3 = (psi1 + U(H1; r, r+h) psi0) / 2              full-step estimate
 *   psi5 = U(H2; r+h/2, r+h) psi4;  H3 from psi5 at r+h
 *   psi7 = (psi1 + U(H3; r, r+h) psi0) / 2              two-half-step estimate
 * with U(H; r_a, r_b) the exponential step of exp_step() from r_a to r_b (path
 * length from the mean cosine of its two ends).  Both estimates are second order and
 * differ only through the predicted end Hamiltonian (H1 from one full step,
 * H3 from two half steps), so psi3 - psi7 = O(h^3).  The error is the maximum
 * over beams, components and re/im parts of |psi3 - psi7| / rtol; an accepted
 * attempt advances to psi7.  Controller as reading J with the exponent of a
 * third-order local error: factor safety * err^(-1/3), clamped to [0.2, 5]. */
static int exp_attempt(or_run* R)
{
    const int64_t namp = 2 * (int64_t)R->n * R->nb;
    const double r = R->r, h = R->h;
    double *psi1 = R->k[0], *psi2 = R->k[1], *psi3 = R->k[2], *psi4 = R->k[3], *psi5 = R->k[4], *psi6 = R->k[5],
           *psi7 = R->k[6];
    const double rm = r + 0.5 * h, re = r + h;
    exp_step(R, r, R->y, r, re, h, R->y, psi1);
    exp_step(R, r, R->y, r, rm, 0.5 * h, R->y, psi4);
    exp_step(R, re, psi1, r, re, h, R->y, psi2);
    average(R, psi1, psi2, psi3);
    exp_step(R, rm, psi4, rm, re, 0.5 * h, psi4, psi5);
    exp_step(R, re, psi5, r, re, h, R->y, psi6);
    average(R, psi1, psi6, psi7);

    double err = 0.0;
    int finite = 1;
    for (int64_t q = 0; q < namp; ++q) {
        double d = fabs(psi3[q] - psi7[q]) / R->p.rtol;
        if (!isfinite(d)) finite = 0;
        else if (d > err) err = d;
    }
    if (!finite) return OR_NONFINITE;
    R->last_err = err;

    const double fmin = 0.2, fmax = 5.0;
    double fac;
    if (err <= 1.0) {
        memcpy(R->y, psi7, sizeof(double) * (size_t)R->ylen);
        if (R->p.renormalize) renormalize(R);
        R->r = r + h;
        R->nacc += 1;
        fac = (err == 0.0) ? fmax : R->p.safety * pow(err, -1.0 / 3.0);
        if (fac > fmax) fac = fmax;
        if (fac < fmin) fac = fmin;
        if (R->last_rejected && fac > 1.0) fac = 1.0;
        R->last_rejected = 0;
    } else {
        R->nrej += 1;
        fac = R->p.safety * pow(err, -1.0 / 3.0);
        if (fac < fmin) fac = fmin;
        R->last_rejected = 1;
    }
    double hn = h * fac;
    if (hn > R->p.dr_max_km) hn = R->p.dr_max_km;
    if (R->r >= R->p.r_end_km) { R->done = 1; R->h = hn; return OR_DONE; }
    if (hn < 1e-14 * R->r) { R->h = hn; return OR_UNDERFLOW; }
    if (R->r + hn > R->p.r_end_km) hn = R->p.r_end_km - R->r;
    R->h = hn;
    return OR_OK;
}

int or_step_exp(or_run* R, int64_t nattempts)
{
    if (R->p.frame != 1) return OR_INVALID;
    for (int64_t s = 0; s < nattempts; ++s) {
        if (R->done) return OR_DONE;
        int st = exp_attempt(R);
        if (st != OR_OK) return st;
    }
    return OR_OK;
}

int or_evolve_exp(or_run* R, double r_target, int64_t max_attempts)
{
    if (R->p.frame != 1) return OR_INVALID;
    double save_end = R->p.r_end_km;
    if (r_target < save_end) R->p.r_end_km = r_target;
    if (R->r + R->h > R->p.r_end_km) R->h = R->p.r_end_km - R->r;
    int st = OR_OK;
    for (int64_t s = 0; (max_attempts <= 0 || s < max_attempts); ++s) {
        if (R->r >= R->p.r_end_km) { st = OR_DONE; break; }
        st = exp_attempt(R);
        if (st != OR_OK) break;
    }
    R->p.r_end_km = save_end;
    if (R->r < save_end) R->done = 0;
    return st;
}

/* ------------------------------------------------------------ output */
void or_probabilities(const or_run* R, double* p)
{
    for (int64_t b = 0; b < R->nb; ++b) {
        cplx z = amp(R, R->y, b, 0);
        p[b] = z.re * z.re + z.im * z.im;
    }
}

/* Energy-averaged flavor content of every trajectory: the second dump mode
 * of Section 4.2.4 (the flavor state of one trajectory averaged over its
 * energy bins).  Reading O: each bin counts with the number flux of the
 * beam's birth flavor in it (nu_e for neutrino beams, nubar_e for
 * antineutrino beams; spectra eq 4.1-4.2 with the luminosities of reading C),
 * and a species whose flux is zero gets the plain mean over bins:
 *   out[s][j][a] = sum_k f_sk |psi_{s,j,k,a}|^2 / sum_k f_sk. */
void or_energy_average(const or_run* R, double* out)
{
    const or_params* p = &R->p;
    const double de = (p->e_max_mev - p->e_min_mev) / (double)R->ne;
    for (int s = 0; s < 2; ++s) {
        /* species s = 0: nu_e (index 0 of the luminosities), s = 1: nubar_e */
        const double f2 = or_fermi_integral(2, p->eta[s]);
        const double temp = p->mean_e_mev[s] * f2 / or_fermi_integral(3, p->eta[s]);
        const double nrel = (p->lum_erg_s[s] / LREF_ERG_S) * (EREF_MEV / p->mean_e_mev[s]);
        for (int j = 0; j < R->na; ++j)
            for (int a = 0; a < R->n; ++a) {
                double num = 0.0, den = 0.0, plain = 0.0;
                for (int k = 0; k < R->ne; ++k) {
                    const double e = p->e_min_mev + ((double)k + 0.5) * de;
                    const double f = de * nrel * spectrum(e, temp, p->eta[s], f2);
                    const cplx z = amp(R, R->y, ((int64_t)s * R->na + j) * R->ne + k, a);
                    const double prob = z.re * z.re + z.im * z.im;
                    num += f * prob;
                    den += f;
                    plain += prob;
                }
                out[((size_t)s * R->na + j) * R->n + a] = den != 0.0 ? num / den : plain / (double)R->ne;
            }
    }
}

double or_last_error(const or_run* R) { return R->last_err; }

void or_stats(const or_run* R, int64_t* accepted, int64_t* rejected, double* r, double* dr)
{
    if (accepted) *accepted = R->nacc;
    if (rejected) *rejected = R->nrej;
    if (r) *r = R->r;
    if (dr) *dr = R->h;
}
