/*
 * Oracle for the bulb-model neutrino flavor evolution -- TEST INFRASTRUCTURE.
 *
 * A plain, slow FP64 CPU implementation written directly from the paper's
 * statement of the problem (Noormofidi, arXiv 1907.05560, Ch. 3 and 4).  It
 * exists only to check the HIP path: only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the library under paper_1907_05560_amd/.
 *
 * Units: radius r in km, Hamiltonians in km^-1, energies in MeV, mass-squared
 * differences in eV^2.
 */
#ifndef NUOSC_ORACLE_H
#define NUOSC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_flavors;      /* 2 or 3 */
    int32_t n_energy;       /* energy bins */
    double  e_min_mev, e_max_mev;
    int32_t n_angle;        /* emission-angle bins; 0 => single-angle model */
    double  lum_erg_s[4];   /* nu_e, nubar_e, nu_x, nubar_x */
    double  mean_e_mev[4];
    double  eta[4];
    double  dm2_ev2, theta;                                  /* two flavors */
    double  dm2_21_ev2, dm2_31_ev2, theta12, theta13, theta23, delta_cp; /* three */
    double  lambda0_km, lambda_rref_km, lambda_power;
    double  mu0_km, r_nu_km;
    double  r_start_km, r_end_km;
    int32_t integrator;     /* 0 classic RK4 fixed step, 1 Dormand-Prince 5(4),
                               2 the paper's exponential stepper (lab frame) */
    int64_t n_fixed_steps;
    double  rtol, dr_init_km, dr_max_km, safety;
    int32_t frame;          /* 0 co-rotating, 1 lab */
    int32_t renormalize;    /* 1: rescale every beam to unit norm after each
                               accepted step (the FP32-amplitude scheme) */
    int32_t n_azimuth;      /* azimuth bins per emission angle: the extended
                               bulb model (eq 3.18); 0 or 1: the bulb model */
    int32_t sum_mode;       /* order and kind of the moment sums (eq 3.8, 3.13):
                               0 plain sums, energies then trajectories
                               ascending (the reference); 1 the same order with
                               compensated (Neumaier) sums; 2 plain sums in
                               descending order; 3 compensated, descending.
                               Modes 1-3 exist to measure how much of a run's
                               sensitivity is summation rounding. */
} or_params;

typedef struct or_run or_run;

/* Status codes returned by the stepping functions. */
enum { OR_OK = 0, OR_DONE = 1, OR_NONFINITE = -4, OR_UNDERFLOW = -5, OR_INVALID = -1 };

or_run* or_create(const or_params* p);
void    or_destroy(or_run* R);

int64_t or_num_beams(const or_run* R);
int32_t or_num_traj(const or_run* R);   /* angle trajectories (1 for single angle) */

/* State, host layout: psi[a][2][b] (flavor component a, re/im, beam b) and
 * phase[j][a] (co-rotating phase of trajectory j, component a). */
int  or_get_state(const or_run* R, double* psi, double* phase);
int  or_set_state(or_run* R, const double* psi, const double* phase, double r_km);

/* J0 and J1 (n*n complex each, row-major, interleaved re/im) of the current
 * state at the current radius. */
void or_moments(const or_run* R, double* j0, double* j1);
/* the extended model's azimuth moments J2 = sum w s cos(phi) S, J3 = sum w s sin(phi) S */
void or_moments_azimuth(const or_run* R, double* j2, double* j3);
/* azimuth angle phi_j of every trajectory (0 for the bulb model) */
void or_azimuth(const or_run* R, double* phi);
/* Collective Hamiltonian H_nunu for every trajectory in the lab frame for the
 * current state: out[j][a][b] complex (interleaved). */
void or_collective(const or_run* R, double* out);
/* Right-hand side d/dr of the flat state (psi then phases) at radius r. */
void or_rhs(const or_run* R, double r, const double* y, double* dydr);
int64_t or_state_len(const or_run* R);

int  or_step_rk4(or_run* R, int64_t nsteps);            /* fixed-step RK4 */
int  or_step_dp54(or_run* R, int64_t nattempts);        /* adaptive attempts */
int  or_evolve_dp54(or_run* R, double r_target, int64_t max_attempts);
/* the paper's exponential stepper (reading Q); frame must be 1 (lab) */
int  or_step_exp(or_run* R, int64_t nattempts);
int  or_evolve_exp(or_run* R, double r_target, int64_t max_attempts);
/* u = exp(-i k t) of a Hermitian n x n matrix k (row-major, interleaved re/im) */
void or_expm_herm(int n, const double* k, double t, double* u);

void or_probabilities(const or_run* R, double* p);      /* |psi_1|^2 per beam */
/* energy-averaged flavor content [2 species][na][n] (reading O) */
void or_energy_average(const or_run* R, double* out);
void or_stats(const or_run* R, int64_t* accepted, int64_t* rejected, double* r, double* dr);
double or_last_error(const or_run* R);  /* scaled error of the last adaptive attempt */
int    or_num_threads(void);              /* threads of the parallel loops: 1 unless built with OpenMP */

/* Tables and pieces, exposed for the tests. */
double or_fermi_integral(int k, double eta);
double or_temperature(double mean_e, double eta);
double or_spectrum(double e, double temperature, double eta);
double or_dilution(double x);                                /* D(r/R), eq 3.17 */
void   or_geometry(const or_run* R, double r, double* c, double* w);
void   or_tables(const or_run* R, double* energy, double* g, double* gbar, double* hvac);
double or_vacuum_coefficient(void);                          /* km^-1 MeV / eV^2 */
/* Dormand-Prince tableau as used: c[7], a[7][6] (row 7 = 5th-order weights),
 * e[7] = 5th-order minus 4th-order weights. */
void   or_dp54_tableau(double* c, double* a, double* e);

#ifdef __cplusplus
}
#endif
#endif
