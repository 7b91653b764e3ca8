// Internal interface between the host runtime (nuosc_runtime.cpp) and the
// gfx950 kernels (nuosc_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nuosc {

// Device control block of one run.  Kernels read r, h and cur at entry; only
// the last workgroup of the final stage kernel of a step writes it.
struct Control {
    double r;          // radius of the current accepted state y_n
    double h;          // step of the next attempt (clipped to r_end)
    double h_prop;     // controller proposal before the clip to r_end
    double r_end;      // radius the current evolve call stops at
    double err;        // scaled error of the last attempt
    int64_t nacc, nrej, attempts, istep;
    int32_t cur;            // state buffer holding y_n (0/1)
    int32_t last_rejected;
    int32_t status;         // 0 running, 1 reached r_end, <0 nuosc_status error
    int32_t pad;
};

// Packed Hermitian n x n matrix: n real diagonal entries followed by the
// upper triangle (a < b, row-major) as (re, im) pairs: n*n doubles in total.
template <int N> struct Herm { static constexpr int size = N * N; };

// FP64 Hamiltonian pieces of one trajectory at one stage of the current
// attempt, written by the launch that completes the stage and read by later
// launches of the same attempt.  A, B: K~ = A + B / E of neutrinos, packed as
// n real diagonal entries then the upper triangle (re, im).
struct TrajStage {
    double c, w;        // propagation cosine and angle weight at the stage radius
    double G[3];        // d Phi / dr of the co-rotating frame
    double phi[3];      // stage phase
    double z[3][2];     // e^{i(phi_a - phi_b)}, upper pairs
    double A[9];
    double B[9];
};

// Everything a kernel needs about a run, passed by value.
struct RunConst {
    int32_t n, ne, na, ma;       // flavors, energy bins, trajectories, multi-angle flag
    int64_t nb, nb_pad;          // beams, padded stride of one component array
    int32_t frame, precision, integrator, pad0;
    double r_nu, mu0, lambda0, lambda_rref, lambda_power;
    double rtol, safety, dr_max;
    double r_start, h_fixed;
    int64_t n_fixed, max_steps;
    double vac[3][3][2];         // H_vac(E) = vac * (1/E), traceless, complex
    // device buffers
    void* psi[2];                // state buffers: [2n][nb_pad] of T
    double* phase[2];            // [na][n]
    const double* inv_e;         // [ne]
    const double* g;             // [ne]  neutrino weights
    const double* gbar;          // [ne]  antineutrino weights
    double* jhist;               // [8][2][n*n] packed J0, J1 per stage
    double* partial;             // [na][2*n*n] per-trajectory weighted sums
    double* errpart;             // [na]
    TrajStage* tab;              // [kMaxStages][na]
    Control* ctrl;
    unsigned* counter;           // [2] last-block counters
};

constexpr int kBlock = 256;
constexpr int kMaxStages = 8;

// Launch the kernel that forms stage `stage` of the current attempt (stage 0 =
// moments of the current state; stage == S = final: new state, error, control).
hipError_t launch_stage(const RunConst& rc, int stage, hipStream_t s);
hipError_t launch_probabilities(const RunConst& rc, double* p_dev, hipStream_t s);
hipError_t launch_init_state(const RunConst& rc, hipStream_t s);
int num_stages(int integrator);

}  // namespace nuosc
