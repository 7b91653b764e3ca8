// Internal interface between the host runtime (nuosc_runtime.cpp) and the
// gfx950 kernels (nuosc_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nuosc {

// Device control block of one run.  Two copies live on the device: ctrl[1] is
// the state between attempts (the host reads and writes it; the stage-0
// kernels and the first stage kernel of an attempt read it), ctrl[0] the copy
// the rest of an attempt reads.  The first stage kernel of an attempt copies
// ctrl[1] into ctrl[0]; the control kernel after the last stage writes the
// updated block into ctrl[1].  No kernel reads a copy that a workgroup of the
// same launch writes.
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
// upper triangle (a < b, row-major) as (re, im) pairs, n*n reals in total.
template <int N> struct Shape {
    static constexpr int NU = N * (N - 1) / 2;  // upper off-diagonal entries
    static constexpr int NM = N * N;            // reals of a packed Hermitian matrix
    __host__ __device__ static constexpr int up(int a, int b) { return a * N - a * (a + 1) / 2 + (b - a - 1); }
};

// Stage matrix of one trajectory in the co-rotating frame, K = A + B u with
// u = +1/E for neutrinos and u = -1/E for antineutrinos (whose amplitudes are
// held complex-conjugated on the device).  Packed Hermitian, h A then h B (the
// attempt's step size folded in), in the arithmetic type T of the stage
// kernels.  Written by the beam launch that
// completes the stage, read by the later beam launches of the same attempt.
template <typename T, int N> struct alignas(16) StageMat {
    T a[Shape<N>::NM];
    T b[Shape<N>::NM];
};
constexpr size_t kStageMatBytes = sizeof(StageMat<double, 3>);

// FP64 geometry and frame data of one trajectory at one stage radius.
struct TrajGeo {
    double c, w, wc, ic;  // cos(theta), angle weight w, w*c (0 single angle), 1/c
    double P[3];          // phase sum sum_{m < l} coef(l, m) G_m of stage l, G_m = d Phi / dr of
                          // the co-rotating frame at stage m (accumulated by the beam launches)
    double z[3][2];       // e^{i(Phi_a - Phi_b)}, upper pairs
};

// Everything a kernel needs about a run, passed by value.
struct RunConst {
    int32_t n, ne, na, ma;       // flavors, energy bins, trajectories, multi-angle flag
    int64_t nb, nb_pad;          // beams, padded stride of one component array
    int32_t frame, precision, integrator, nblk;  // nblk: stage workgroups (partials)
    int32_t np, nj;              // azimuth bins per emission angle (1: bulb model); angle moments (2 or 4)
    int32_t nth, pad2;           // emission-angle bins (na / np)
    double r_nu, mu0, lambda0, lambda_rref, lambda_power;
    double rtol, safety, dr_max;
    double r_start, h_fixed;
    int64_t n_fixed, max_steps;
    double vac[3][3][2];         // H_vac(E) = vac * (1/E), traceless, complex
    // device buffers
    void* psi[2];                // state buffers: [2n][nb_pad] of the storage type
    double* phase[2];            // [na][n]
    const double* uinv64;        // [2 ne] signed 1/E per beam slot of a trajectory
    const float* uinv32;         // [2 ne] the same in FP32
    const double* wgt;           // [2 ne] g (neutrino slots), -gbar (antineutrino slots)
    const double* flux;          // [2 ne] number flux of the slot's birth flavor in its energy bin
    const double* azi;           // [na][2] cos, sin of each trajectory's azimuth
    double* jhist;               // [kMaxStages + 1][nj n n] packed J0, J1 (J2, J3) per stage
    double* partial;             // [2][nj n n][nblk] per-workgroup weighted sums of the last two
                                 // beam launches (launch I uses [I & 1]), value-major
    double* errpart;             // [nblk]
    void* errv;                  // [2n][nb_pad] of the arithmetic type: sum_{i<S-1} e_i k_i of
                                 // an embedded first-same-as-last pair (else unused)
    double* xbuf;                // [2][2n][nb_pad] FP64: psi1 and psi4 of the exponential stepper's
                                 // attempt (else unused)
    void* mat;                   // [kMaxStages][na] StageMat<T, n>
    TrajGeo* geo;                // [kMaxStages + 1][na]
    Control* ctrl;               // [2]
};

constexpr int kMaxStages = 8;
constexpr int kFinBlock = 256;     // threads per control / prepare workgroup

// Trajectories per beam workgroup (one partial density sum each): 16 for the
// FP32-arithmetic form, 8 for the FP64-arithmetic forms.
inline int traj_per_block(int precision) { return precision == 1 ? 16 : 8; }

// The runs one launch covers.  Run i of the launch is runs[slot[i]] and owns
// the workgroups [first[i], first[i + 1]); a workgroup never spans two runs,
// so every run computes exactly what it would alone.  All runs of a launch
// share the flavor count, precision and integrator (template parameters).
constexpr int kMaxRuns = 64;
struct LaunchSet {
    const RunConst* runs;          // device array of run constants
    int32_t count;
    int32_t pad;
    int32_t slot[kMaxRuns];
    int32_t first[kMaxRuns + 1];
};

// Host view of the runs a launch covers: rc[i] is a host copy of the constants
// stored at runs_dev[slot[i]].
struct RunList {
    const RunConst* runs_dev;
    int count;
    const int* slot;
    const RunConst* const* rc;
};

// One stage of the current attempt of every listed run: the beam kernel
// (stage 0 = moments of the current state; stage == S = final launch),
// followed after stage 0 and stage S by the control kernel.  ev, if not null,
// receives three events: before the beam kernel, after it, and after the
// control kernel (if any).
hipError_t launch_stage(const RunList& runs, int stage, hipStream_t s, hipEvent_t* ev = nullptr);
// Geometry and frame factors of stage 0 for the current state (before a
// stage-0 launch).
hipError_t launch_prepare(const RunList& runs, hipStream_t s);
hipError_t launch_probabilities(const RunList& runs, double* p_dev, hipStream_t s);  // first run only
hipError_t launch_init_state(const RunList& runs, hipStream_t s);
// Energy-averaged flavor content [2][na][n] of the first listed run.
hipError_t launch_energy_average(const RunList& runs, double* out_dev, hipStream_t s);
int num_stages(int integrator);

// The paper's own stepper (exponential steps with averaging, lab frame, FP64):
// launch `stage` 1..kExpLaunches of an attempt (a beam kernel and a reduction
// kernel; the last reduction is the step control), or 0: J of the current
// state.  One run per call.  ev as for launch_stage.
constexpr int kExpLaunches = 3;
constexpr int kExpTrajPerBlock = 4;  // trajectories (wavefronts) per workgroup of its beam kernels
hipError_t launch_exp_stage(const RunList& runs, int stage, hipStream_t s, hipEvent_t* ev = nullptr);

}  // namespace nuosc
