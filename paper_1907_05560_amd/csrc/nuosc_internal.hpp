// Internal interface between the host runtime (nuosc_runtime.cpp) and the
// gfx950 kernels (nuosc_kernels.hip, nuosc_exp.hip).  Not part of the public
// C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nuosc {

// Device control block of one run.  Two copies live on the device: ctrl[1] is
// the state between attempts (the host reads and writes it; the first launch
// of an attempt reads it), ctrl[0] the copy the rest of an attempt reads.  The
// first launch of an attempt copies ctrl[1] into ctrl[0]; the last launch
// (step control) writes the updated block into ctrl[1].  No kernel reads a
// copy that a workgroup of the same launch writes.
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
    int32_t fresh;          // Runge-Kutta forms: J of y_n is still in the moment partials of the
                            // power-moment launch (the next attempt's first launch sums them)
};

// Packed Hermitian n x n matrix: n real diagonal entries followed by the
// upper triangle (a < b, row-major) as (re, im) pairs, n*n reals in total.
template <int N> struct Shape {
    static constexpr int NU = N * (N - 1) / 2;  // upper off-diagonal entries
    static constexpr int NM = N * N;            // reals of a packed Hermitian matrix
    static constexpr int NC = 2 * N * N;        // reals of a full complex matrix (row-major, re/im)
    __host__ __device__ static constexpr int up(int a, int b) { return a * N - a * (a + 1) / 2 + (b - a - 1); }
};

// Everything a kernel needs about a run, passed by value.
struct RunConst {
    int32_t n, ne, na, ma;       // flavors, energy bins, trajectories, multi-angle flag
    int64_t nb, nb_pad;          // beams, padded stride of one component array
    int32_t frame, precision, integrator, nblk;  // nblk: workgroups that write moment partials
    int32_t np, nj;              // azimuth bins per emission angle (1: bulb model); angle moments (2 or 4)
    int32_t nth, nblkf;          // emission-angle bins (na / np); workgroups of the state-update launch
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
    const double* geo;           // [na][4] multi-angle trajectories: u^2, 1 - u^2, u du / np, 0 (u: the
                                 // emission cosine of the trajectory's bin, du = 1 / nth)
    double* jhist;               // [kMaxStages + 1][nj n n] packed J0, J1 (J2, J3) per stage
    double* partial;             // [2][nj n n][pstride] per-workgroup weighted sums of the last two
                                 // moment launches (launch l uses [l & 1]), value-major
    double* errpart;             // [max(nblk, nblkf)] per-workgroup step-error maxima
    double* qbuf;                // Runge-Kutta forms: [na][qstride] power moments of the current state as
                                 // full complex matrices (rewritten only when a new state is accepted)
    double* dbuf;                // [na][dstride] stage-derivative coefficient matrices of the attempt
    double* gbuf;                // [na][kMaxStages][n] co-rotating frame rates of the attempt's stages
    double* zbuf;                // [na][8] rotation factors (cos, sin per upper pair) of the stage the
                                 // last stage launch formed
    void* ftab;                  // [na][fstride bytes] coefficients of the state update and the error
    double* xbuf;                // [2][2n][nb_pad] FP64: psi1 and psi4 of the exponential stepper's
                                 // attempt (else unused)
    Control* ctrl;               // [2]
    int32_t qstride, dstride;    // doubles per trajectory in qbuf, dbuf
    int32_t fstride;             // bytes per trajectory in ftab
    int32_t nblkp;               // workgroups of the power-moment launch (partials it writes)
    int32_t pstride;             // stride of one value in the partial buffer: max(nblk, nblkp)
    int32_t pad3;
};

constexpr int kMaxStages = 8;
constexpr int kMaxLaunches = 10;   // launches of one attempt (Runge-Kutta: stages + 2)
constexpr int kFinBlock = 256;     // threads per small reduction workgroup

// Trajectories per workgroup of the Runge-Kutta launches: the per-trajectory
// launches (16), the power-moment launch (16) and the state update (8).
constexpr int kTrajPerBlock = 16;
constexpr int kPowerTrajPerBlock = 16;  // the power-moment launch: two trajectories per wavefront
inline int final_traj_per_block(int) { return 8; }

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

// Sizes of the Runge-Kutta tables of a run (doubles per trajectory in qbuf and
// dbuf, bytes per trajectory in ftab).
struct PolySizes {
    int qstride, dstride, fstride;
};
PolySizes poly_sizes(int n, int integrator, int precision);

// Launch `stage` of the current attempt of every listed run (Runge-Kutta
// integrators): 1..S-1 the per-trajectory stage launches, S the completion of
// the last stage and the update coefficients, S+1 the state update, S+2 the
// step control and the power moments of the accepted state (S+2 launches per
// attempt, num_stages()); 0 the power moments and J of the current state
// (after a new state or radius).  ev, if not null, receives three events:
// before the launch's main kernel, after it, and after its second kernel (only
// launch 0 has one).
hipError_t launch_stage(const RunList& runs, int stage, hipStream_t s, hipEvent_t* ev = nullptr);
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

// Library-owned device memory for runs made without allocation: one array of
// kStaticScratchBytes per device, held until the process ends.  static_scratch
// gives the current device's index and the array's address on it (looked up
// once per device and cached).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(int* device, void** addr);

}  // namespace nuosc
