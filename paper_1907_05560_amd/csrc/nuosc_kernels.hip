// gfx950 kernels of the bulb-model flavor evolution: explicit Runge-Kutta
// attempts in stage-polynomial form.
//
// Within one attempt the Hamiltonian of stage l depends on the beams only
// through the global angle moments J_l (eq 3.13-3.17).  Once J_l is known,
// every beam of trajectory j obeys a linear map: the stage derivative is
// h k_l = -i h K_l(u) Y_l with K_l(u) = A_l + B_l u, where u = +1/E for
// neutrinos and u = -1/E for antineutrinos (held complex-conjugated, see
// below), A_l the per-trajectory collective and matter part and B_l the
// vacuum part divided by the propagation cosine.  Every stage input is
// therefore a matrix polynomial in u applied to y_n:
//   Y_l = C_l(u) y_n,   C_0 = 1,   C_l(u) = 1 + sum_{m<l} a_lm D_m(u),
//   h k_m = D_m(u) y_n, D_m(u) = -i h (A_m + B_m u) C_m(u),
// and so are the new state y_{n+1} = (1 + sum_m b_m D_m(u)) y_n and the
// embedded error h sum_m e_m k_m = (sum_m e_m D_m(u)) y_n.  The density sum of
// stage l over the energies of a trajectory needs only power moments of y_n:
//   sum_k w_k Y_k Y_k^+ = sum_{d,d'} C_{l,d} Q_{d+d'} C_{l,d'}^+,
//   Q_p = sum_k w_k u_k^p y_k y_k^+,   p = 0 .. 2(S-1).
// This is exact algebra on the Runge-Kutta stages (only the rounding order
// differs from forming every stage state).  One attempt of an S-stage tableau
// is S + 2 launches:
//   k_traj<l>, l = 1..S-1 (32 lanes per trajectory, no beam data): J_{l-1}
//     as the fixed-order sum of the previous launch's partials; completion of
//     stage l-1 (matter term, collective term, co-rotating frame rate, the
//     coefficient matrices D_{l-1}); the coefficients C_l and the stage-l
//     density sum from Q, rotated to the lab frame and weighted by the angle
//     weights of stage l (eq 3.14-3.15) into one partial per workgroup;
//   k_traj<S>: completion of the last stage and the coefficient tables of the
//     update polynomial (arithmetic type) and the error polynomial (FP64);
//   k_final (beam pass): y_{n+1} as power sums in u with the coefficients in
//     scalar registers, renormalisation of FP32 amplitudes, the error
//     polynomial in FP64, per-workgroup error maxima;
//   k_power (beam pass): global error maximum and the step controller (every
//     workgroup gets the same result); for an accepted attempt the power
//     moments of the new state and its J partials, which the next attempt's
//     first launch sums.
// The beams are read twice and written once per attempt.
//
// Antineutrino amplitudes are held complex-conjugated on the device.  With
// phi = conj(psibar), the antineutrino equation in the co-rotating frame reads
// d phi / dr = -i (A - B / E) phi with the neutrino's A and B, so one matrix
// pair per trajectory and stage serves both species (u = +1/E or -1/E per
// beam slot), and the density sum takes the same form w psi psi^dagger for
// both species with weight w = g or -gbar.
#include "nuosc_internal.hpp"
#include "nuosc_device.hpp"

#include <math.h>
#include <array>
#include <mutex>
#include <type_traits>
#include <utility>

// Device memory of runs made without allocation (nuosc_create_static): every
// device holds its own copy from module load until the process ends.
static __device__ __align__(256) unsigned char scratch[nuosc::kStaticScratchBytes];

namespace nuosc {
namespace {

// ------------------------------------------------------------------ tableaus
// Classic fourth-order Runge-Kutta.
struct TabRK4 {
    static constexpr int S = 4;
    static constexpr bool fsal = false;
    static constexpr bool embedded = false;
    static constexpr double C[8] = {0.0, 0.5, 0.5, 1.0};
    static constexpr double A[8][8] = {{0}, {0.5}, {0.0, 0.5}, {0.0, 0.0, 1.0}};
    static constexpr double B[8] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    static constexpr double E[8] = {0};
};

// Dormand-Prince RK5(4)7M: the last stage is the new state (first same as
// last), E = fifth-order minus fourth-order weights.
struct TabDP54 {
    static constexpr int S = 7;
    static constexpr bool fsal = true;
    static constexpr bool embedded = true;
    static constexpr double C[8] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
    static constexpr double A[8][8] = {
        {0},
        {1.0 / 5.0},
        {3.0 / 40.0, 9.0 / 40.0},
        {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0},
        {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0},
        {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0},
        {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
    static constexpr double B[8] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                                    -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
    static constexpr double E[8] = {71.0 / 57600.0, 0.0, -71.0 / 16695.0, 71.0 / 1920.0,
                                    -17253.0 / 339200.0, 22.0 / 525.0, -1.0 / 40.0};
};

// Degrees and table sizes of the stage polynomials of a tableau.
template <typename TAB>
struct Poly {
    static constexpr int S = TAB::S;
    static constexpr int NQ = 2 * (S - 1) + 1;          // power moments Q_0 .. Q_{NQ-1}
    // D_m has degree m + 1; the update 1 + sum b_m D_m and the error sum e_m D_m
    // have the degree of their last nonzero weight plus one
    static constexpr int last_nonzero(const double* w)
    {
        int d = -1;
        for (int m = 0; m < S; ++m)
            if (w[m] != 0.0) d = m;
        return d;
    }
    static constexpr int DN = last_nonzero(TAB::B) + 1;
    static constexpr int DE = TAB::embedded ? last_nonzero(TAB::E) + 1 : 0;
    // D_m occupies m + 2 coefficient matrices; offset of D_m in matrices
    __host__ __device__ static constexpr int doff(int m) { return m * (m + 3) / 2; }
    static constexpr int ND = doff(S - 1);               // stored: D_0 .. D_{S-2}
};

// ------------------------------------------------------------------ helpers
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Orders the LDS accesses of one wavefront (its own LDS region only).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Global-memory views of the beam arrays.  uniform_global(p) takes a
// wave-uniform pointer into a scalar register as a global-address-space
// pointer: loads and stores through it become global (not flat) operations
// with a scalar base and a 32-bit vector offset (every array indexed this way
// is below 4 GiB).
template <typename T> using global = __attribute__((address_space(1))) T;
// A (re, im) pair as one 16-byte value (a plain vector type, so that it can be
// read and written through any address space).
typedef double d2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ global<T>* uniform_global(T* p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return reinterpret_cast<global<T>*>(((uint64_t)hi << 32) | lo);
}

// The same view of any run buffer, and plain-data structs copied through it in
// 8-byte words.  Flat operations (generic pointers) also count against the LDS
// counter, and one still in flight makes every later wait for a global load a
// wait for all of them; global operations keep both counters apart.
template <typename T>
__device__ __forceinline__ global<T>* gview(T* p)
{
    return reinterpret_cast<global<T>*>(reinterpret_cast<uint64_t>(p));
}
template <typename T>
__device__ __forceinline__ T gload(const T* p)
{
    static_assert(sizeof(T) % 8 == 0, "8-byte words");
    constexpr int NW = (int)(sizeof(T) / 8);
    uint64_t w[NW];
    const global<const uint64_t>* s = reinterpret_cast<const global<const uint64_t>*>(reinterpret_cast<uint64_t>(p));
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = s[i];
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, const T& v)
{
    static_assert(sizeof(T) % 8 == 0, "8-byte words");
    constexpr int NW = (int)(sizeof(T) / 8);
    uint64_t w[NW];
    __builtin_memcpy(w, &v, sizeof(T));
    global<uint64_t>* d = reinterpret_cast<global<uint64_t>*>(reinterpret_cast<uint64_t>(p));
#pragma unroll
    for (int i = 0; i < NW; ++i) d[i] = w[i];
}

// Lane k < NV stores v[k] to dst[k]: NV values that every lane of the
// wavefront holds, written with one store instruction instead of NV.
template <int NV>
__device__ __forceinline__ void lane_scatter(global<double>* dst, const double (&v)[NV], int lane)
{
    if (lane < NV) {
        double x = v[0];
#pragma unroll
        for (int k = 1; k < NV; ++k) {
            x = (lane == k) ? v[k] : x;
            asm volatile("" : "+v"(x));  // a select chain, not a table in scratch memory
        }
        dst[lane] = x;
    }
}

template <typename T>
__device__ __forceinline__ global<T>* elem(global<T>* base, uint32_t i)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<global<T>*>(reinterpret_cast<global<B>*>(base) + (uint64_t)(i * (uint32_t)sizeof(T)));
}

// Read-only data of the launch through the constant address space: a
// wave-uniform address turns into scalar loads, and the values feed the
// vector ALU as scalar-register operands.
template <typename T> using cptr = const __attribute__((address_space(4))) T*;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Run of workgroup blockIdx.x in launch set ls (binary search over the
// cumulative offsets; wave-uniform) and the workgroup's index within the run.
__device__ __forceinline__ int run_of_block(const LaunchSet& ls, int& blk)
{
    const int b = blockIdx.x;
    int lo = 0, hi = ls.count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ls.first[mid] <= b) lo = mid;
        else hi = mid;
    }
    blk = b - ls.first[lo];
    return ls.slot[lo];
}

template <typename T> __device__ __forceinline__ const T* uinv_table(const RunConst& rc);
template <> __device__ __forceinline__ const float* uinv_table<float>(const RunConst& rc) { return rc.uinv32; }
template <> __device__ __forceinline__ const double* uinv_table<double>(const RunConst& rc) { return rc.uinv64; }

// Index pair (a, b), a < b, of upper entry q.
template <int N>
__host__ __device__ constexpr void pair_of(int q, int& a, int& b)
{
    a = 0;
    b = 1;
    for (int aa = 0; aa < N; ++aa)
        for (int bb = aa + 1; bb < N; ++bb)
            if (Shape<N>::up(aa, bb) == q) { a = aa; b = bb; }
}

// ------------------------------------------------------------------ physics
// Stage radius l of the attempt described by C (l < S).
template <typename TAB>
__device__ __forceinline__ double stage_radius(const Control& C, int l)
{
    return fma(TAB::C[l], C.h, C.r);
}

// Geometry of trajectory j at radius r (eq 3.14-3.15, with 1 - (R/r)^2 formed
// as (r - R)(r + R) / r^2; single angle: c = 1, w = D(r/R) of eq 3.17), and
// 1 / c.  The per-trajectory constants (u^2, 1 - u^2, u du / np) come from a
// table, so a reciprocal of r and a reciprocal square root (c = c^2 / c) are
// all the divisions.
__device__ __forceinline__ void traj_geometry(const RunConst& rc, int j, double r, double& c, double& w, double& ic)
{
    const double ir = 1.0 / r;
    const double xr = rc.r_nu * ir;
    const double x = xr * xr;
    const double y = (r - rc.r_nu) * (r + rc.r_nu) * (ir * ir);
    if (rc.ma) {
        const global<const double>* g = gview(rc.geo) + 4 * (size_t)j;
        const double q = fma(g[1], y, g[0]);
        ic = rsqrt(q);
        c = q * ic;
        w = x * g[2] * ic;
    } else {
        c = 1.0;
        ic = 1.0;
        const double s = 1.0 - sqrt(y);
        w = 0.5 * s * s;
    }
}

__device__ __forceinline__ double matter(const RunConst& rc, double r)
{
    const double x = rc.lambda_rref / r, p = rc.lambda_power;
    if (p == 3.0) return rc.lambda0 * (x * x * x);  // the bulb profile, without pow
    return rc.lambda0 * pow(x, p);
}

// Co-rotating phase of stage l: Phi_n + h sum_{m<l} a_lm G_m (explicit fma
// chain, so every launch that forms it gets the same bits).
template <typename TAB, int N>
__device__ __forceinline__ void stage_phase(int l, double h, const double* phn, const double (*G)[N], double* ph)
{
#pragma unroll
    for (int a = 0; a < N; ++a) {
        double acc = 0.0;
        for (int m = 0; m < l; ++m) acc = fma(l < TAB::S ? TAB::A[l][m] : TAB::B[m], G[m][a], acc);
        ph[a] = fma(h, acc, phn[a]);
    }
}

// e^{i(Phi_a - Phi_b)} of the upper pairs, computed by a group of lanes that
// share one trajectory (first lane `base`, lane li within the group): lane q <
// NU of the group evaluates pair q and every lane of the group receives all NU
// factors.
template <int N>
__device__ __forceinline__ void rotation(const double* ph, double (*z)[2], int li, int base)
{
    constexpr int NU = Shape<N>::NU;
    double d = ph[0] - ph[1];
#pragma unroll
    for (int q = 1; q < NU; ++q) {
        int a = 0, b = 1;
        pair_of<N>(q, a, b);
        d = (li == q) ? ph[a] - ph[b] : d;
    }
    double sn, cs;
    fast_sincos(d, sn, cs);
#pragma unroll
    for (int q = 0; q < NU; ++q) {
        z[q][0] = __shfl(cs, base + q, 64);
        z[q][1] = __shfl(sn, base + q, 64);
    }
}

// Angle weights of one trajectory for the NJ moments at a stage radius:
// w, w c (0 single angle) and, for the extended model (eq 3.18), w s cos(phi),
// w s sin(phi) with s = sin(theta).
template <int NJ>
__device__ __forceinline__ void angle_weights(const RunConst& rc, double c, double w, double cph, double sph,
                                              double* f)
{
    f[0] = w;
    f[1] = rc.ma ? w * c : 0.0;
    if constexpr (NJ == 4) {
        const double s = sqrt((1.0 - c) * (1.0 + c));
        f[2] = (w * s) * cph;
        f[3] = (w * s) * sph;
    }
}

// Step controller (readings J, K of the oracle's header; fixed-step RK4 always
// accepts a finite step).  Returns whether the attempt is accepted.
template <typename TAB>
__device__ bool control_step(const RunConst& rc, Control& C, double m)
{
    C.attempts += 1;
    bool accepted = false;
    const double h = C.h;
    if constexpr (!TAB::embedded) {
        if (!(m <= 1.0e300)) {
            C.status = -4;
        } else {
            accepted = true;
            C.istep += 1;
            C.nacc += 1;
            C.cur ^= 1;
            C.r = rc.r_start + (double)C.istep * rc.h_fixed;
            C.h = rc.h_fixed;
            if (C.istep >= rc.n_fixed || C.r >= C.r_end) C.status = 1;
        }
    } else {
        const double err = m / rc.rtol;
        C.err = err;
        if (!(err <= 1.0e300)) {
            C.status = -4;
        } else {
            const double f_lo = 0.2, f_hi = 5.0;
            double fac, rn = C.r;
            if (err <= 1.0) {
                accepted = true;
                rn = C.r + h;
                C.r = rn;
                C.nacc += 1;
                C.cur ^= 1;
                fac = (err == 0.0) ? f_hi : rc.safety * pow(err, -0.2);
                fac = fmin(fmax(fac, f_lo), f_hi);
                if (C.last_rejected && fac > 1.0) fac = 1.0;
                C.last_rejected = 0;
            } else {
                C.nrej += 1;
                fac = fmax(rc.safety * pow(err, -0.2), f_lo);
                C.last_rejected = 1;
            }
            double hn = fmin(h * fac, rc.dr_max);
            C.h_prop = hn;
            if (rn >= C.r_end) {
                C.status = 1;
            } else if (hn < 1e-14 * rn) {
                C.status = -5;
            } else {
                if (rn + hn > C.r_end) hn = C.r_end - rn;
            }
            C.h = hn;
        }
    }
    if (C.status == 0 && rc.max_steps > 0 && C.attempts >= rc.max_steps) C.status = -6;
    return accepted;
}

// ------------------------------------------------------------------ partial sums
// Sum of the value-major partials of buffer `par` (nblk workgroups) by the NW
// wavefronts of a workgroup: value v by wavefront v mod NW, lane l adding
// partials l, l + 64, ... in order, then the row sums (DPP) and the four rows
// added in one fixed order.  Every workgroup running this gets the same bits.
// Split in two so that the loads of the first 256 partials are in flight while
// independent work runs.
template <int NV, int NW>
struct PartialRegs {
    static constexpr int VPW = (NV + NW - 1) / NW;  // values per wavefront
    double x[VPW][4];
};

template <int NV, int NW>
__device__ __forceinline__ void load_partials(const RunConst& rc, int par, int nblk, PartialRegs<NV, NW>& r)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ps = rc.pstride;
    const global<const double>* src = gview<const double>(rc.partial) + (size_t)(par & 1) * NV * ps;
#pragma unroll
    for (int i = 0; i < PartialRegs<NV, NW>::VPW; ++i) {
        const int v = wave + i * NW;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int p = lane + 64 * k;
            r.x[i][k] = (v < NV && p < nblk) ? src[(size_t)v * ps + p] : 0.0;
        }
    }
}

template <int NV, int NW>
__device__ void finish_partials(const RunConst& rc, int par, int nblk, const PartialRegs<NV, NW>& r, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ps = rc.pstride;
    const global<const double>* src = gview<const double>(rc.partial) + (size_t)(par & 1) * NV * ps;
#pragma unroll
    for (int i = 0; i < PartialRegs<NV, NW>::VPW; ++i) {
        const int v = wave + i * NW;
        if (v >= NV) continue;
        double acc = r.x[i][0];
        acc += r.x[i][1];
        acc += r.x[i][2];
        acc += r.x[i][3];
        for (int p = lane + 256; p < nblk; p += 64) acc += src[(size_t)v * ps + p];
        acc = wave_sum_rows(acc);
        if (lane == 0) out[v] = acc;
    }
    __syncthreads();
}

// A beam-pass read of the state.  FP64 states are read non-temporally: each
// value is used once per launch, and keeping it out of the caches leaves them
// to the tables (measured: the FP64 state update and power moments 6% and 20%
// faster; the FP32 state, half the size, gains nothing).
template <typename TS>
__device__ __forceinline__ TS load_state(global<const TS>* p)
{
    if constexpr (std::is_same<TS, double>::value) return __builtin_nontemporal_load(p);
    else return *p;
}

// ------------------------------------------------------------------ power moments
// Launch S + 2 of an attempt (TAIL) and the moment launch after a new state or
// radius (FORCE).  TAIL first takes the global maximum of the state-update
// launch's error maxima and runs the controller in every workgroup (the same
// result everywhere; workgroup 0 stores the control block); a rejected attempt
// ends here.  Then, for the current state y (the accepted new state):
//   Q_p[j] = sum_k w_k u_k^p y y^+,  p = 0 .. NQ-1  (FP64, stored as full
//   complex matrices).
// The neutrino and the antineutrino beam of one energy bin have u = 1/E and
// u = -1/E, so the antineutrino's u^p is (-1)^p u^p and one energy bin adds
//   u^p (w y y^+ + (-1)^p wbar ybar ybar^+)
// to Q_p: the even powers take one combination of the two densities and the
// odd powers the other, half the multiply-adds of one sum per beam.  Two
// trajectories per wavefront (32 lanes each), two lanes per energy bin (the
// first adds the even powers 2k, the second the odd powers 2k + 1, k < H),
// 16 energy bins of a trajectory per wavefront iteration: each row of 16 lanes
// holds one trajectory and one parity of the powers, so that the lanes' sums
// are row sums (cross-lane moves of the vector ALU).  FP64 amplitudes: the
// even row loads the neutrino beams, the odd row the antineutrino beams (each
// amplitude loaded once), each row forms its own beam's weighted density and
// a row swap gives every lane both densities; FP32 amplitudes: both rows load
// both beams and form both densities (measured faster for them: half the
// bytes, and no swaps in the lanes' instruction stream).  The first bins are
// requested before the step controller has decided, from the buffer an
// accepted step makes current (a rejected attempt drops them).  Q_0 is the
// density sum of the state itself: rotated to the lab frame and weighted at
// the state's radius, it gives the workgroup's partial of J_0 (buffer 0).
constexpr int kPowerWaves = kTrajPerBlock / 2;
static_assert(kPowerTrajPerBlock == kTrajPerBlock, "the power-moment launch covers kTrajPerBlock trajectories per workgroup");

template <typename TS, int N, typename TAB, int NJ, bool FORCE>
__device__ __forceinline__ void power_body(const RunConst& rc, const int blk)
{
    constexpr int NM = Shape<N>::NM, NU = Shape<N>::NU, NV = NJ * NM;
    constexpr int NQ = Poly<TAB>::NQ;
    constexpr int H = (NQ + 1) / 2;  // powers per lane (p = 2k + parity)
    constexpr int NSLOT = 2;         // energy bins of a lane in flight
    constexpr uint32_t STRIDE = 16;  // energy-bin stride of a lane
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    __shared__ double swave[kTrajPerBlock][NV];
    __shared__ double serr[kPowerWaves];
    __shared__ double sq[kTrajPerBlock][NQ * NM];
    __shared__ double sjz[kTrajPerBlock][2 * (NU > 0 ? NU : 1)];  // J_0 partial: rotation factors
    __shared__ double sjf[kTrajPerBlock][4];                      // and angle weights

    Control C;
    double m = 0.0;
    if constexpr (FORCE) {
        C = gload(rc.ctrl + 1);
    } else {
        // the control block and the error maxima requested together
        C = gload(rc.ctrl);
        for (int p = tid; p < rc.nblkf; p += 64 * kPowerWaves) m = fmax(m, gview(rc.errpart)[p]);
        if (C.status != 0) return;  // the attempt did not run
    }
    // an accepted attempt makes the other buffer current
    const int cur = FORCE ? C.cur : (C.cur ^ 1);
    const int g = lane >> 5, hb = (lane >> 4) & 1, q = lane & 15;
    const int jt = 2 * wave + g;
    const int j = blk * kTrajPerBlock + jt;
    const bool active = j < rc.na;
    const uint32_t ne = (uint32_t)rc.ne;
    // bins of the wavefront's loop (both trajectories of a wavefront are idle together)
    const uint32_t nel = (blk * kTrajPerBlock + 2 * wave < rc.na) ? ne : 0u;
    // neutrino and antineutrino beams of trajectory j (of trajectory 0 for an
    // idle lane group, whose loads are never used)
    const uint32_t base0 = active ? (uint32_t)j * ne : 0u;
    const uint32_t base1 = active ? (uint32_t)(j + rc.na) * ne : (uint32_t)rc.na * ne;
    const size_t ld = (size_t)rc.nb_pad;
    const TS* src = reinterpret_cast<const TS*>(rc.psi[cur]);
    global<const TS>* __restrict__ srcq[2 * N];
#pragma unroll
    for (int x = 0; x < 2 * N; ++x) srcq[x] = uniform_global(src + x * ld);
    global<const double>* __restrict__ uinv = uniform_global(rc.uinv64);
    global<const double>* __restrict__ wgtp = uniform_global(rc.wgt);

    // energy bin e: u = 1/E, and the lane's own beam (the row's species) or
    // both beams, with their weights.  Unconditional (a bin past the end reads
    // bin 0 and adds with weight 0), so that the loop is straight-line code in
    // which each load refills the registers of its slot: no copies, and no
    // wait for loads still in flight.
    constexpr bool SWAP = sizeof(TS) == 8;
    constexpr int NB = SWAP ? 1 : 2;  // beams a lane loads per bin
    const uint32_t bown = hb ? base1 : base0, wown = hb ? ne : 0u;
    auto fetch = [&](uint32_t e, TS* vv, double& uv, double* wv) __attribute__((always_inline)) {
        const uint32_t ec = e < ne ? e : 0u;
        if constexpr (SWAP) {
#pragma unroll
            for (int x = 0; x < 2 * N; ++x) vv[x] = load_state(elem(srcq[x], bown + ec));
            wv[0] = *elem(wgtp, wown + ec);
        } else {
#pragma unroll
            for (int x = 0; x < 2 * N; ++x) vv[x] = load_state(elem(srcq[x], base0 + ec));
#pragma unroll
            for (int x = 0; x < 2 * N; ++x) vv[2 * N + x] = load_state(elem(srcq[x], base1 + ec));
            wv[0] = *elem(wgtp, ec);
            wv[1] = *elem(wgtp, ne + ec);
        }
        uv = *elem(uinv, ec);
    };
    TS vs[NSLOT][NB * 2 * N];
    double us[NSLOT], ws[NSLOT][NB];
    const uint32_t e0 = (uint32_t)q;
    static_for<0, NSLOT>([&](auto Sc) {
        constexpr int sl = decltype(Sc)::value;
        fetch(e0 + sl * STRIDE, vs[sl], us[sl], ws[sl]);
    });

    if constexpr (!FORCE) {
        m = wave_max_rows(m);
        if (lane == 0) serr[wave] = m;
        __syncthreads();
        m = serr[0];
        for (int w = 1; w < kPowerWaves; ++w) m = fmax(m, serr[w]);
        const bool accepted = control_step<TAB>(rc, C, m);
        C.fresh = accepted ? 1 : 0;
        if (blk == 0 && tid == 0) gstore(rc.ctrl + 1, C);
        if (!accepted) return;
    }

    // for the J_0 partial of the new state, before the beam loop (kept in LDS,
    // not in registers): the rotation factors of both trajectories of the
    // wavefront and the angle weights at the state's radius
    {
        double ph[N], zz[2][NU > 0 ? NU : 1][2];
        for (int gg = 0; gg < 2; ++gg) {
            const int jj = blk * kTrajPerBlock + 2 * wave + gg;
            for (int a = 0; a < N; ++a) ph[a] = jj < rc.na ? gview(rc.phase[cur])[(size_t)jj * N + a] : 0.0;
            rotation<N>(ph, zz[gg], lane, 0);
        }
        if ((lane & 31) == 0) {
            for (int u = 0; u < NU; ++u) {
                sjz[jt][2 * u] = g ? zz[1][u][0] : zz[0][u][0];
                sjz[jt][2 * u + 1] = g ? zz[1][u][1] : zz[0][u][1];
            }
            double f[4] = {0.0, 0.0, 0.0, 0.0};
            if (active) {
                double c, w, ic;
                traj_geometry(rc, j, C.r, c, w, ic);
                double cph = 1.0, sph = 0.0;
                if constexpr (NJ == 4) {
                    cph = gview(rc.azi)[2 * (size_t)j];
                    sph = gview(rc.azi)[2 * (size_t)j + 1];
                }
                angle_weights<NJ>(rc, c, w, cph, sph, f);
            }
            for (int m2 = 0; m2 < NJ; ++m2) sjf[jt][m2] = f[m2];
        }
    }

    double acc[H][NM];
#pragma unroll
    for (int k = 0; k < H; ++k)
#pragma unroll
        for (int x = 0; x < NM; ++x) acc[k][x] = 0.0;

    auto process = [&](uint32_t e, const TS* vv, double u, const double* wv) __attribute__((always_inline)) {
        // u^(2k + parity): the odd lanes start at u
        const double u2 = u * u;
        double pw[H];
        pw[0] = hb ? u : 1.0;
#pragma unroll
        for (int k = 1; k < H; ++k) pw[k] = pw[k - 1] * u2;
        auto add = [&](int x, double v) __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < H; ++k) acc[k][x] = fma(v, pw[k], acc[k][x]);
        };
        // Re and Im of v_a conj(t_b)
        auto re = [&](const double* v, const double* t, int a, int b) __attribute__((always_inline)) {
            return fma(v[2 * a], t[2 * b], v[2 * a + 1] * t[2 * b + 1]);
        };
        auto im = [&](const double* v, const double* t, int a, int b) __attribute__((always_inline)) {
            return fma(v[2 * a + 1], t[2 * b], -(v[2 * a] * t[2 * b + 1]));
        };
        if constexpr (SWAP) {
            // each row forms its own beam's weighted density (w y y^+ in the
            // even row, wbar z z^+ in the odd one); a row swap gives both in
            // every lane, combined with the sign (-1)^parity
            double ww = wv[0];
            if (!(active && e < ne)) ww = 0.0;
            double y[2 * N], yw[2 * N];
#pragma unroll
            for (int x = 0; x < 2 * N; ++x) {
                y[x] = (double)vv[x];
                yw[x] = ww * y[x];
            }
            const double sg = hb ? -1.0 : 1.0;
            auto put = [&](int x, double own) __attribute__((always_inline)) {
                double ev, od;
                row_pair(own, ev, od);
                add(x, fma(sg, od, ev));
            };
#pragma unroll
            for (int a = 0; a < N; ++a) put(a, re(yw, y, a, a));
#pragma unroll
            for (int a = 0; a < N; ++a)
#pragma unroll
                for (int b = a + 1; b < N; ++b) {
                    const int x = N + 2 * Shape<N>::up(a, b);
                    put(x, re(yw, y, a, b));
                    put(x + 1, im(yw, y, a, b));
                }
        } else {
            // both beams in every lane: X = w y y^+ + s z z^+ with
            // s = (-1)^parity wbar, entry by entry
            double w = wv[0], wb = wv[1];
            if (!(active && e < ne)) w = wb = 0.0;
            const double s = hb ? -wb : wb;
            double y[2 * N], z[2 * N];
#pragma unroll
            for (int x = 0; x < 2 * N; ++x) {
                y[x] = (double)vv[x];
                z[x] = (double)vv[2 * N + x];
            }
#pragma unroll
            for (int a = 0; a < N; ++a) add(a, fma(w, re(y, y, a, a), s * re(z, z, a, a)));
#pragma unroll
            for (int a = 0; a < N; ++a)
#pragma unroll
                for (int b = a + 1; b < N; ++b) {
                    const int x = N + 2 * Shape<N>::up(a, b);
                    add(x, fma(w, re(y, y, a, b), s * re(z, z, a, b)));
                    add(x + 1, fma(w, im(y, y, a, b), s * im(z, z, a, b)));
                }
        }
    };

#pragma unroll 1
    for (uint32_t e = 0; e < nel; e += NSLOT * STRIDE) {
        static_for<0, NSLOT>([&](auto Sc) {
            constexpr int sl = decltype(Sc)::value;
            const uint32_t es = e + e0 + sl * STRIDE;
            process(es, vs[sl], us[sl], ws[sl]);
            fetch(es + NSLOT * STRIDE, vs[sl], us[sl], ws[sl]);
            // keep the refill of this slot ahead of the next slot's work
            __builtin_amdgcn_sched_barrier(0);
        });
    }

    // sums over the 16 lanes of a row (one trajectory, one parity of the powers)
#pragma unroll
    for (int k = 0; k < H; ++k)
#pragma unroll
        for (int x = 0; x < NM; ++x) acc[k][x] = row_sum16(acc[k][x]);

    // the workgroup's Q (packed) to LDS; stored as full matrices below
    if (q == 0) {
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int p = 2 * k + hb;
            if (p < NQ)
#pragma unroll
                for (int x = 0; x < NM; ++x) sq[jt][p * NM + x] = acc[k][x];
        }
    }

    // the J_0 partial: Q_0 (lane 32 g) rotated to the lab frame and weighted
    if ((lane & 31) == 0) {
        double sl[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) sl[v] = 0.0;
        if (active) {
            double f[4];
            for (int m2 = 0; m2 < NJ; ++m2) f[m2] = sjf[jt][m2];
            double Sv[NM];
            for (int a = 0; a < N; ++a) Sv[a] = 2.0 * acc[0][a];
            for (int u = 0; u < NU; ++u) {
                const double cs = sjz[jt][2 * u], sn = sjz[jt][2 * u + 1];
                const double xr = acc[0][N + 2 * u], xi = acc[0][N + 2 * u + 1];
                Sv[N + 2 * u] = 2.0 * (cs * xr + sn * xi);
                Sv[N + 2 * u + 1] = 2.0 * (cs * xi - sn * xr);
            }
            for (int m = 0; m < NJ; ++m)
                for (int v = 0; v < NM; ++v) sl[m * NM + v] = f[m] * Sv[v];
        }
        for (int v = 0; v < NV; ++v) swave[jt][v] = sl[v];
    }
    __syncthreads();
    if (tid < NV) {
        double s = swave[0][tid];
        for (int w = 1; w < kTrajPerBlock; ++w) s += swave[w][tid];
        gview(rc.partial)[(size_t)tid * rc.pstride + blk] = s;  // buffer 0
    }
    // Q_p as full complex matrices (row-major, re/im adjacent: the layout the
    // stage launches compute with), one 16-byte entry per thread and pass,
    // consecutive threads on consecutive entries
    {
        constexpr int NN = N * N, NC = Shape<N>::NC;
        constexpr int UNITS = kTrajPerBlock * NQ * NN;
        for (int u = tid; u < UNITS; u += 64 * kPowerWaves) {
            const int t = u / (NQ * NN), r = u - t * (NQ * NN);
            const int p = r / NN, e = r - p * NN;
            const int a = e / N, b = e - a * N;
            const double* P = &sq[t][p * NM];
            double re, im = 0.0;
            if (a == b) {
                re = P[a];
            } else {
                const int lo = a < b ? a : b, hi = a < b ? b : a;
                const int x = N + 2 * Shape<N>::up(lo, hi);
                re = P[x];
                im = a < b ? P[x + 1] : -P[x + 1];
            }
            const int jj = blk * kTrajPerBlock + t;
            if (jj < rc.na)
                *reinterpret_cast<global<d2>*>(gview(rc.qbuf) + (size_t)jj * rc.qstride + p * NC + 2 * e) = d2{re, im};
        }
    }
}

// ------------------------------------------------------------------ per-trajectory stages
// Launch L of an attempt.  A group of kTrajLanes lanes works on one trajectory
// (two per wavefront, kTrajPerBlock per workgroup), its lanes on items (d, e):
// coefficient degree d and matrix entry e = (a, b) of a full complex n x n
// matrix.
//   1. J_{L-1}: the fixed-order sum of the previous launch's partials (L = 1:
//      the power-moment launch's, or J_0 kept from a rejected attempt).  While
//      it is in flight: geometry and frame of stage L-1, the stored coefficient
//      matrices summed into C_{L-1} = 1 + sum_{m<L-1} a_{L-1,m} D_m and into
//      the part of C_L (or of the update and error tables) without D_{L-1}.
//   2. Completion of stage L-1 at its radius: collective term
//      C = mu0 traceless(J0 - c J1 [- s cos(phi) J2 - s sin(phi) J3]), frame
//      rate G = diag(H_m + C) / c (co-rotating frame, 0 in the lab frame),
//      A = e^{i(Phi_a - Phi_b)} C_ab / c off the diagonal (diagonal 0, lab
//      frame (H_m + C)_aa / c), B = e^{i(Phi_a - Phi_b)} V_ab / c with
//      H_vac = V / E; N0 = -i h A, N1 = -i h B.
//   3. D_{L-1,d} = N0 C_{L-1,d} + N1 C_{L-1,d-1} (stored for later launches).
//   L < S:
//   4. C_L = 1 + sum_{m<L} a_Lm D_m; T_d = sum_{d'} Q_{d+d'} C_{L,d'}^+;
//      X_d = C_{L,d} T_d; the stage-L density sum sum_d X_d (co-rotating).
//   5. Rotation to the lab frame with the stage-L phase, angle weights of
//      stage L, one partial per workgroup (buffer L & 1).  Dormand-Prince:
//      stage S-1 is the new state, whose phase is stored.
//   L = S:
//   4. Tables of the update 1 + sum_m b_m D_m (type TF) and of the error
//      sum_m e_m D_m (FP64) for k_final, row by row (row a: degree 0, 1, ...
//      of its 2n reals); RK4: the new state's phase.
// Entry k (re, im) of a full complex matrix in LDS, row-major with re and im
// adjacent: one 16-byte read (the matrices are 16-byte aligned).
__device__ __forceinline__ double2 ldsc(const double* m, int k)
{
    return *reinterpret_cast<const double2*>(m + 2 * k);
}

constexpr int kTrajLanes = 32;
constexpr int kTrajWaves = kTrajPerBlock * kTrajLanes / 64;

template <int N, typename TAB, int NJ, int L, typename TF>
__device__ __forceinline__ void traj_body(const RunConst& rc, const int blk)
{
    using PY = Poly<TAB>;
    constexpr int S = TAB::S, NM = Shape<N>::NM, NU = Shape<N>::NU, NC = Shape<N>::NC, NN = N * N;
    constexpr int NV = NJ * NM;
    constexpr bool TABLES = (L == S);
    constexpr int LT = kTrajLanes;
    constexpr int DMAX = TABLES ? S : L;                 // largest degree an item handles
    constexpr int ITEMS = (DMAX + 1) * NN;
    constexpr int NIT = (ITEMS + LT - 1) / LT;
    constexpr int NH = L - 1;                            // stored matrices D_0 .. D_{L-2}
    constexpr int NQL = TABLES ? 1 : 2 * L + 1;          // power moments stage L needs
    constexpr int QU = NQL * NC / 2;                     // their 16-byte (re, im) entries
    constexpr int QV = (QU + LT - 1) / LT;               // of them per lane
    constexpr int TPB = kTrajPerBlock;
    constexpr int NW = kTrajWaves;
    constexpr int NUA = NU > 0 ? NU : 1;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & (LT - 1);                      // lane within the trajectory's group
    const int gbase = lane & ~(LT - 1);                  // first lane of the group
    const int jt = wave * (64 / LT) + lane / LT;         // trajectory within the workgroup
    const int j = blk * TPB + jt;
    const bool active = j < rc.na;

    // Q_p as full complex matrices (row-major, re/im adjacent, so that an
    // entry is one 16-byte LDS read); later the X_d (packed)
    __shared__ __align__(16) double sQ[TPB][NQL * NC];
    __shared__ __align__(16) double sC[TPB][S * NC];                   // C_{L-1}, then C_L
    __shared__ __align__(16) double sT[TPB][TABLES ? 2 : S * NC];      // T_d
    __shared__ __align__(16) double sN[TPB][2 * NC];                   // N0, N1
    __shared__ double swave[TPB][NV];
    __shared__ double sJ[NV];

    // ---- everything that does not depend on J_{L-1} is requested at entry:
    //      control block (ctrl[1] between attempts, ctrl[0] during one), the
    //      previous launch's partials, both phase buffers, the frame rates of
    //      the earlier stages, the power moments
    Control C{};
    {
        global<Control>* vc = gview(rc.ctrl) + (L == 1 ? 1 : 0);
        C.r = __hip_atomic_load(&vc->r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        C.h = __hip_atomic_load(&vc->h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        C.cur = __hip_atomic_load(&vc->cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        C.status = __hip_atomic_load(&vc->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        C.fresh = __hip_atomic_load(&vc->fresh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    PartialRegs<NV, NW> xp;
    // L = 1: the power-moment launch's (used if fresh)
    const int npart = L == 1 ? rc.nblkp : rc.nblk;
    load_partials<NV, NW>(rc, L - 1, npart, xp);
    const int jl = active ? j : 0;
    double ph01[2][N], G[L][N];
    for (int a = 0; a < N; ++a) {
        ph01[0][a] = gview(rc.phase[0])[(size_t)jl * N + a];
        ph01[1][a] = gview(rc.phase[1])[(size_t)jl * N + a];
    }
    for (int m = 0; m < NH; ++m)
        for (int a = 0; a < N; ++a) G[m][a] = gview(rc.gbuf)[((size_t)jl * kMaxStages + m) * N + a];
    d2 qv[QV];
    {
        const global<d2>* qs = reinterpret_cast<const global<d2>*>(gview(rc.qbuf) + (size_t)jl * rc.qstride);
#pragma unroll
        for (int i = 0; i < QV; ++i) qv[i] = (!TABLES && li + LT * i < QU) ? qs[li + LT * i] : d2{0.0, 0.0};
    }
    // the rotation factors of stage L-1, stored by the previous launch
    double zl[2 * NUA];
    if constexpr (L > 1) {
#pragma unroll
        for (int i = 0; i < 2 * NU; ++i) zl[i] = gview(rc.zbuf)[(size_t)jl * 8 + i];
    }
    // the stored coefficient matrices each item needs (in range for every lane)
    double Dh[NIT][NH > 0 ? NH : 1][2];
    {
        const global<double>* dsrc = gview(rc.dbuf) + (size_t)jl * rc.dstride;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = li + LT * it, d = idx / NN, e = idx - d * NN;
#pragma unroll
            for (int m = 0; m < NH; ++m) {
                const bool have = idx < ITEMS && d <= m + 1;
                // one 16-byte (re, im) read (dbuf rows and entries are 16-byte aligned)
                const d2 v = *reinterpret_cast<const global<d2>*>(dsrc + (have ? (size_t)(PY::doff(m) + d) * NC + 2 * e : 0));
                Dh[it][m][0] = have ? v.x : 0.0;
                Dh[it][m][1] = have ? v.y : 0.0;
            }
        }
    }
    double cph = 1.0, sph = 0.0;
    if constexpr (NJ == 4) {
        cph = gview(rc.azi)[2 * (size_t)jl];
        sph = gview(rc.azi)[2 * (size_t)jl + 1];
    }
    if (L == 1 && blk == 0 && tid == 0) gstore(rc.ctrl, gload(rc.ctrl + 1));
    if (C.status != 0) return;  // run finished: attempts are no-ops
    const int cur = C.cur;
    const double h = C.h;
    double phn[N];
    for (int a = 0; a < N; ++a) phn[a] = cur ? ph01[1][a] : ph01[0][a];

    // ---- while J_{L-1} is summed: geometry and frame of stage L-1 (and the
    //      geometry of stage L), the stored coefficient matrices summed into
    //      C_{L-1} (to LDS) and into the parts of C_L or of the tables
    //      without D_{L-1} (registers), Q to LDS
    const double rP = stage_radius<TAB>(C, L - 1);
    double cP, wP;
    double icP;
    traj_geometry(rc, jl, rP, cP, wP, icP);
    double sc = 0.0, ss = 0.0;
    if constexpr (NJ == 4) {
        const double s0 = sqrt((1.0 - cP) * (1.0 + cP));
        sc = s0 * cph;
        ss = s0 * sph;
    }
    double zP[NUA][2];
    if constexpr (L == 1) {
        double ph[N];
        stage_phase<TAB, N>(L - 1, h, phn, G, ph);
        rotation<N>(ph, zP, li, gbase);
    } else {
#pragma unroll
        for (int q = 0; q < NU; ++q) {
            zP[q][0] = zl[2 * q];
            zP[q][1] = zl[2 * q + 1];
        }
    }
    double cL = 1.0, wL = 0.0;
    if constexpr (!TABLES) {
        double icL;
        traj_geometry(rc, jl, stage_radius<TAB>(C, L), cL, wL, icL);
    }
    // per item: next = C_L without its D_{L-1} term (L < S), or the update
    // (next) and error (nerr) tables without it (L = S), each summed from the
    // identity in ascending m as C_{L-1} is
    double next[NIT][2], nerr[NIT][2];
    if (active) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = li + LT * it, d = idx / NN, e = idx - d * NN;
            const int a = e / N, b = e - (e / N) * N;
            const double id = (d == 0 && a == b) ? 1.0 : 0.0;
            double cr = id, ci = 0.0, xr = id, xi = 0.0, er = 0.0, ei = 0.0;
            if (idx < ITEMS) {
                static_for<0, NH>([&](auto Mc) {
                    constexpr int m = decltype(Mc)::value;
                    {
                        const double dr = Dh[it][m][0], di = Dh[it][m][1];
                        constexpr double ca = TAB::A[L - 1][m];
                        if constexpr (ca != 0.0) {
                            cr = fma(ca, dr, cr);
                            ci = fma(ca, di, ci);
                        }
                        constexpr double cn = TABLES ? TAB::B[m] : TAB::A[L][m];
                        if constexpr (cn != 0.0) {
                            xr = fma(cn, dr, xr);
                            xi = fma(cn, di, xi);
                        }
                        if constexpr (TABLES && TAB::E[m] != 0.0) {
                            er = fma(TAB::E[m], dr, er);
                            ei = fma(TAB::E[m], di, ei);
                        }
                    }
                });
                if (d <= L - 1) {
                    sC[jt][d * NC + 2 * e] = cr;
                    sC[jt][d * NC + 2 * e + 1] = ci;
                }
            }
            next[it][0] = xr;
            next[it][1] = xi;
            nerr[it][0] = er;
            nerr[it][1] = ei;
        }
        if constexpr (!TABLES) {
#pragma unroll
            for (int i = 0; i < QV; ++i) {
                const int v = li + LT * i;
                if (v < QU) *reinterpret_cast<d2*>(&sQ[jt][2 * v]) = qv[i];
            }
        }
    }

    // ---- J_{L-1}
    if (L > 1 || C.fresh) {
        finish_partials<NV, NW>(rc, L - 1, npart, xp, sJ);
        if (blk == 0 && tid < NV) gview(rc.jhist)[(size_t)(L - 1) * NV + tid] = sJ[tid];
    } else {
        if (tid < NV) sJ[tid] = gview(rc.jhist)[tid];
        __syncthreads();
    }

    if (li == 0 && !TABLES)
        for (int v = 0; v < NV; ++v) swave[jt][v] = 0.0;
    if (active) {
        // ---- completion of stage L-1: the diagonal in every lane of the group
        //      (the frame rate G_{L-1} enters the phase of stage L), then lane
        //      li < 2 n^2 forms entry li of N0 = -i h A (li < n^2) or of
        //      N1 = -i h B (row-major) as one (re, im) pair
        const double lam = matter(rc, rP);
        auto kern = [&](int x) __attribute__((always_inline)) {
            double v = sJ[x] - cP * sJ[NM + x];
            if constexpr (NJ == 4) v = (v - sc * sJ[2 * NM + x]) - ss * sJ[3 * NM + x];
            return v;
        };
        double Cd[N], tr = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            Cd[a] = kern(a);
            tr += Cd[a];
        }
        double hd[N];
#pragma unroll
        for (int a = 0; a < N; ++a) {
            hd[a] = lam * ((a == 0 ? 1.0 : 0.0) - 1.0 / N) + rc.mu0 * (Cd[a] - tr / N);
            G[L - 1][a] = (rc.frame == 0) ? hd[a] * icP : 0.0;
        }
        if (li < 2 * NN) {
            const int mtx = li >= NN ? 1 : 0, e = li - mtx * NN;
            const int a = e / N, b = e - (e / N) * N;
            const int lo = a < b ? a : b, hi = a < b ? b : a;
            const int u = a == b ? 0 : Shape<N>::up(lo, hi);
            // the values of pair u and of diagonal entry a, picked from
            // registers (wave-uniform tables, lane-dependent index)
            double cs = zP[0][0], sn = zP[0][1], vr = rc.vac[0][1][0], vi = rc.vac[0][1][1];
#pragma unroll
            for (int q = 1; q < NU; ++q) {
                int qa = 0, qb = 1;
                pair_of<N>(q, qa, qb);
                if (u == q) {
                    cs = zP[q][0];
                    sn = zP[q][1];
                    vr = rc.vac[qa][qb][0];
                    vi = rc.vac[qa][qb][1];
                }
            }
            double hda = hd[0], vda = rc.vac[0][0][0];
#pragma unroll
            for (int q = 1; q < N; ++q)
                if (a == q) {
                    hda = hd[q];
                    vda = rc.vac[q][q][0];
                }
            // off the diagonal: e^{i(Phi_lo - Phi_hi)} X_lo,hi / c, conjugated below
            const double kr = kern(N + 2 * u), ki = kern(N + 2 * u + 1);
            const double Xr = mtx == 0 ? rc.mu0 * kr : vr, Xi = mtx == 0 ? rc.mu0 * ki : vi;
            double xr = (cs * Xr - sn * Xi) * icP, xi = (cs * Xi + sn * Xr) * icP;
            if (a > b) xi = -xi;
            if (a == b) {
                xr = (mtx == 0 ? (rc.frame == 0 ? 0.0 : hda) : vda) * icP;
                xi = 0.0;
            }
            // -i h X: real part h Im X, imaginary part -h Re X
            *reinterpret_cast<d2*>(&sN[jt][mtx * NC + 2 * e]) = d2{h * xi, -h * xr};
        }
        if (li == 0)
            for (int a = 0; a < N; ++a) gview(rc.gbuf)[((size_t)j * kMaxStages + (L - 1)) * N + a] = G[L - 1][a];
        wave_sync();

        // ---- D_{L-1,d} = N0 C_{L-1,d} + N1 C_{L-1,d-1}
        double Dn[NIT][2];
        global<double>* ddst = gview(rc.dbuf) + (size_t)j * rc.dstride + (size_t)PY::doff(L - 1) * NC;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int idx = li + LT * it, d = idx / NN, e = idx - d * NN;
            Dn[it][0] = Dn[it][1] = 0.0;
            if (idx < ITEMS && d <= L) {
                const int a = e / N, b = e - (e / N) * N;
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    if (d <= L - 1) {
                        const double2 x = ldsc(&sN[jt][0], a * N + c), y = ldsc(&sC[jt][d * NC], c * N + b);
                        re = fma(x.x, y.x, fma(-x.y, y.y, re));
                        im = fma(x.x, y.y, fma(x.y, y.x, im));
                    }
                    if (d >= 1) {
                        const double2 x = ldsc(&sN[jt][NC], a * N + c), y = ldsc(&sC[jt][(d - 1) * NC], c * N + b);
                        re = fma(x.x, y.x, fma(-x.y, y.y, re));
                        im = fma(x.x, y.y, fma(x.y, y.x, im));
                    }
                }
                Dn[it][0] = re;
                Dn[it][1] = im;
                if constexpr (!TABLES) *reinterpret_cast<global<d2>*>(ddst + (size_t)d * NC + 2 * e) = d2{re, im};
            }
        }
        wave_sync();

        if constexpr (TABLES) {
            // ---- update and error tables for the state-update launch
            constexpr int DN = PY::DN, DE = PY::DE;
            global<char>* tb = gview(reinterpret_cast<char*>(rc.ftab)) + (size_t)j * rc.fstride;
            global<TF>* cn = reinterpret_cast<global<TF>*>(tb);
            global<double>* ce = reinterpret_cast<global<double>*>(tb + (((DN + 1) * NC * sizeof(TF) + 15) / 16) * 16);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int idx = li + LT * it, d = idx / NN, e = idx - d * NN;
                if (idx < ITEMS) {
                    const int a = e / N, b = e - (e / N) * N;
                    if (d <= DN) {
                        double re = next[it][0], im = next[it][1];
                        if constexpr (TAB::B[S - 1] != 0.0) {
                            re = fma(TAB::B[S - 1], Dn[it][0], re);
                            im = fma(TAB::B[S - 1], Dn[it][1], im);
                        }
                        cn[(a * (DN + 1) + d) * 2 * N + 2 * b] = (TF)re;
                        cn[(a * (DN + 1) + d) * 2 * N + 2 * b + 1] = (TF)im;
                    }
                    if constexpr (TAB::embedded) {
                        if (d <= DE) {
                            double re = nerr[it][0], im = nerr[it][1];
                            if constexpr (TAB::E[S - 1] != 0.0) {
                                re = fma(TAB::E[S - 1], Dn[it][0], re);
                                im = fma(TAB::E[S - 1], Dn[it][1], im);
                            }
                            *reinterpret_cast<global<d2>*>(ce + (a * (DE + 1) + d) * 2 * N + 2 * b) = d2{re, im};
                        }
                    }
                }
            }
            if constexpr (!TAB::fsal) {
                // the new state's phase Phi_n + h sum_m b_m G_m
                double ph[N];
                stage_phase<TAB, N>(S, h, phn, G, ph);
                lane_scatter(gview(rc.phase[cur ^ 1]) + (size_t)j * N, ph, li);
            }
        } else {
            // ---- C_L = (1 + sum_{m<L-1} a_Lm D_m) + a_{L,L-1} D_{L-1}
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int idx = li + LT * it, d = idx / NN, e = idx - d * NN;
                if (idx < ITEMS && d <= L) {
                    double re = next[it][0], im = next[it][1];
                    constexpr double cl = TAB::A[L][L - 1];
                    if constexpr (cl != 0.0) {
                        re = fma(cl, Dn[it][0], re);
                        im = fma(cl, Dn[it][1], im);
                    }
                    sC[jt][d * NC + 2 * e] = re;
                    sC[jt][d * NC + 2 * e + 1] = im;
                }
            }
            // frame of stage L (its phase needs G_{L-1}), while the LDS writes land
            double zL[NUA][2], ph[N];
            stage_phase<TAB, N>(L, h, phn, G, ph);
            if constexpr (TAB::fsal && L == S - 1) lane_scatter(gview(rc.phase[cur ^ 1]) + (size_t)j * N, ph, li);
            rotation<N>(ph, zL, li, gbase);
            {
                // for the next launch, whose stage L-1 this is
                double zf[2 * NUA];
#pragma unroll
                for (int q = 0; q < NU; ++q) {
                    zf[2 * q] = zL[q][0];
                    zf[2 * q + 1] = zL[q][1];
                }
                lane_scatter<2 * NU>(gview(rc.zbuf) + (size_t)j * 8, zf, li);
            }
            wave_sync();

            // ---- T_d = sum_{d'} Q_{d+d'} C_{L,d'}^+   (item (d, a, b))

#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int idx = li + LT * it, d = idx / NN, e = idx - d * NN;
                if (idx < ITEMS && d <= L) {
                    const int a = e / N, b = e - (e / N) * N;
                    // one accumulator pair per dd (independent chains), added in order
                    double rdd[L + 1], idd[L + 1];
#pragma unroll
                    for (int dd = 0; dd <= L; ++dd) {
                        double re = 0.0, im = 0.0;
#pragma unroll
                        for (int c = 0; c < N; ++c) {
                            const double2 q = ldsc(&sQ[jt][(d + dd) * NC], a * N + c);
                            const double2 cc = ldsc(&sC[jt][dd * NC], b * N + c);
                            // Q_{d+dd}[a][c] conj(C_dd[b][c])
                            re = fma(q.x, cc.x, fma(q.y, cc.y, re));
                            im = fma(q.y, cc.x, fma(-q.x, cc.y, im));
                        }
                        rdd[dd] = re;
                        idd[dd] = im;
                    }
                    double re = rdd[0], im = idd[0];
#pragma unroll
                    for (int dd = 1; dd <= L; ++dd) {
                        re += rdd[dd];
                        im += idd[dd];
                    }
                    sT[jt][d * NC + 2 * e] = re;
                    sT[jt][d * NC + 2 * e + 1] = im;
                }
            }
            wave_sync();

            // ---- X_d = C_{L,d} T_d, packed entries only (into sQ's space)
            constexpr int NK = N + NU;
            constexpr int XITEMS = (L + 1) * NK;
#pragma unroll
            for (int it = 0; it < (XITEMS + LT - 1) / LT; ++it) {
                const int idx = li + LT * it;
                if (idx < XITEMS) {
                    const int d = idx / NK, k = idx - d * NK;
                    int a = k, b = k;
                    if (k >= N) pair_of<N>(k - N, a, b);
                    double re = 0.0, im = 0.0;
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        const double2 x = ldsc(&sC[jt][d * NC], a * N + c), y = ldsc(&sT[jt][d * NC], c * N + b);
                        re = fma(x.x, y.x, fma(-x.y, y.y, re));
                        im = fma(x.x, y.y, fma(x.y, y.x, im));
                    }
                    double* X = &sQ[jt][d * NM];
                    if (k < N) {
                        X[k] = re;
                    } else {
                        X[N + 2 * (k - N)] = re;
                        X[N + 2 * (k - N) + 1] = im;
                    }
                }
            }
            wave_sync();

            // ---- density sum of stage L, its lab-frame rotation and weights
            if (li < NM) {
                const int v = li;
                double Sx = sQ[jt][v];
                for (int d = 1; d <= L; ++d) Sx += sQ[jt][d * NM + v];
                // pair partner (re with im) of an off-diagonal value
                const int vo = v < N ? v : (((v - N) & 1) ? v - 1 : v + 1);
                double So = sQ[jt][vo];
                for (int d = 1; d <= L; ++d) So += sQ[jt][d * NM + vo];
                double Sv;
                if (v < N) {
                    Sv = 2.0 * Sx;
                } else {
                    const int u = (v - N) >> 1;
                    double cs = zL[0][0], sn = zL[0][1];
#pragma unroll
                    for (int q = 1; q < NU; ++q)
                        if (u == q) {
                            cs = zL[q][0];
                            sn = zL[q][1];
                        }
                    const double xr = ((v - N) & 1) ? So : Sx, xi = ((v - N) & 1) ? Sx : So;
                    Sv = ((v - N) & 1) ? 2.0 * (cs * xi - sn * xr) : 2.0 * (cs * xr + sn * xi);
                }
                double f[4];
                angle_weights<NJ>(rc, cL, wL, cph, sph, f);
#pragma unroll
                for (int m = 0; m < NJ; ++m) swave[jt][m * NM + v] = f[m] * Sv;
            }
        }
    }
    if constexpr (!TABLES) {
        __syncthreads();
        if (tid < NV) {
            double s0 = swave[0][tid];
            for (int w = 1; w < TPB; ++w) s0 += swave[w][tid];
            gview(rc.partial)[((size_t)(L & 1) * NV + tid) * rc.pstride + blk] = s0;
        }
    }
}

// ------------------------------------------------------------------ state update
// Launch S + 1: one wavefront per trajectory, lanes over its 2 N_E beam slots
// (two groups of two beams of a lane in flight).  Per beam:
//   y_{n+1} = M(u) y_n,  M(u) = sum_d Cn_d u^d (arithmetic type T),
//   FP32 amplitudes: y_{n+1} / |y_{n+1}|, written in the storage type;
//   embedded pair: delta = E(u) y_n in FP64 (E = sum_m e_m D_m, the step error
//   h sum_m e_m k_m), and the maximum of |Re|, |Im| over the components;
//   RK4: whether the new state is finite.
// The coefficients are wave-uniform: they are read through the constant
// address space into scalar registers, once per group of beams.

// p, passed through an empty asm that also takes v: loads through the result
// cannot be issued before v has been computed.
template <typename V>
__device__ __forceinline__ uint64_t after(uint64_t p, V v)
{
    asm volatile("" : "+s"(p) : "v"(v));
    return p;
}
// The same after all NR values of v.
template <int NR, typename V>
__device__ __forceinline__ uint64_t after_all(uint64_t p, const V (&v)[NR])
{
#pragma unroll
    for (int x = 0; x < NR; ++x) asm volatile("" : "+s"(p) : "v"(v[x]));
    return p;
}

// M_g[x] = sum_{d<=D} c[d NR + x] u_g^d, x < NR, for the G beams of a group:
// one row of a coefficient matrix polynomial, stored degree after degree from
// byte address `base` (wave-uniform, read through the constant address space,
// so the coefficients arrive in scalar registers and serve all G beams),
// summed in ascending degree with the powers up[g][d] = u_g^d.  The
// coefficient is the multiplicand of every fma, so it is used straight from
// its scalar register.  The row is requested in chunks of at most 48 scalar
// registers; the address of each chunk depends on the partial sums of the
// previous one, so the compiler cannot hoist later requests (which would
// exhaust the scalar registers).
template <int D, int NR, int G, typename T, typename CT>
__device__ __forceinline__ void powsum_row(uint64_t base, const T (&up)[G][D + 1], T (&M)[G][NR])
{
    constexpr int K = (48 * 4) / (NR * (int)sizeof(CT));  // degrees per request
    constexpr int NK = (D + 1 + K - 1) / K;
    static_for<0, NK>([&](auto Kc) {
        constexpr int k = decltype(Kc)::value;
        constexpr int d0 = k * K;
        constexpr int d1 = (d0 + K < D + 1) ? d0 + K : D + 1;
        uint64_t p = base;
        if constexpr (k > 0) p = after_all(after_all(base, M[0]), M[G - 1]);
        const cptr<CT> c = reinterpret_cast<cptr<CT>>(p);
        CT cv[d1 - d0][NR];
#pragma unroll
        for (int d = d0; d < d1; ++d)
#pragma unroll
            for (int x = 0; x < NR; ++x) cv[d - d0][x] = c[d * NR + x];
#pragma unroll
        for (int d = d0; d < d1; ++d)
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int x = 0; x < NR; ++x)
                    M[g][x] = (d == 0) ? (T)cv[0][x] : fma((T)cv[d - d0][x], up[g][d], M[g][x]);
    });
}

// (P(u_g) y_g)_a for the G beams of a group and every row a, handed to
// sink(g, a, re, im) as soon as the row is formed; P is a matrix polynomial of
// degree D over full complex N x N matrices, stored row by row: row a holds
// the 2N reals (re/im of its N entries) of degree 0, then of degree 1, ...,
// (D + 1) 2N values of type CT from byte address base + a (D + 1) 2N
// sizeof(CT).  Each row's request waits for the previous row's result.
template <int D, int N, int G, typename T, typename CT, typename Sink>
__device__ __forceinline__ void poly_rows(uint64_t base, const T (&up)[G][D + 1], const T (&y)[G][2 * N],
                                          Sink&& sink)
{
    T M[G][2 * N];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int x = 0; x < 2 * N; ++x) M[g][x] = y[g][x];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const uint64_t row = after_all(after_all(base + (uint64_t)(a * (D + 1) * 2 * N * (int)sizeof(CT)), M[0]),
                                       M[G - 1]);
        powsum_row<D, 2 * N, G, T, CT>(row, up, M);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            T re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                re = fma(M[g][2 * b], y[g][2 * b], fma(-M[g][2 * b + 1], y[g][2 * b + 1], re));
                im = fma(M[g][2 * b], y[g][2 * b + 1], fma(M[g][2 * b + 1], y[g][2 * b], im));
            }
            sink(g, a, re, im);
        }
    }
}

// out_g = P(u_g) y_g (poly_rows with the rows stored).
template <int D, int N, int G, typename T, typename CT>
__device__ __forceinline__ void poly_apply(uint64_t base, const T (&up)[G][D + 1], const T (&y)[G][2 * N],
                                           T (&out)[G][2 * N])
{
    poly_rows<D, N, G, T, CT>(base, up, y, [&](int g, int a, T re, T im) __attribute__((always_inline)) {
        out[g][2 * a] = re;
        out[g][2 * a + 1] = im;
    });
}

// u^0 .. u^D.
template <int D, typename T>
__device__ __forceinline__ void powers(T u, T (&up)[D + 1])
{
    up[0] = T(1);
    up[1] = u;
#pragma unroll
    for (int d = 2; d <= D; ++d) up[d] = up[d - 1] * u;
}

// Eight wavefronts per workgroup, WPT of them on each trajectory (its beams
// dealt out in turn, G x NGRP x 64 beams at a time).  The launch bounds ask
// for four wavefronts per SIMD (at most 128 registers), which with one group
// of beams in flight the kernel fits without spilling: every trajectory's
// wavefront is resident at once on the 3.2M-beam grid.
template <typename T> struct FinalShape {
    static constexpr int waves = 8;
    static constexpr int wpt = 1;
    static constexpr int traj = waves / wpt;
    static constexpr int block = 64 * waves;
};

template <typename TS, typename T, int N, typename TAB, int NJ>
__device__ __forceinline__ void final_body(const RunConst& rc, const int blk)
{
    using PY = Poly<TAB>;
    constexpr int NC = Shape<N>::NC;
    constexpr int DN = PY::DN, DE = PY::DE;
    constexpr bool ERROR = TAB::embedded;
    constexpr int TPB = FinalShape<T>::traj;
    constexpr int WPT = FinalShape<T>::wpt;
    constexpr int NWV = FinalShape<T>::waves;
    constexpr int G = 2;       // beams of a lane sharing each coefficient load
    constexpr int NGRP = std::is_same<T, float>::value ? 2 : 1;  // groups of a lane in flight
    constexpr uint32_t STRIDE = 64;
    constexpr int EOFF = (((DN + 1) * NC * (int)sizeof(T) + 15) / 16) * 16;  // byte offset of the error table

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = blk * TPB + wave / WPT;
    const uint32_t sub = (uint32_t)(wave % WPT);
    const bool active = j < rc.na;
    __shared__ double swave[NWV];

    const global<Control>* vc = gview(rc.ctrl);  // ctrl[0]
    const int status = __hip_atomic_load(&vc->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const int cur = __hip_atomic_load(&vc->cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (status != 0) return;

    const uint32_t ne = (uint32_t)rc.ne;
    const uint32_t nbt = active ? 2u * ne : 0u;
    const uint32_t base0 = active ? (uint32_t)j * ne : 0u;
    const uint32_t delta = (uint32_t)(rc.na - 1) * ne;
    const size_t ld = (size_t)rc.nb_pad;
    // one scalar base per state buffer; component x of a beam at byte offset
    // sizeof(TS) (off + x nb_pad) (all below 4 GiB)
    global<const char>* __restrict__ srcb = uniform_global(reinterpret_cast<const char*>(rc.psi[cur]));
    global<char>* __restrict__ dstb = uniform_global(reinterpret_cast<char*>(rc.psi[cur ^ 1]));
    const uint32_t ldb = (uint32_t)(ld * sizeof(TS));
    global<const T>* __restrict__ uinv = uniform_global(uinv_table<T>(rc));
    global<const double>* __restrict__ uinv64 = uniform_global(rc.uinv64);
    const uint64_t tb0 = reinterpret_cast<uint64_t>(rc.ftab) + (uint64_t)(active ? j : 0) * (uint64_t)rc.fstride;
    // (readfirstlane returns a signed int: both halves are taken as uint32_t
    // before widening, so the low word is not sign-extended)
    const uint32_t tb_lo = __builtin_amdgcn_readfirstlane((uint32_t)tb0);
    const uint32_t tb_hi = __builtin_amdgcn_readfirstlane((uint32_t)(tb0 >> 32));
    const uint64_t tb = ((uint64_t)tb_hi << 32) | (uint64_t)tb_lo;

    double emax = 0.0;
    double chk = 0.0;  // stays 0 while every error component is finite, NaN otherwise
    bool bad = false;
    auto offset = [&](uint32_t t) __attribute__((always_inline)) { return t + base0 + (t >= ne ? delta : 0u); };
    // one group: the G beams t, t + 64, ... of the lane.  A beam past the end
    // is replaced by the trajectory's first beam, whose update is not stored
    // (its error is that beam's own, so the maximum is unchanged).  The loads
    // are unconditional: each refills its slot's registers, so the loop holds
    // no copies that would wait for loads in flight.
    auto fetch = [&](uint32_t t, TS (&yv)[G][2 * N], T (&uv)[G], double (&u64v)[G]) __attribute__((always_inline)) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t tg = t + g * STRIDE;
            const uint32_t tc = tg < nbt ? tg : 0u;
            const uint32_t off = offset(tc) * (uint32_t)sizeof(TS);
#pragma unroll
            for (int x = 0; x < 2 * N; ++x)
                yv[g][x] = load_state(reinterpret_cast<global<const TS>*>(srcb + (uint64_t)(off + (uint32_t)x * ldb)));
            uv[g] = *elem(uinv, tc);
            if constexpr (ERROR && !std::is_same<T, double>::value) u64v[g] = *elem(uinv64, tc);
        }
    };
    // the first GC of the group's G beams (GC = 1: a group whose second beam
    // slot lies wholly past the end)
    auto process = [&](auto GC, uint32_t t, const TS (&yv)[G][2 * N], const T (&u)[G], const double (&u64v)[G])
                       __attribute__((always_inline)) {
        constexpr int GG = decltype(GC)::value;
        T y[GG][2 * N], yn[GG][2 * N];
        {
            T up[GG][DN + 1];
#pragma unroll
            for (int g = 0; g < GG; ++g) {
#pragma unroll
                for (int x = 0; x < 2 * N; ++x) y[g][x] = (T)yv[g][x];
                powers<DN>(u[g], up[g]);
            }
            poly_apply<DN, N, GG, T, T>(tb, up, y, yn);
        }
#pragma unroll
        for (int g = 0; g < GG; ++g) {
            if constexpr (std::is_same<TS, float>::value) {
                // FP32 amplitudes are renormalised whenever a new state is formed
                T nn = 0;
#pragma unroll
                for (int x = 0; x < 2 * N; ++x) nn = fma(yn[g][x], yn[g][x], nn);
                const T sc = rsqrt(nn);  // renormalisation: a 1-ulp reciprocal square root suffices
#pragma unroll
                for (int x = 0; x < 2 * N; ++x) yn[g][x] = yn[g][x] * sc;
            }
            const uint32_t tg = t + g * STRIDE;
            if (tg < nbt) {
                const uint32_t off = offset(tg) * (uint32_t)sizeof(TS);
#pragma unroll
                for (int x = 0; x < 2 * N; ++x)
                    *reinterpret_cast<global<TS>*>(dstb + (uint64_t)(off + (uint32_t)x * ldb)) = (TS)yn[g][x];
                if constexpr (!ERROR) {
#pragma unroll
                    for (int x = 0; x < 2 * N; ++x) bad |= !isfinite(yn[g][x]);
                }
            }
        }
        if constexpr (ERROR) {
            double y64[GG][2 * N], up[GG][DE + 1];
#pragma unroll
            for (int g = 0; g < GG; ++g) {
#pragma unroll
                for (int x = 0; x < 2 * N; ++x) y64[g][x] = (double)yv[g][x];
                if constexpr (std::is_same<T, double>::value) powers<DE>((double)u[g], up[g]);
                else powers<DE>(u64v[g], up[g]);
            }
            // the error's max-norm, each row folded in as it is formed
            poly_rows<DE, N, GG, double, double>(
                after_all(tb + EOFF, yn[0]), up, y64, [&](int, int, double re, double im) __attribute__((always_inline)) {
                    emax = fmax(emax, fmax(fabs(re), fabs(im)));
                    chk = fma(re, 0.0, fma(im, 0.0, chk));
                });
        }
    };

    TS ys[NGRP][G][2 * N];
    T us[NGRP][G];
    double u64s[NGRP][G] = {};
    constexpr uint32_t SPAN = NGRP * G * STRIDE;  // beams of one pass of a wavefront
    const uint32_t t0 = (uint32_t)lane + sub * SPAN;
    static_for<0, NGRP>([&](auto Sc) {
        constexpr int sl = decltype(Sc)::value;
        fetch(t0 + sl * G * STRIDE, ys[sl], us[sl], u64s[sl]);
    });
    // wave-uniform loop over the passes; a group wholly past the end is
    // skipped, one whose later beam slots are is formed for its first only
#pragma unroll 1
    for (uint32_t tw = sub * SPAN; tw < nbt; tw += WPT * SPAN) {
        static_for<0, NGRP>([&](auto Sc) {
            constexpr int sl = decltype(Sc)::value;
            const uint32_t ts = tw + (uint32_t)lane + sl * G * STRIDE;
            const uint32_t gs = tw + sl * G * STRIDE;  // first beam slot of the group (wave-uniform)
            if (gs + (G - 1) * STRIDE < nbt)
                process(std::integral_constant<int, G>{}, ts, ys[sl], us[sl], u64s[sl]);
            else if (gs < nbt)
                process(std::integral_constant<int, 1>{}, ts, ys[sl], us[sl], u64s[sl]);
            fetch(ts + WPT * SPAN, ys[sl], us[sl], u64s[sl]);
        });
    }

    double e = (bad || chk != chk) ? (double)INFINITY : emax;
    e = wave_max_rows(e);
    if (lane == 0) swave[wave] = active ? e : 0.0;
    __syncthreads();
    if (tid == 0) {
        double m = swave[0];
        for (int w = 1; w < NWV; ++w) m = fmax(m, swave[w]);
        gview(rc.errpart)[blk] = m;
    }
}

// ------------------------------------------------------------------ kernels
template <typename TS, int N, typename TAB, int NJ, bool FORCE>
__global__ void __launch_bounds__(64 * kPowerWaves) k_power(const LaunchSet ls)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    power_body<TS, N, TAB, NJ, FORCE>(rc, blk);
}
template <typename TS, int N, typename TAB, int NJ, bool FORCE>
__global__ void __launch_bounds__(64 * kPowerWaves) k_power_one(const RunConst rc)
{
    power_body<TS, N, TAB, NJ, FORCE>(rc, blockIdx.x);
}

template <int N, typename TAB, int NJ, int L, typename TF>
__global__ void __launch_bounds__(64 * kTrajWaves) k_traj(const LaunchSet ls)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    traj_body<N, TAB, NJ, L, TF>(rc, blk);
}
template <int N, typename TAB, int NJ, int L, typename TF>
__global__ void __launch_bounds__(64 * kTrajWaves) k_traj_one(const RunConst rc)
{
    traj_body<N, TAB, NJ, L, TF>(rc, blockIdx.x);
}

template <typename TS, typename T, int N, typename TAB, int NJ>
__global__ void __launch_bounds__(FinalShape<T>::block, 4) k_final(const LaunchSet ls)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    final_body<TS, T, N, TAB, NJ>(rc, blk);
}
template <typename TS, typename T, int N, typename TAB, int NJ>
__global__ void __launch_bounds__(FinalShape<T>::block, 4) k_final_one(const RunConst rc)
{
    final_body<TS, T, N, TAB, NJ>(rc, blockIdx.x);
}

// J_0 of the current state from the power-moment launch's partials (after a
// new state or radius): one workgroup per run.
template <int NV>
__device__ __forceinline__ void jsum_body(const RunConst& rc)
{
    constexpr int NW = kFinBlock / 64;
    __shared__ double sJ[NV];
    PartialRegs<NV, NW> x;
    load_partials<NV, NW>(rc, 0, rc.nblkp, x);
    finish_partials<NV, NW>(rc, 0, rc.nblkp, x, sJ);
    if ((int)threadIdx.x < NV) gview(rc.jhist)[threadIdx.x] = sJ[threadIdx.x];
}
template <int NV>
__global__ void __launch_bounds__(kFinBlock) k_jsum(const LaunchSet ls)
{
    int blk;
    jsum_body<NV>(ls.runs[run_of_block(ls, blk)]);
}
template <int NV>
__global__ void __launch_bounds__(kFinBlock) k_jsum_one(const RunConst rc)
{
    jsum_body<NV>(rc);
}

// ------------------------------------------------------------------ small kernels
template <typename T, int N>
__global__ void k_probabilities(const LaunchSet ls, double* __restrict__ p)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    const int64_t b = (int64_t)blk * blockDim.x + threadIdx.x;
    if (b >= rc.nb) return;
    const T* src = reinterpret_cast<const T*>(rc.psi[rc.ctrl[1].cur]);
    const double re = (double)src[0 * rc.nb_pad + b], im = (double)src[1 * rc.nb_pad + b];
    p[b] = re * re + im * im;
}

// Energy-averaged flavor content of every trajectory (the paper's second
// dump mode, Section 4.2.4): for species s and trajectory j,
//   out[s][j][a] = sum_k f_sk |psi_{s,j,k,a}|^2 / sum_k f_sk,
// f_sk the number flux of the species' birth flavor (nu_e, nubar_e) in
// energy bin k (eq 4.1-4.2); the plain mean over bins if it sums to zero.
// |psi_a|^2 is the same in the co-rotating frame and for the conjugated
// antineutrino amplitudes held on the device.  One wavefront per trajectory,
// lanes over its beam slots; FP64 sums.  It reads the state once.
constexpr int kAvgTraj = 4;  // trajectories (wavefronts) per workgroup
template <typename T, int N>
__global__ void __launch_bounds__(64 * kAvgTraj) k_energy_average(const LaunchSet ls, double* __restrict__ out)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    const int lane = threadIdx.x & 63;
    const int j = blk * kAvgTraj + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (j >= rc.na) return;
    const uint32_t ne = (uint32_t)rc.ne;
    const uint32_t delta = (uint32_t)(rc.na - 1) * ne;
    const uint32_t base0 = (uint32_t)j * ne;
    const T* src = reinterpret_cast<const T*>(rc.psi[rc.ctrl[1].cur]);
    global<const T>* __restrict__ q0 = uniform_global(src);
    const size_t ld = (size_t)rc.nb_pad;
    // weighted sums, weight sums, plain sums and bin counts per species
    double num[2][N], pm[2][N], den[2], cnt[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        den[s] = cnt[s] = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) num[s][a] = pm[s][a] = 0.0;
    }
    // four beams of each lane per round: all their loads issued first
    constexpr int U = 4;
    for (uint32_t t0 = lane; t0 < 2u * ne; t0 += 64 * U) {
        T y[U][2 * N];
        double g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t t = t0 + 64 * u;
            const uint32_t off = t + base0 + (t >= ne ? delta : 0u);
            g[u] = 0.0;
            if (t < 2u * ne) {
                g[u] = rc.flux[t];
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) y[u][q] = *elem(q0 + q * ld, off);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t t = t0 + 64 * u;
            if (t >= 2u * ne) break;
            const bool nub = t >= ne;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const double re = (double)y[u][2 * a], im = (double)y[u][2 * a + 1];
                const double v = re * re + im * im;
                num[0][a] += nub ? 0.0 : g[u] * v;
                num[1][a] += nub ? g[u] * v : 0.0;
                pm[0][a] += nub ? 0.0 : v;
                pm[1][a] += nub ? v : 0.0;
            }
            den[0] += nub ? 0.0 : g[u];
            den[1] += nub ? g[u] : 0.0;
            cnt[0] += nub ? 0.0 : 1.0;
            cnt[1] += nub ? 1.0 : 0.0;
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        den[s] = wave_sum(den[s]);
        cnt[s] = wave_sum(cnt[s]);
#pragma unroll
        for (int a = 0; a < N; ++a) {
            num[s][a] = wave_sum(num[s][a]);
            pm[s][a] = wave_sum(pm[s][a]);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < N; ++a)
                out[((size_t)s * rc.na + j) * N + a] = den[s] != 0.0 ? num[s][a] / den[s] : pm[s][a] / cnt[s];
    }
}

template <typename T, int N>
__global__ void k_init(const LaunchSet ls)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    const int64_t b = (int64_t)blk * blockDim.x + threadIdx.x;
    if (b < rc.nb_pad) {
        T* dst = reinterpret_cast<T*>(rc.psi[rc.ctrl[1].cur]);
        for (int q = 0; q < 2 * N; ++q) dst[q * rc.nb_pad + b] = (q == 0 && b < rc.nb) ? T(1) : T(0);
    }
    if (b < (int64_t)rc.na * N) rc.phase[rc.ctrl[1].cur][b] = 0.0;
}

// ------------------------------------------------------------------ dispatch
using KernFn = void (*)(const LaunchSet);
using OneFn = void (*)(const RunConst);

// The kernels of one launch: over launch sets (k, f) and over one run (k1,
// f1); f, f1: the second kernel (launch 0 only), else nullptr.  grid: which
// workgroup count the main kernel takes (0: nblk, 1: nblkf).
struct StageKernels {
    KernFn k = nullptr, f = nullptr;
    OneFn k1 = nullptr, f1 = nullptr;
    unsigned block = 0;
    int grid = 0;  // workgroups: 0 nblk (per-trajectory launches), 1 nblkf (state update), 2 nblkp (power moments)
};

template <typename TF, int N, typename TAB, int NJ, int L>
using TrajTF = typename std::conditional<L == TAB::S, TF, double>::type;

template <typename TF, int N, typename TAB, int NJ>
struct TrajTable {
    static constexpr int clamp(int l) { return (l >= 1 && l <= TAB::S) ? l : 1; }
    template <int... Is>
    static constexpr std::array<KernFn, kMaxLaunches> make(std::integer_sequence<int, Is...>)
    {
        return {{((Is >= 1 && Is <= TAB::S)
                      ? (KernFn)&k_traj<N, TAB, NJ, clamp(Is), TrajTF<TF, N, TAB, NJ, clamp(Is)>>
                      : nullptr)...}};
    }
    template <int... Is>
    static constexpr std::array<OneFn, kMaxLaunches> make1(std::integer_sequence<int, Is...>)
    {
        return {{((Is >= 1 && Is <= TAB::S)
                      ? (OneFn)&k_traj_one<N, TAB, NJ, clamp(Is), TrajTF<TF, N, TAB, NJ, clamp(Is)>>
                      : nullptr)...}};
    }
    static constexpr std::array<KernFn, kMaxLaunches> fns = make(std::make_integer_sequence<int, kMaxLaunches>{});
    static constexpr std::array<OneFn, kMaxLaunches> fns1 = make1(std::make_integer_sequence<int, kMaxLaunches>{});
};

template <typename TS, typename T, int N, typename TAB, int NJ>
void pick_tab(int stage, StageKernels& K)
{
    constexpr int S = TAB::S;
    if (stage == 0) {
        K.k = (KernFn)&k_power<TS, N, TAB, NJ, true>;
        K.k1 = (OneFn)&k_power_one<TS, N, TAB, NJ, true>;
        K.f = (KernFn)&k_jsum<NJ * N * N>;
        K.f1 = (OneFn)&k_jsum_one<NJ * N * N>;
        K.block = 64 * kPowerWaves;
        K.grid = 2;
    } else if (stage <= S) {
        K.k = TrajTable<T, N, TAB, NJ>::fns[stage];
        K.k1 = TrajTable<T, N, TAB, NJ>::fns1[stage];
        K.block = 64 * kTrajWaves;
    } else if (stage == S + 1) {
        K.k = (KernFn)&k_final<TS, T, N, TAB, NJ>;
        K.k1 = (OneFn)&k_final_one<TS, T, N, TAB, NJ>;
        K.block = FinalShape<T>::block;
        K.grid = 1;
    } else if (stage == S + 2) {
        K.k = (KernFn)&k_power<TS, N, TAB, NJ, false>;
        K.k1 = (OneFn)&k_power_one<TS, N, TAB, NJ, false>;
        K.block = 64 * kPowerWaves;
        K.grid = 2;
    }
}

template <typename TS, typename T, int NJ>
void pick_n(int n, int integrator, int stage, StageKernels& K)
{
    if (n == 2) {
        if (integrator == 0) pick_tab<TS, T, 2, TabRK4, NJ>(stage, K);
        else pick_tab<TS, T, 2, TabDP54, NJ>(stage, K);
    } else {
        if (integrator == 0) pick_tab<TS, T, 3, TabRK4, NJ>(stage, K);
        else pick_tab<TS, T, 3, TabDP54, NJ>(stage, K);
    }
}

// The bulb model (two angle moments) or the extended one (four).
template <typename TS, typename T>
void pick_nj(int nj, int n, int integrator, int stage, StageKernels& K)
{
    if (nj == 4) pick_n<TS, T, 4>(n, integrator, stage, K);
    else pick_n<TS, T, 2>(n, integrator, stage, K);
}

// Launches fn over the listed runs, at most kMaxRuns runs per launch, with
// blocks(rc) workgroups per run; launches nothing for an empty list.
template <typename Blocks, typename Launch>
hipError_t for_launch_sets(const RunList& runs, Blocks blocks, Launch launch)
{
    for (int i0 = 0; i0 < runs.count; i0 += kMaxRuns) {
        LaunchSet ls{};
        ls.runs = runs.runs_dev;
        ls.count = runs.count - i0 < kMaxRuns ? runs.count - i0 : kMaxRuns;
        ls.first[0] = 0;
        for (int i = 0; i < ls.count; ++i) {
            ls.slot[i] = runs.slot[i0 + i];
            const long long nb = blocks(*runs.rc[i0 + i]);
            if (nb < 1 || (long long)ls.first[i] + nb > 0x7fffffffLL) return hipErrorInvalidValue;
            ls.first[i + 1] = ls.first[i] + (int)nb;
        }
        hipError_t e = launch(ls, (unsigned)ls.first[ls.count]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

bool same_kind(const RunList& runs)
{
    for (int i = 1; i < runs.count; ++i) {
        const RunConst& a = *runs.rc[0];
        const RunConst& b = *runs.rc[i];
        if (a.n != b.n || a.precision != b.precision || a.integrator != b.integrator || a.nj != b.nj) return false;
    }
    return true;
}

}  // namespace

int num_stages(int integrator) { return (integrator == 0 ? TabRK4::S : TabDP54::S) + 2; }

PolySizes poly_sizes(int n, int integrator, int precision)
{
    const int nm = n * n, nc = 2 * n * n;
    const int S = integrator == 0 ? TabRK4::S : TabDP54::S;
    const int nq = 2 * (S - 1) + 1;
    const int nd = (S - 1) * (S + 2) / 2;  // matrices of D_0 .. D_{S-2}
    const int dn = integrator == 0 ? Poly<TabRK4>::DN : Poly<TabDP54>::DN;
    const int de = integrator == 0 ? -1 : Poly<TabDP54>::DE;
    const int tsz = precision == 1 ? 4 : 8;
    PolySizes p;
    p.qstride = nq * nc;  // full complex matrices (16-byte entries)
    p.dstride = (nd * nc + 7) / 8 * 8;
    const int cn = ((dn + 1) * nc * tsz + 15) / 16 * 16;  // the error table starts 16-byte aligned
    const int ce = (de + 1) * nc * 8;
    p.fstride = (cn + ce + 255) / 256 * 256;
    return p;
}

hipError_t launch_stage(const RunList& runs, int stage, hipStream_t s, hipEvent_t* ev)
{
    if (runs.count < 1) return hipSuccess;
    if (!same_kind(runs)) return hipErrorInvalidValue;
    const RunConst& r0 = *runs.rc[0];
    if (stage < 0 || stage > num_stages(r0.integrator)) return hipErrorInvalidValue;
    StageKernels K;
    switch (r0.precision) {
    case 0: pick_nj<double, double>(r0.nj, r0.n, r0.integrator, stage, K); break;  // FP64
    case 1: pick_nj<float, float>(r0.nj, r0.n, r0.integrator, stage, K); break;    // FP32 amplitudes
    case 2: pick_nj<float, double>(r0.nj, r0.n, r0.integrator, stage, K); break;   // FP32 amplitudes, FP64 math
    default: break;
    }
    if (!K.k || !K.k1) return hipErrorInvalidValue;
    const bool one = runs.count == 1;
    auto blocks = [&](const RunConst& rc) {
        return (long long)(K.grid == 1 ? rc.nblkf : K.grid == 2 ? rc.nblkp : rc.nblk);
    };
    if (ev) {
        hipError_t e = hipEventRecord(ev[0], s);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipSuccess;
    if (one) {
        hipLaunchKernelGGL(K.k1, dim3((unsigned)blocks(r0)), dim3(K.block), 0, s, r0);
        e = hipGetLastError();
    } else {
        e = for_launch_sets(runs, blocks, [&](const LaunchSet& ls, unsigned grid) {
            hipLaunchKernelGGL(K.k, dim3(grid), dim3(K.block), 0, s, ls);
            return hipGetLastError();
        });
    }
    if (e != hipSuccess) return e;
    if (ev) {
        e = hipEventRecord(ev[1], s);
        if (e != hipSuccess) return e;
    }
    if (K.f && one) {
        hipLaunchKernelGGL(K.f1, dim3(1), dim3(kFinBlock), 0, s, r0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    } else if (K.f) {
        e = for_launch_sets(runs, [](const RunConst&) { return 1LL; }, [&](const LaunchSet& ls, unsigned grid) {
            hipLaunchKernelGGL(K.f, dim3(grid), dim3(kFinBlock), 0, s, ls);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    if (ev) {
        e = hipEventRecord(ev[2], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_probabilities(const RunList& runs, double* p, hipStream_t s)
{
    if (runs.count < 1) return hipSuccess;
    const RunList one{runs.runs_dev, 1, runs.slot, runs.rc};
    const RunConst& r0 = *runs.rc[0];
    using PFn = void (*)(const LaunchSet, double*);
    PFn k;
    if (r0.precision == 0) k = r0.n == 2 ? (PFn)&k_probabilities<double, 2> : (PFn)&k_probabilities<double, 3>;
    else k = r0.n == 2 ? (PFn)&k_probabilities<float, 2> : (PFn)&k_probabilities<float, 3>;
    return for_launch_sets(one, [](const RunConst& rc) { return (long long)((rc.nb + 255) / 256); },
                           [&](const LaunchSet& ls, unsigned grid) {
                               hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, s, ls, p);
                               return hipGetLastError();
                           });
}

hipError_t launch_energy_average(const RunList& runs, double* out, hipStream_t s)
{
    if (runs.count < 1) return hipSuccess;
    const RunList one{runs.runs_dev, 1, runs.slot, runs.rc};
    const RunConst& r0 = *runs.rc[0];
    using AFn = void (*)(const LaunchSet, double*);
    AFn k;
    if (r0.precision == 0) k = r0.n == 2 ? (AFn)&k_energy_average<double, 2> : (AFn)&k_energy_average<double, 3>;
    else k = r0.n == 2 ? (AFn)&k_energy_average<float, 2> : (AFn)&k_energy_average<float, 3>;
    return for_launch_sets(one, [](const RunConst& rc) { return (long long)((rc.na + kAvgTraj - 1) / kAvgTraj); },
                           [&](const LaunchSet& ls, unsigned grid) {
                               hipLaunchKernelGGL(k, dim3(grid), dim3(64 * kAvgTraj), 0, s, ls, out);
                               return hipGetLastError();
                           });
}

hipError_t launch_init_state(const RunList& runs, hipStream_t s)
{
    if (runs.count < 1) return hipSuccess;
    if (!same_kind(runs)) return hipErrorInvalidValue;
    const RunConst& r0 = *runs.rc[0];
    KernFn k;
    if (r0.precision == 0) k = r0.n == 2 ? (KernFn)&k_init<double, 2> : (KernFn)&k_init<double, 3>;
    else k = r0.n == 2 ? (KernFn)&k_init<float, 2> : (KernFn)&k_init<float, 3>;
    auto blocks = [](const RunConst& rc) {
        const long long work = rc.nb_pad > (long long)rc.na * rc.n ? rc.nb_pad : (long long)rc.na * rc.n;
        return (work + 255) / 256;
    };
    return for_launch_sets(runs, blocks, [&](const LaunchSet& ls, unsigned grid) {
        hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, s, ls);
        return hipGetLastError();
    });
}

// The device memory of runs made without allocation.  Host code never uses
// the array's name as an address: the kernels get the address that
// hipGetSymbolAddress reports for the current device.
hipError_t static_scratch(int* device, void** addr)
{
    static std::mutex mu;
    static void* base[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!base[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        base[dev] = p;
    }
    *device = dev;
    *addr = base[dev];
    return hipSuccess;
}

}  // namespace nuosc
