// gfx950 kernels of the bulb-model flavor evolution.
//
// One step attempt of an explicit Runge-Kutta tableau with S stages runs as S
// beam launches k_stage<I>, I = 1..S, and one control launch:
//   * k_stage<I> (one wavefront per emission-angle trajectory j, lanes over
//     its 2 N_E beams):
//       prologue: every workgroup adds the partial density sums of launch I-1
//         in one fixed order (all workgroups get the same J_{I-1}; launch 1
//         takes J_0 of the accepted state) and completes stage I-1 of its own
//         trajectories: collective Hamiltonian (eq 3.13 / 3.16), matter term,
//         frame rate G, stage matrices h K_{I-1} = h (A + B u);
//       beam loop: reads y_n once, recomputes k_0..k_{I-1} from y_n and the
//         stage matrices, forms the input of stage I (the new state in the
//         launch that forms it, written back in the storage type) and adds
//         its weighted density matrix in FP64.  Embedded pair with first
//         same as last (k_{S-1} = f(y_{n+1})): launch S-1 also writes the
//         partial error sum sum_{i<S-1} e_i k_i per beam, and launch S reads
//         it with y_{n+1}, evaluates k_{S-1} only and forms the step error
//         h sum_i e_i k_i;
//       epilogue: prepares stage I (geometry eq 3.14-3.15, co-rotating phase,
//         rotation factors) and adds the rotated, angle-weighted density sums
//         of its trajectories into one partial per workgroup.
//   * k_control (one workgroup per run): global error maximum, step
//     controller, and J_0 of the next attempt.
// Only y_n is read from HBM per beam launch and only y_{n+1} is written (by
// the launch that forms it, with the partial error sum): every stage
// derivative is recomputed from y_n and the small per-trajectory tables
// instead of being stored.
//
// Antineutrino amplitudes are held complex-conjugated on the device.  With
// phi = conj(psibar), the antineutrino equation in the co-rotating frame reads
// d phi / dr = -i (A - B / E) phi with the neutrino's A and B, so one matrix
// per trajectory and stage serves both species (u = +1/E or -1/E per beam),
// and the density sum takes the same form g psi psi^dagger for both species
// with weight g or -gbar.
#include "nuosc_internal.hpp"

#include <math.h>
#include <array>
#include <type_traits>
#include <utility>

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
    [[maybe_unused]] static constexpr double E[8] = {0};
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

// Coefficient of k_m in the state formed for stage l (l == S: the new state).
template <typename TAB>
__host__ __device__ constexpr double coef(int l, int m)
{
    return l < TAB::S ? TAB::A[l][m] : TAB::B[m];
}

// ------------------------------------------------------------------ helpers
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// coef(l, M) for a runtime stage l in (M, LAST], else 0.
template <typename TAB, int M, int LAST>
__device__ __forceinline__ double coef_of_column(int l)
{
    double r = 0.0;
    static_for<M + 1, LAST + 1>([&](auto Lc) {
        constexpr int ll = decltype(Lc)::value;
        if (l == ll) r = coef<TAB>(ll, M);
    });
    return r;
}

// Lane k < NV stores v[k] to dst[k]: NV values that every lane of the
// wavefront holds, written with one store instruction instead of NV.
template <int NV, typename D>
__device__ __forceinline__ void lane_scatter(D* dst, const double (&v)[NV], int lane)
{
    if (lane < NV) {
        double x = v[0];
#pragma unroll
        for (int k = 1; k < NV; ++k) {
            x = (lane == k) ? v[k] : x;
            asm volatile("" : "+v"(x));  // a select chain, not a table in scratch memory
        }
        dst[lane] = (D)x;
    }
}

// Empty asm that takes v as a register operand: the computation of v must be
// complete here, which bounds how far the scheduler spreads one stage's loads
// and arithmetic into the next (register pressure).  Emits no instruction.
template <typename T>
__device__ __forceinline__ void pin(T& v)
{
    asm volatile("" : "+v"(v));
}

// Element i of an array at a wave-uniform base: a 32-bit byte offset from a
// 64-bit base, which maps onto the scalar-base + vector-offset addressing of
// global loads and stores (every array indexed this way is below 4 GiB).
template <typename T>
__device__ __forceinline__ T* elem(T* base, uint32_t i)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + (uint64_t)(i * (uint32_t)sizeof(T)));
}

// Global-memory views of the beam arrays.  uniform_global(p) takes a
// wave-uniform pointer into a scalar register as a global-address-space
// pointer: loads and stores through it become global (not flat) operations
// with a scalar base and a 32-bit vector offset, and one such base per
// amplitude component keeps the per-component address arithmetic out of the
// vector ALU.
template <typename T> using global = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ global<T>* uniform_global(T* p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return reinterpret_cast<global<T>*>(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ global<T>* elem(global<T>* base, uint32_t i)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<global<T>*>(reinterpret_cast<global<B>*>(base) + (uint64_t)(i * (uint32_t)sizeof(T)));
}

// K y for one beam with K = A + B u (packed Hermitian).  y, ky: [2N] as (re,
// im) per component.  The derivative is k = -i K y: Re k_a = Im (K y)_a and
// Im k_a = -Re (K y)_a.  The kernels keep K y and fold -i into the Runge-Kutta
// coefficients (c k[q] = ksign(q) c ky[q ^ 1]), which saves the negations.
template <typename T, int N>
__device__ __forceinline__ void eval_ky(const T* A, const T* B, T u, const T* y, T* k)
{
    constexpr int NU = Shape<N>::NU;
    T kd[N], ku[NU][2];
#pragma unroll
    for (int a = 0; a < N; ++a) kd[a] = fma(B[a], u, A[a]);
#pragma unroll
    for (int q = 0; q < NU; ++q) {
        ku[q][0] = fma(B[N + 2 * q], u, A[N + 2 * q]);
        ku[q][1] = fma(B[N + 2 * q + 1], u, A[N + 2 * q + 1]);
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
        T p = kd[a] * y[2 * a], q = kd[a] * y[2 * a + 1];
#pragma unroll
        for (int b = 0; b < N; ++b) {
            if (b == a) continue;
            T kr, ki;
            if (a < b) { kr = ku[Shape<N>::up(a, b)][0]; ki = ku[Shape<N>::up(a, b)][1]; }
            else { kr = ku[Shape<N>::up(b, a)][0]; ki = -ku[Shape<N>::up(b, a)][1]; }
            p = fma(kr, y[2 * b], fma(-ki, y[2 * b + 1], p));
            q = fma(kr, y[2 * b + 1], fma(ki, y[2 * b], q));
        }
        k[2 * a] = p;
        k[2 * a + 1] = q;
    }
}

__host__ __device__ constexpr double ksign(int q) { return (q & 1) ? -1.0 : 1.0; }

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

// ------------------------------------------------------------------ per-trajectory tables
// Stage radius l of the attempt described by C (l == S: the new state).
template <typename TAB>
__device__ __forceinline__ double stage_radius(const RunConst& rc, const Control& C, int l)
{
    if (l < TAB::S) return C.r + TAB::C[l] * C.h;
    return (rc.integrator == 0) ? rc.r_start + (double)(C.istep + 1) * rc.h_fixed : C.r + C.h;
}

// Geometry of trajectory j at radius r (eq 3.14-3.15, with 1 - (R/r)^2 formed
// as (r - R)(r + R) / r^2; single angle: c = 1, w = D(r/R) of eq 3.17).
__device__ __forceinline__ void traj_geometry(const RunConst& rc, int j, double r, double& c, double& w)
{
    const double x = (rc.r_nu / r) * (rc.r_nu / r);
    const double y = (r - rc.r_nu) * (r + rc.r_nu) / (r * r);
    if (rc.ma) {
        // trajectory j: emission-angle bin j / np, azimuth bin j % np (the
        // azimuth bins share the emission-angle weight)
        const double du = 1.0 / (double)rc.nth;
        const double u = ((double)(rc.np > 1 ? j / rc.np : j) + 0.5) * du;
        c = sqrt(fma(1.0 - u * u, y, u * u));
        w = x * u * du / c;
        if (rc.np > 1) w /= (double)rc.np;
    } else {
        c = 1.0;
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

// Frame data of one trajectory at one stage radius.
template <int N>
struct Frame {
    double c, w, wc, ic, s;
    double z[Shape<N>::NU > 0 ? Shape<N>::NU : 1][2];  // e^{i(Phi_a - Phi_b)}, upper pairs
};

// Index pair (a, b), a < b, of upper entry q.
template <int N>
__device__ __forceinline__ void pair_of(int q, int& a, int& b)
{
    a = 0;
    b = 1;
    for (int aa = 0; aa < N; ++aa)
        for (int bb = aa + 1; bb < N; ++bb)
            if (Shape<N>::up(aa, bb) == q) { a = aa; b = bb; }
}

// Frame of stage l of trajectory j with geometry (c, w) and co-rotating
// phases ph[], computed by one wavefront: the NU rotation factors one per lane
// (lanes 0..NU-1) and broadcast.  Lane 0 stores it in geo[l].
template <int N>
__device__ Frame<N> prepare_wave(const RunConst& rc, int j, int l, double c, double w, const double* ph, int lane)
{
    constexpr int NU = Shape<N>::NU;
    Frame<N> f;
    f.c = c;
    f.w = w;
    f.wc = rc.ma ? f.w * f.c : 0.0;
    f.ic = 1.0 / f.c;
    f.s = sqrt((1.0 - f.c) * (1.0 + f.c));
    int a, b;
    pair_of<N>(lane < NU ? lane : 0, a, b);
    double sn, cs;
    sincos(ph[a] - ph[b], &sn, &cs);
#pragma unroll
    for (int q = 0; q < NU; ++q) {
        f.z[q][0] = __shfl(cs, q, 64);
        f.z[q][1] = __shfl(sn, q, 64);
    }
    TrajGeo& g = rc.geo[(size_t)l * rc.na + j];
    const double head[4] = {f.c, f.w, f.wc, f.ic};
    double zz[2 * (NU > 0 ? NU : 1)];
    for (int q = 0; q < NU; ++q) {
        zz[2 * q] = f.z[q][0];
        zz[2 * q + 1] = f.z[q][1];
    }
    lane_scatter(&g.c, head, lane);    // c, w, wc, ic are contiguous
    if constexpr (NU > 0) lane_scatter(&g.z[0][0], zz, lane);
    return f;
}

// The same frame computed by one thread (for the stage-0 preparation kernel);
// the same arithmetic, so the same bits.
template <int N>
__device__ void prepare_thread(const RunConst& rc, int j, int l, double rl, const double* ph)
{
    constexpr int NU = Shape<N>::NU;
    TrajGeo& g = rc.geo[(size_t)l * rc.na + j];
    double c, w;
    traj_geometry(rc, j, rl, c, w);
    g.c = c;
    g.w = w;
    g.wc = rc.ma ? w * c : 0.0;
    g.ic = 1.0 / c;
    for (int q = 0; q < NU; ++q) {
        int a, b;
        pair_of<N>(q, a, b);
        double sn, cs;
        sincos(ph[a] - ph[b], &sn, &cs);
        g.z[q][0] = cs;
        g.z[q][1] = sn;
    }
}

// Completes stage l of trajectory j from J_l (J0, J1 and for the extended
// model J2, J3, packed) and the matter potential lam at the stage radius
// (uniform values in every lane):
//   C = mu0 traceless(J0 - c J1)                       (eq 3.13; single angle: J1 = 0)
//   extended model (eq 3.18): C = mu0 traceless(J0 - c J1 - sc J2 - ss J3),
//     sc = sin(theta) cos(phi), ss = sin(theta) sin(phi) of the trajectory
//   G = diag(H_m + C) / c in the co-rotating frame, 0 in the lab frame
//   A_ab = e^{i(Phi_a - Phi_b)} C_ab / c (a < b), A_aa = 0 (co-rotating) or (H_m + C)_aa / c (lab)
//   B_ab = e^{i(Phi_a - Phi_b)} V_ab / c,  B_aa = V_aa / c  (H_vac = V / E)
// Stores h A and h B (the step size folded in: the beam kernels form
// h k = -i h K y directly) in mat[l] and in M (LDS); G is returned.
template <typename T, int N, int NJ>
__device__ void complete_wave(const RunConst& rc, int j, int l, const double c, const double ic, double sc,
                              double ss, const double (*z)[2], double lam, const double* J, double h, double* G,
                              StageMat<T, N>* M, int lane)
{
    constexpr int NM = Shape<N>::NM;
    // the angle-kernel combination of the moments for value x of the packed matrix
    auto kern = [&](int x) __attribute__((always_inline)) {
        double v = J[x] - c * J[NM + x];
        if constexpr (NJ == 4) v = (v - sc * J[2 * NM + x]) - ss * J[3 * NM + x];
        return v;
    };
    double Cd[N], tr = 0.0;
    for (int a = 0; a < N; ++a) {
        Cd[a] = kern(a);
        tr += Cd[a];
    }
    double av[NM], bv[NM];
    for (int a = 0; a < N; ++a) {
        const double hd = lam * ((a == 0 ? 1.0 : 0.0) - 1.0 / N) + rc.mu0 * (Cd[a] - tr / N);
        G[a] = (rc.frame == 0) ? hd * ic : 0.0;
        av[a] = (rc.frame == 0) ? 0.0 : hd * ic;
        bv[a] = rc.vac[a][a][0] * ic;
    }
    for (int a = 0; a < N; ++a)
        for (int b = a + 1; b < N; ++b) {
            const int q = Shape<N>::up(a, b);
            const double cs = z[q][0], sn = z[q][1];
            const double cr = rc.mu0 * kern(N + 2 * q) * ic;
            const double ci = rc.mu0 * kern(N + 2 * q + 1) * ic;
            const double vr = rc.vac[a][b][0] * ic, vi = rc.vac[a][b][1] * ic;
            av[N + 2 * q] = cs * cr - sn * ci;
            av[N + 2 * q + 1] = cs * ci + sn * cr;
            bv[N + 2 * q] = cs * vr - sn * vi;
            bv[N + 2 * q + 1] = cs * vi + sn * vr;
        }
    double hab[2 * NM];
    for (int x = 0; x < NM; ++x) {
        hab[x] = h * av[x];
        hab[NM + x] = h * bv[x];
    }
    StageMat<T, N>& Mh = reinterpret_cast<StageMat<T, N>*>(rc.mat)[(size_t)l * rc.na + j];
    lane_scatter(Mh.a, hab, lane);   // a and b are contiguous
    lane_scatter(M->a, hab, lane);
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

// Sum of the value-major partials of stage `st` (nblk workgroups) into
// out[NV] (LDS), by all BLK threads of a workgroup in one fixed order: thread
// (v, c) adds partials c, c + CH, ... of value v (CH = BLK / NV chunks per
// value), then one thread per value adds the CH chunk sums.  Every workgroup
// running this gets the same bits.
template <int NV, int BLK>
__device__ void reduce_partials(const RunConst& rc, int st, double* out, double (*sred)[BLK / NV])
{
    constexpr int CH = BLK / NV;
    const int t = threadIdx.x;
    const int nblk = rc.nblk;
    const double* src = rc.partial + (size_t)(st & 1) * NV * nblk;
    if (t < NV * CH) {
        const int v = t / CH, c = t - v * CH;
        const double* pv = src + (size_t)v * nblk;
        double acc = 0.0;
        int p = c;
        for (; p + 3 * CH < nblk; p += 4 * CH) {
            const double x0 = pv[p], x1 = pv[p + CH], x2 = pv[p + 2 * CH], x3 = pv[p + 3 * CH];
            acc += x0;
            acc += x1;
            acc += x2;
            acc += x3;
        }
        for (; p < nblk; p += CH) acc += pv[p];
        sred[v][c] = acc;
    }
    __syncthreads();
    if (t < NV) {
        double sum = sred[t][0];
        for (int c = 1; c < CH; ++c) sum += sred[t][c];
        out[t] = sum;
    }
    __syncthreads();
}

// The same sum done by the NW wavefronts of a workgroup: value v by wavefront
// v mod NW, lane l adding partials l, l + 64, ... in order, then a butterfly
// whose lane-0 result is kept (one fixed order).  Every workgroup running this
// gets the same bits.  Split in two so that the loads of the first 256
// partials are in flight while independent work runs.
template <int NV, int NW>
struct PartialRegs {
    static constexpr int VPW = (NV + NW - 1) / NW;  // values per wavefront
    double x[VPW][4];
};

template <int NV, int NW>
__device__ __forceinline__ void load_partials_waves(const RunConst& rc, int st, PartialRegs<NV, NW>& r)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nblk = rc.nblk;
    const double* src = rc.partial + (size_t)(st & 1) * NV * nblk;
#pragma unroll
    for (int i = 0; i < PartialRegs<NV, NW>::VPW; ++i) {
        const int v = wave + i * NW;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int p = lane + 64 * k;
            r.x[i][k] = (v < NV && p < nblk) ? src[(size_t)v * nblk + p] : 0.0;
        }
    }
}

template <int NV, int NW>
__device__ void finish_partials_waves(const RunConst& rc, int st, const PartialRegs<NV, NW>& r, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nblk = rc.nblk;
    const double* src = rc.partial + (size_t)(st & 1) * NV * nblk;
#pragma unroll
    for (int i = 0; i < PartialRegs<NV, NW>::VPW; ++i) {
        const int v = wave + i * NW;
        if (v >= NV) continue;
        // partials 256..511 (launches with more than 256 workgroups): all four
        // loads issued before the first add, then any further ones in turn
        double t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int p = lane + 256 + 64 * k;
            t[k] = p < nblk ? src[(size_t)v * nblk + p] : 0.0;
        }
        double acc = r.x[i][0];
        acc += r.x[i][1];
        acc += r.x[i][2];
        acc += r.x[i][3];
        acc += t[0];
        acc += t[1];
        acc += t[2];
        acc += t[3];
        for (int p = lane + 512; p < nblk; p += 64) acc += src[(size_t)v * nblk + p];
        acc = wave_sum(acc);
        if (lane == 0) out[v] = acc;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ beam kernel
// Launch shape of the beam kernels: one wavefront per trajectory.  FP32
// arithmetic: 16 trajectories per workgroup, three beams of each lane in
// flight, at most 128 VGPRs, so every wavefront of a 4000-trajectory grid is
// resident at once.  FP64 arithmetic: 8 trajectories per workgroup.
template <typename T> struct BeamShape {
    static constexpr bool fp64 = std::is_same<T, double>::value;
    static constexpr int traj = fp64 ? 8 : 16;
    static constexpr int block = 64 * traj;
};

// Beams in flight per lane and the wavefronts per SIMD the register
// allocation must allow, per launch.  FP32 arithmetic: three beams, four
// wavefronts.  FP64 arithmetic needs about twice the registers per beam;
// with two beams in flight the middle launches exceed 128 VGPRs and their
// grid runs in two rounds.  Measured on the 3.2M-beam grid, these launches
// are faster with one beam in flight and four wavefronts per SIMD (the
// compiler spills a few registers of the prologue), the others with two
// beams: stages 2-4 (FP64 storage; also its final launch of a split error)
// and 3-5 (FP32 storage).
template <typename TS, typename T, typename TAB, int I> struct BeamPlan {
    static constexpr bool fp64 = BeamShape<T>::fp64;
    static constexpr bool split_final = TAB::fsal && TAB::embedded && I == TAB::S;
    static constexpr bool narrow =
        fp64 && (std::is_same<TS, double>::value ? ((I >= 2 && I <= 4) || split_final) : (I >= 3 && I <= 5));
    static constexpr int slots = fp64 ? (narrow ? 1 : 2) : 3;
    static constexpr int waves_per_eu = (!fp64 || narrow) ? 4 : 1;
};

// Beam launch I of the attempt (the file header describes the whole step).
// Prologue: J_{I-1} from the previous launch's partials, then stage I-1 of
// this workgroup's trajectories is completed (launch 1 also prepares stage 0
// for the new control block).  Beam loop: k_0..k_{I-1} recomputed from y_n.
// Epilogue: stage I is prepared (phase, rotation factors, geometry) and the
// density sum of the formed state is rotated, weighted and added per
// workgroup.  TS: amplitude type in HBM; T: arithmetic type of the stage
// update (density sums are FP64 in every form).
template <typename TS, typename T, int N, typename TAB, int I, int NJ>
__device__ __forceinline__ void stage_body(const RunConst& rc, const int blk)
{
    constexpr int kTrajPerBlock = BeamShape<T>::traj;
    constexpr int S = TAB::S;
    constexpr bool FINAL = (I == S);
    constexpr int NM = Shape<N>::NM, NU = Shape<N>::NU;
    constexpr int NV = NJ * NM;                          // angle moments J0, J1 (J2, J3)
    constexpr int NF = NJ == 4 ? 4 : 2;                  // epilogue weights per trajectory
    constexpr bool ERROR = FINAL && TAB::embedded;
    constexpr bool FSAL_FINAL = FINAL && TAB::fsal;      // derivatives and error only
    constexpr bool MOMENTS = !FSAL_FINAL;                // density sum of the formed state
    constexpr bool NEWSTATE = TAB::fsal ? (I == S - 1) : FINAL;
    // Embedded pair with first-same-as-last: the launch that forms y_{n+1}
    // also stores sum_{m<S-1} e_m k_m per beam component, and the final launch
    // evaluates only k_{S-1} = f(y_{n+1}) and adds its term.
    constexpr bool SPLIT = TAB::fsal && TAB::embedded;
    constexpr bool ERRSTORE = SPLIT && I == S - 1;
    constexpr bool ERRLAST = SPLIT && FINAL;
    constexpr int NSLOT = BeamPlan<TS, T, TAB, I>::slots;
    constexpr int NK = ERRLAST ? 1 : I;                  // derivatives evaluated per beam
    constexpr uint32_t STRIDE = 64;                      // beam-slot stride of one lane
    using Mat = StageMat<T, N>;

    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int jt = wave;
    const int j = blk * kTrajPerBlock + jt;
    const bool active = j < rc.na;

    __shared__ Mat smat[kTrajPerBlock][NK > 0 ? NK : 1];
    __shared__ double swave[kTrajPerBlock][NV + 1];
    __shared__ double sJ[NV];
    __shared__ double sF[kTrajPerBlock][NF + 2 * (NU > 0 ? NU : 1)];  // weights, z of stage I (-> epilogue)

    // ---- the control block first (the longest dependent chain starts here);
    //      ctrl[1] holds it between attempts, ctrl[0] during one
    // (relaxed atomic loads: issued here rather than sunk to their first use)
    Control C{};
    {
        Control* vc = rc.ctrl + (I <= 1 ? 1 : 0);
        C.r = __hip_atomic_load(&vc->r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        C.h = __hip_atomic_load(&vc->h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        C.istep = __hip_atomic_load(&vc->istep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        C.cur = __hip_atomic_load(&vc->cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        C.status = __hip_atomic_load(&vc->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    // ---- stage matrices of k_0..k_{I-2} (raw dwords, by the trajectory's
    //      wavefront), in flight while the control block arrives; stored to
    //      LDS after the stage completion
    constexpr int MPER = sizeof(Mat) / 4;
    constexpr int NKS = NK > 1 ? NK - 1 : 0;             // stored matrices
    constexpr int MREG = (NKS * MPER + (int)STRIDE - 1) / (int)STRIDE;
    uint32_t mreg[MREG > 0 ? MREG : 1];
    if constexpr (NKS > 0) {
        const uint32_t* msrc = reinterpret_cast<const uint32_t*>(rc.mat);
#pragma unroll
        for (int i = 0; i < MREG; ++i) {
            const int x = lane + i * (int)STRIDE;
            if (active && x < NKS * MPER) {
                const int l = x / MPER, q = x - l * MPER;
                mreg[i] = msrc[((size_t)l * rc.na + j) * MPER + q];
            }
        }
    }

    // ---- prologue inputs that do not depend on the control block (in flight
    //      while it is read): launch I-1's partial density sums, the frame of
    //      stage I-1, and the phase sums of stages I, I+1, ... (lane k: stage
    //      I + k) that the earlier launches of this attempt accumulated
    constexpr int LASTPREP = TAB::fsal ? S - 1 : S;      // last launch that prepares a stage frame
    PartialRegs<NV, kTrajPerBlock> xp;
    if constexpr (I >= 2) load_partials_waves<NV, kTrajPerBlock>(rc, I - 1, xp);
    double cP = 1.0, icP = 1.0, zP[NU > 0 ? NU : 1][2];
    double sP = 0.0, cph = 1.0, sph = 0.0;                 // sin(theta) of stage I-1; azimuth
    double psum[N];
#pragma unroll
    for (int a = 0; a < N; ++a) psum[a] = 0.0;
    if (active) {
        if constexpr (NJ == 4) {
            cph = rc.azi[2 * (size_t)j];
            sph = rc.azi[2 * (size_t)j + 1];
        }
        if constexpr (I >= 2) {
            const TrajGeo& g = rc.geo[(size_t)(I - 1) * rc.na + j];
            cP = g.c;
            icP = g.ic;
            if constexpr (NJ == 4) sP = sqrt((1.0 - g.c) * (1.0 + g.c));
            for (int q = 0; q < NU; ++q) {
                zP[q][0] = g.z[q][0];
                zP[q][1] = g.z[q][1];
            }
            if constexpr (MOMENTS) {
                if (I + lane <= LASTPREP)
                    for (int a = 0; a < N; ++a) psum[a] = rc.geo[(size_t)(I + lane) * rc.na + j].P[a];
            }
        }
    }

    // the first launch of an attempt takes the control block between attempts
    if (I == 1 && blk == 0 && threadIdx.x == 0) rc.ctrl[0] = rc.ctrl[1];
    if (I > 0 && C.status != 0) return;  // run finished: attempts are no-ops
    const int cur = C.cur;
    const double h = C.h;

    // ---- per-beam data
    // slot t < N_E: neutrino of energy bin t; t >= N_E: antineutrino of bin t - N_E
    const uint32_t ne = (uint32_t)rc.ne;
    const uint32_t nbt = active ? 2u * ne : 0u;
    const uint32_t base0 = (uint32_t)j * ne;
    const uint32_t delta = (uint32_t)(rc.na - 1) * ne;
    const TS* src = reinterpret_cast<const TS*>(rc.psi[ERRLAST ? cur ^ 1 : cur]);
    TS* dst = reinterpret_cast<TS*>(rc.psi[cur ^ 1]);
    T* errv = reinterpret_cast<T*>(rc.errv);
    const size_t ld = (size_t)rc.nb_pad;
    global<const T>* __restrict__ uinv = uniform_global(uinv_table<T>(rc));
    global<const double>* __restrict__ wgtp = uniform_global(rc.wgt);
    // per-component bases: state read (y_n, or y_{n+1} for the final launch of
    // a split error), state written, partial error sums
    global<const TS>* __restrict__ srcq[2 * N];
    global<TS>* __restrict__ dstq[2 * N];
    global<T>* __restrict__ errq[2 * N];
#pragma unroll
    for (int q = 0; q < 2 * N; ++q) {
        srcq[q] = uniform_global(src + q * ld);
        dstq[q] = uniform_global(dst + q * ld);
        errq[q] = uniform_global(errv + q * ld);
    }
    const Mat* mats = smat[jt];

    double macc[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) macc[i] = 0.0;
    T emax = 0;
    bool bad = false;

    auto offset = [&](uint32_t t) __attribute__((always_inline)) { return t + base0 + (t >= ne ? delta : 0u); };
    auto fetch = [&](uint32_t t, TS* yv, T* dv, T& uv, double& wv) __attribute__((always_inline)) {
        if (t < nbt) {
            const uint32_t off = offset(t);
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) yv[q] = *elem(srcq[q], off);
            if constexpr (ERRLAST) {
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) dv[q] = *elem(errq[q], off);
            }
            uv = *elem(uinv, t);
            if constexpr (MOMENTS) wv = *elem(wgtp, t);
        }
    };
    auto process = [&](uint32_t t, const TS* yv, const T* dv, T u, double wt) __attribute__((always_inline)) {
        T y[2 * N];
#pragma unroll
        for (int q = 0; q < 2 * N; ++q) y[q] = (T)yv[q];
        if constexpr (ERRLAST) {
            // y = y_{n+1}, dv = sum_{m<S-1} e_m k_m: the error h sum_m e_m k_m
            T k[2 * N];
            eval_ky<T, N>(mats[0].a, mats[0].b, u, y, k);
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) {
                T d = dv[q];
                if constexpr (TAB::E[S - 1] != 0.0) d = fma((T)(ksign(q) * TAB::E[S - 1]), k[q ^ 1], d);
                const T e = fabs(d);
                bad |= !isfinite(e);
                emax = fmax(emax, e);
            }
            return;
        }
        // Compiler-only barrier: re-read the (wave-uniform) stage matrices from
        // LDS for every beam instead of holding all of them in registers.
        asm volatile("" ::: "memory");

        T kk[NK > 0 ? NK : 1][2 * N];
        static_for<0, NK>([&](auto Lc) {
            constexpr int l = decltype(Lc)::value;
            T Y[2 * N];
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) {
                // Y_l = y_n + sum_m a_lm (h k_m), added onto y_n term by term
                T acc = y[q];
                static_for<0, l>([&](auto Mc) {
                    constexpr int m = decltype(Mc)::value;
                    if constexpr (TAB::A[l][m] != 0.0) {
                        constexpr double a_lm = TAB::A[l][m];
                        acc = fma((T)(ksign(q) * a_lm), kk[m][q ^ 1], acc);
                    }
                });
                Y[q] = acc;
            }
            // keep only this stage's matrix live: no LDS reads hoisted across stages
            asm volatile("" ::: "memory");
            eval_ky<T, N>(mats[l].a, mats[l].b, u, Y, kk[l]);
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) pin(kk[l][q]);
        });

        if constexpr (ERRSTORE) {
            // the error terms of k_0..k_{S-2}, summed in the order of the final sum
            const uint32_t off = offset(t);
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) {
                T d = 0;
                bool first = true;
                static_for<0, NK>([&](auto Mc) {
                    constexpr int m = decltype(Mc)::value;
                    if constexpr (TAB::E[m] != 0.0) {
                        d = first ? (T)(ksign(q) * TAB::E[m]) * kk[m][q ^ 1] : fma((T)(ksign(q) * TAB::E[m]), kk[m][q ^ 1], d);
                        first = false;
                    }
                });
                *elem(errq[q], off) = d;
            }
        }

        if constexpr (ERROR && !SPLIT) {
            // h sum_m e_m k_m per real component
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) {
                T d = 0;
                bool first = true;
                static_for<0, S>([&](auto Mc) {
                    constexpr int m = decltype(Mc)::value;
                    if constexpr (TAB::E[m] != 0.0) {
                        d = first ? (T)(ksign(q) * TAB::E[m]) * kk[m][q ^ 1] : fma((T)(ksign(q) * TAB::E[m]), kk[m][q ^ 1], d);
                        first = false;
                    }
                });
                const T e = fabs(d);
                bad |= !isfinite(e);
                emax = fmax(emax, e);
            }
        }

        if constexpr (MOMENTS) {
            // the state this launch forms: Y_I, or y_{n+1} for the last launch of
            // a tableau without first-same-as-last (y_n itself for I == 0)
            T Yo[2 * N];
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) {
                if constexpr (I == 0) {
                    Yo[q] = y[q];
                } else if constexpr (NEWSTATE) {
                    // y_{n+1}: the increment summed first, then added to y_n once
                    T acc = 0;
                    bool first = true;
                    static_for<0, NK>([&](auto Mc) {
                        constexpr int m = decltype(Mc)::value;
                        if constexpr (coef<TAB>(I, m) != 0.0) {
                            constexpr double c_im = coef<TAB>(I, m);
                            acc = first ? (T)(ksign(q) * c_im) * kk[m][q ^ 1] : fma((T)(ksign(q) * c_im), kk[m][q ^ 1], acc);
                            first = false;
                        }
                    });
                    Yo[q] = y[q] + acc;
                } else {
                    // a stage input: the same operations as its recomputation
                    // in the later launches
                    T acc = y[q];
                    static_for<0, NK>([&](auto Mc) {
                        constexpr int m = decltype(Mc)::value;
                        if constexpr (coef<TAB>(I, m) != 0.0) {
                            constexpr double c_im = coef<TAB>(I, m);
                            acc = fma((T)(ksign(q) * c_im), kk[m][q ^ 1], acc);
                        }
                    });
                    Yo[q] = acc;
                }
            }
            if constexpr (NEWSTATE) {
                // FP32 amplitudes are renormalised whenever a new state is
                // formed; the moments are those of the stored values.
                if constexpr (std::is_same<TS, float>::value) {
                    T nn = 0;
#pragma unroll
                    for (int q = 0; q < 2 * N; ++q) nn = fma(Yo[q], Yo[q], nn);
                    const T sc = T(1) / sqrt(nn);
#pragma unroll
                    for (int q = 0; q < 2 * N; ++q) Yo[q] = (T)(TS)(Yo[q] * sc);
                }
                const uint32_t off = offset(t);
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) *elem(dstq[q], off) = (TS)Yo[q];
                if constexpr (!TAB::embedded) {
#pragma unroll
                    for (int q = 0; q < 2 * N; ++q) bad |= !isfinite(Yo[q]);
                }
            }
            // weighted density sum in the rotated frame: wt psi_a conj(psi_b)
            double z[2 * N], wz[2 * N];
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) {
                z[q] = (double)Yo[q];
                wz[q] = wt * z[q];
            }
#pragma unroll
            for (int a = 0; a < N; ++a) macc[a] = fma(wz[2 * a], z[2 * a], fma(wz[2 * a + 1], z[2 * a + 1], macc[a]));
#pragma unroll
            for (int a = 0; a < N; ++a)
#pragma unroll
                for (int b = a + 1; b < N; ++b) {
                    const int q = Shape<N>::up(a, b);
                    macc[N + 2 * q] = fma(wz[2 * a], z[2 * b], fma(wz[2 * a + 1], z[2 * b + 1], macc[N + 2 * q]));
                    macc[N + 2 * q + 1] = fma(wz[2 * a + 1], z[2 * b], fma(-wz[2 * a], z[2 * b + 1], macc[N + 2 * q + 1]));
                }
        }
    };

    // ---- phase of the accepted state and geometry of stage I (wave-uniform)
    double phn[N];
    double cN = 1.0, wN = 0.0;
    if (active) {
        if constexpr (MOMENTS && I > 0) {
            for (int a = 0; a < N; ++a) phn[a] = rc.phase[cur][(size_t)j * N + a];
            traj_geometry(rc, j, stage_radius<TAB>(rc, C, I), cN, wN);
        }
    }

    // ---- the first beam of every slot: in flight from here on (no stage
    //      frame to prepare), else (register pressure) from the end of the
    //      stage completion on, overlapping the frame preparation
    constexpr bool EARLY_FETCH = !(MOMENTS && I > 0);
    TS ys[NSLOT][2 * N];
    T ds[NSLOT][ERRLAST ? 2 * N : 1];
    T us[NSLOT];
    double ws[NSLOT];
    const uint32_t t0 = (uint32_t)lane;
    auto fetch_first = [&]() __attribute__((always_inline)) {
        static_for<0, NSLOT>([&](auto Sc) {
            constexpr int sl = decltype(Sc)::value;
            us[sl] = 0;
            ws[sl] = 0.0;
            fetch(t0 + sl * STRIDE, ys[sl], ds[sl], us[sl], ws[sl]);
        });
    };
    if constexpr (EARLY_FETCH) fetch_first();


    // ---- J_{I-1}: the previous launch's partials (launch 1: J_0 of the state)
    if constexpr (NK > 0) {
        if constexpr (I == 1) {
            if ((int)threadIdx.x < NV) sJ[threadIdx.x] = rc.jhist[threadIdx.x];
            __syncthreads();
        } else {
            finish_partials_waves<NV, kTrajPerBlock>(rc, I - 1, xp, sJ);
            if (blk == 0 && (int)threadIdx.x < NV) rc.jhist[(size_t)(I - 1) * NV + threadIdx.x] = sJ[threadIdx.x];
        }
        // stored matrices -> LDS; stage I-1 completed for this trajectory
        uint32_t* mdst = reinterpret_cast<uint32_t*>(&smat[jt][0]);
#pragma unroll
        for (int i = 0; i < MREG; ++i) {
            const int x = lane + i * (int)STRIDE;
            if (active && x < NKS * MPER) mdst[x] = mreg[i];
        }
        if (active) {
            double J[NV];
            for (int v = 0; v < NV; ++v) J[v] = sJ[v];
            if constexpr (I == 1) {
                double c0, w0;
                traj_geometry(rc, j, stage_radius<TAB>(rc, C, 0), c0, w0);
                const Frame<N> f0 = prepare_wave<N>(rc, j, 0, c0, w0, phn, lane);
                cP = f0.c;
                icP = f0.ic;
                sP = f0.s;
                for (int q = 0; q < NU; ++q) {
                    zP[q][0] = f0.z[q][0];
                    zP[q][1] = f0.z[q][1];
                }
            }
            double GP[N];
            complete_wave<T, N, NJ>(rc, j, I - 1, cP, icP, sP * cph, sP * sph, zP,
                                    matter(rc, stage_radius<TAB>(rc, C, I - 1)), J, h, GP, &smat[jt][NK - 1], lane);
            if constexpr (!EARLY_FETCH) fetch_first();
            if constexpr (MOMENTS) {
                // phase sums sum_{m < l} coef(l, m) G_m: lane k adds the term of
                // G_{I-1} to that of stage l = I + k and passes it on to launch l
                const int l = I + lane;
                const double cf = coef_of_column<TAB, I - 1, LASTPREP>(l);
                if (cf != 0.0)
                    for (int a = 0; a < N; ++a) psum[a] += cf * GP[a];
                if (lane >= 1 && l <= LASTPREP)
                    for (int a = 0; a < N; ++a) rc.geo[(size_t)l * rc.na + j].P[a] = psum[a];
                // stage I prepared now, its frame kept for the epilogue: phase
                // Phi_n + h sum_{m < I} coef(I, m) G_m, rotation factors, geometry
                double ph[N];
                for (int a = 0; a < N; ++a) ph[a] = phn[a] + h * __shfl(psum[a], 0, 64);
                const Frame<N> f = prepare_wave<N>(rc, j, I, cN, wN, ph, lane);
                if (I == LASTPREP)  // the new state's phase; kept only if the attempt is accepted
                    lane_scatter(rc.phase[cur ^ 1] + (size_t)j * N, ph, lane);
                double fw[NF + 2 * (NU > 0 ? NU : 1)];
                fw[0] = f.w;
                fw[1] = f.wc;
                if constexpr (NJ == 4) {
                    fw[2] = (f.w * f.s) * cph;
                    fw[3] = (f.w * f.s) * sph;
                }
                for (int q = 0; q < NU; ++q) {
                    fw[NF + 2 * q] = f.z[q][0];
                    fw[NF + 1 + 2 * q] = f.z[q][1];
                }
                lane_scatter(sF[jt], fw, lane);
            }
        }
        // the stage matrices in LDS are this wavefront's own: a wavefront-level
        // barrier orders its LDS writes before the beam loop reads them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // ---- beam loop: NSLOT-slot load pipeline, the next beams of the other
    //      slots in flight while one is computed (unrolled by NSLOT, no copies)
#pragma unroll 1
    for (uint32_t t = t0; t < nbt; t += NSLOT * STRIDE) {
        static_for<0, NSLOT>([&](auto Sc) {
            constexpr int sl = decltype(Sc)::value;
            const uint32_t ts = t + sl * STRIDE;
            if (sl == 0 || ts < nbt) process(ts, ys[sl], ds[sl], us[sl], ws[sl]);
            fetch(ts + NSLOT * STRIDE, ys[sl], ds[sl], us[sl], ws[sl]);
        });
    }

    // ---- epilogue: stage I prepared, density sum rotated and weighted
    if constexpr (MOMENTS) {
#pragma unroll
        for (int i = 0; i < NM; ++i) macc[i] = wave_sum(macc[i]);
        double sl[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) sl[v] = 0.0;
        if (active) {
            Frame<N> f;
            double wsc = 0.0, wss = 0.0;  // w sin(theta) cos(phi), w sin(theta) sin(phi)
            if constexpr (I == 0) {
                // stage-0 frame prepared before this launch
                const TrajGeo& g = rc.geo[j];
                f.c = g.c;
                f.w = g.w;
                f.wc = g.wc;
                f.ic = g.ic;
                if constexpr (NJ == 4) {
                    const double s0 = sqrt((1.0 - g.c) * (1.0 + g.c));
                    wsc = (g.w * s0) * cph;
                    wss = (g.w * s0) * sph;
                }
                for (int q = 0; q < NU; ++q) {
                    f.z[q][0] = g.z[q][0];
                    f.z[q][1] = g.z[q][1];
                }
            } else {
                // frame of stage I prepared in the prologue
                f.w = sF[jt][0];
                f.wc = sF[jt][1];
                if constexpr (NJ == 4) {
                    wsc = sF[jt][2];
                    wss = sF[jt][3];
                }
                for (int q = 0; q < NU; ++q) {
                    f.z[q][0] = sF[jt][NF + 2 * q];
                    f.z[q][1] = sF[jt][NF + 1 + 2 * q];
                }
            }
            // S_ab = 2 e^{-i(Phi_a - Phi_b)} S~_ab ; S_aa = 2 S~_aa, weighted by w and w c
            double Sv[NM];
            for (int a = 0; a < N; ++a) Sv[a] = 2.0 * macc[a];
            for (int q = 0; q < NU; ++q) {
                const double cs = f.z[q][0], sn = f.z[q][1];
                const double xr = macc[N + 2 * q], xi = macc[N + 2 * q + 1];
                Sv[N + 2 * q] = 2.0 * (cs * xr + sn * xi);
                Sv[N + 2 * q + 1] = 2.0 * (cs * xi - sn * xr);
            }
            for (int v = 0; v < NM; ++v) {
                sl[v] = f.w * Sv[v];
                sl[NM + v] = f.wc * Sv[v];
                if constexpr (NJ == 4) {
                    sl[2 * NM + v] = wsc * Sv[v];
                    sl[3 * NM + v] = wss * Sv[v];
                }
            }
        }
        if (lane == 0)
            for (int v = 0; v < NV; ++v) swave[jt][v] = sl[v];
    }
    if constexpr (FINAL) {
        double e = bad ? (double)INFINITY : (double)emax;
        e = wave_max(e);
        if (lane == 0) swave[jt][NV] = active ? e : 0.0;
    }
    __syncthreads();
    if constexpr (MOMENTS) {
        if ((int)threadIdx.x < NV) {
            const int v = threadIdx.x;
            double acc = swave[0][v];
            for (int w = 1; w < kTrajPerBlock; ++w) acc += swave[w][v];
            rc.partial[((size_t)(I & 1) * NV + v) * rc.nblk + blk] = acc;
        }
    }
    if constexpr (FINAL) {
        if (threadIdx.x == 0) {
            double e = swave[0][NV];
            for (int w = 1; w < kTrajPerBlock; ++w) e = fmax(e, swave[w][NV]);
            rc.errpart[blk] = e;
        }
    }
}

// Beam launch over a launch set (any number of runs) and over one run whose
// constants travel as the kernel argument (no table lookup before the first
// loads).
template <typename TS, typename T, int N, typename TAB, int I, int NJ>
__global__ void __launch_bounds__(BeamShape<T>::block)
__attribute__((amdgpu_waves_per_eu(BeamPlan<TS, T, TAB, I>::waves_per_eu))) k_stage(const LaunchSet ls)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    stage_body<TS, T, N, TAB, I, NJ>(rc, blk);
}

template <typename TS, typename T, int N, typename TAB, int I, int NJ>
__global__ void __launch_bounds__(BeamShape<T>::block)
__attribute__((amdgpu_waves_per_eu(BeamPlan<TS, T, TAB, I>::waves_per_eu))) k_stage_one(const RunConst rc)
{
    stage_body<TS, T, N, TAB, I, NJ>(rc, blockIdx.x);
}

// After the last beam launch of an attempt, one workgroup per run: the global
// step-error maximum (order-independent), the controller, and J_0 of the next
// attempt (J of the accepted state, else unchanged).  For a tableau without
// first-same-as-last, J of the new state is summed from the last launch's
// partials here.  Also used after a stage-0 launch (I == 0) to sum J_0.
template <int N, typename TAB, int I, int NJ>
__device__ __forceinline__ void control_body(const RunConst& rc)
{
    constexpr int S = TAB::S;
    constexpr int NV = NJ * Shape<N>::NM;
    constexpr bool SUM = (I == 0) || !TAB::fsal;
    __shared__ double sred[NV][kFinBlock / NV];
    __shared__ double sJ[NV];
    __shared__ double serr[kFinBlock / 64];
    if constexpr (I == 0) {
        reduce_partials<NV, kFinBlock>(rc, 0, sJ, sred);
        if ((int)threadIdx.x < NV) rc.jhist[threadIdx.x] = sJ[threadIdx.x];
        return;
    } else {
        const Control* ctl = rc.ctrl;
        if (ctl->status != 0) return;
        if constexpr (SUM) reduce_partials<NV, kFinBlock>(rc, S, sJ, sred);
        double m = 0.0;
        for (int p = threadIdx.x; p < rc.nblk; p += kFinBlock) m = fmax(m, rc.errpart[p]);
        m = wave_max(m);
        if ((threadIdx.x & 63) == 0) serr[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < kFinBlock / 64; ++w) m = fmax(m, serr[w]);
            Control c = *ctl;
            const bool acc = control_step<TAB>(rc, c, m);
            if (acc)
                for (int v = 0; v < NV; ++v)
                    rc.jhist[v] = TAB::fsal ? rc.jhist[(size_t)(S - 1) * NV + v] : sJ[v];
            rc.ctrl[1] = c;
        }
    }
}

template <int N, typename TAB, int I, int NJ>
__global__ void __launch_bounds__(kFinBlock) k_control(const LaunchSet ls)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    control_body<N, TAB, I, NJ>(rc);
}

template <int N, typename TAB, int I, int NJ>
__global__ void __launch_bounds__(kFinBlock) k_control_one(const RunConst rc)
{
    control_body<N, TAB, I, NJ>(rc);
}

// Stage-0 frame of the current state (before a stage-0 launch).
template <int N, typename TAB>
__global__ void __launch_bounds__(kFinBlock) k_prepare(const LaunchSet ls)
{
    int blk;
    const RunConst& rc = ls.runs[run_of_block(ls, blk)];
    const int j = blk * kFinBlock + threadIdx.x;
    if (j >= rc.na) return;
    const Control C = rc.ctrl[1];
    double ph[N];
    for (int a = 0; a < N; ++a) ph[a] = rc.phase[C.cur][(size_t)j * N + a];
    prepare_thread<N>(rc, j, 0, stage_radius<TAB>(rc, C, 0), ph);
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

template <typename TS, typename T, int N, typename TAB, int NJ>
struct StageTable {
    template <int... Is>
    static constexpr std::array<KernFn, kMaxStages> make(std::integer_sequence<int, Is...>)
    {
        return {{(Is <= TAB::S ? (KernFn)&k_stage<TS, T, N, TAB, (Is <= TAB::S ? Is : 0), NJ> : nullptr)...}};
    }
    static constexpr std::array<KernFn, kMaxStages> fns = make(std::make_integer_sequence<int, kMaxStages>{});
};

using OneFn = void (*)(const RunConst);

template <typename TS, typename T, int N, typename TAB, int NJ>
struct StageOneTable {
    template <int... Is>
    static constexpr std::array<OneFn, kMaxStages> make(std::integer_sequence<int, Is...>)
    {
        return {{(Is <= TAB::S ? (OneFn)&k_stage_one<TS, T, N, TAB, (Is <= TAB::S ? Is : 0), NJ> : nullptr)...}};
    }
    static constexpr std::array<OneFn, kMaxStages> fns = make(std::make_integer_sequence<int, kMaxStages>{});
};

// The kernels of beam launch `stage`: over launch sets (k, f) and over one
// run (k1, f1); f, f1: the control kernel that follows stage 0 and the last
// stage, else nullptr.
struct StageKernels {
    KernFn k = nullptr, f = nullptr;
    OneFn k1 = nullptr, f1 = nullptr;
};

template <typename TS, typename T, int N, typename TAB, int NJ>
void pick_tab(int stage, StageKernels& K)
{
    K.k = StageTable<TS, T, N, TAB, NJ>::fns[stage];
    K.k1 = StageOneTable<TS, T, N, TAB, NJ>::fns[stage];
    if (stage == 0) {
        K.f = (KernFn)&k_control<N, TAB, 0, NJ>;
        K.f1 = (OneFn)&k_control_one<N, TAB, 0, NJ>;
    } else if (stage == TAB::S) {
        K.f = (KernFn)&k_control<N, TAB, TAB::S, NJ>;
        K.f1 = (OneFn)&k_control_one<N, TAB, TAB::S, NJ>;
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

long long fin_blocks(const RunConst& rc) { return (rc.na + kFinBlock - 1) / kFinBlock; }

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

int num_stages(int integrator) { return integrator == 0 ? TabRK4::S : TabDP54::S; }

hipError_t launch_stage(const RunList& runs, int stage, hipStream_t s, hipEvent_t* ev)
{
    if (runs.count < 1) return hipSuccess;
    if (!same_kind(runs)) return hipErrorInvalidValue;
    const RunConst& r0 = *runs.rc[0];
    if (stage < 0 || stage > num_stages(r0.integrator)) return hipErrorInvalidValue;
    StageKernels K;
    const unsigned block = r0.precision == 1 ? BeamShape<float>::block : BeamShape<double>::block;
    if ((r0.precision == 1 ? BeamShape<float>::traj : BeamShape<double>::traj) != traj_per_block(r0.precision))
        return hipErrorInvalidValue;
    switch (r0.precision) {
    case 0: pick_nj<double, double>(r0.nj, r0.n, r0.integrator, stage, K); break;  // FP64
    case 1: pick_nj<float, float>(r0.nj, r0.n, r0.integrator, stage, K); break;    // FP32 amplitudes
    case 2: pick_nj<float, double>(r0.nj, r0.n, r0.integrator, stage, K); break;   // FP32 amplitudes, FP64 math
    default: break;
    }
    if (!K.k || !K.k1) return hipErrorInvalidValue;
    const bool one = runs.count == 1;
    if (ev) {
        hipError_t e = hipEventRecord(ev[0], s);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipSuccess;
    if (one) {
        hipLaunchKernelGGL(K.k1, dim3((unsigned)r0.nblk), dim3(block), 0, s, r0);
        e = hipGetLastError();
    } else {
        e = for_launch_sets(runs, [](const RunConst& rc) { return (long long)rc.nblk; },
                            [&](const LaunchSet& ls, unsigned grid) {
                                hipLaunchKernelGGL(K.k, dim3(grid), dim3(block), 0, s, ls);
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

hipError_t launch_prepare(const RunList& runs, hipStream_t s)
{
    if (runs.count < 1) return hipSuccess;
    if (!same_kind(runs)) return hipErrorInvalidValue;
    const RunConst& r0 = *runs.rc[0];
    KernFn k;
    if (r0.n == 2) k = r0.integrator == 0 ? (KernFn)&k_prepare<2, TabRK4> : (KernFn)&k_prepare<2, TabDP54>;
    else k = r0.integrator == 0 ? (KernFn)&k_prepare<3, TabRK4> : (KernFn)&k_prepare<3, TabDP54>;
    return for_launch_sets(runs, fin_blocks, [&](const LaunchSet& ls, unsigned grid) {
        hipLaunchKernelGGL(k, dim3(grid), dim3(kFinBlock), 0, s, ls);
        return hipGetLastError();
    });
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

}  // namespace nuosc
