// gfx950 kernels of the bulb-model flavor evolution.
//
// One step attempt of an explicit Runge-Kutta tableau with S stages runs as S
// launches of k_stage<..., I> for I = 1..S.  Launch I:
//   * per trajectory j (one workgroup): rebuilds, in FP64, the per-trajectory
//     Hamiltonian pieces of stages 0..I-1 from the broadcast moments J_0..J_{I-1}
//     (geometry eq 3.14-3.15, matter eq 3.7, self-interaction eq 3.13/3.16,
//     co-rotating phases) and stores them in LDS as K~ = A + B / E;
//   * per beam (one lane): reads y_n once, recomputes k_0..k_{I-1}, forms the
//     stage state Y_I (or the new state for I = S) and accumulates its
//     contribution to the per-trajectory density sum in FP64;
//   * the workgroup reduces its sum (wave shuffles, then LDS, fixed order),
//     rotates it to the lab frame, weights it by w_j and w_j c_j and writes
//     it; the last workgroup to finish adds all trajectories in a fixed order
//     into J_I (deterministic), or for I = S reduces the step error and runs
//     the step controller.
// Only y_n is read from HBM per launch and only y_{n+1} is written (in the
// final launch): every stage derivative is recomputed from y_n and the small
// J history instead of being stored.
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

// ------------------------------------------------------------------ helpers
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
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

template <int N> struct Shape {
    static constexpr int NU = N * (N - 1) / 2;  // upper off-diagonal entries
    static constexpr int NM = N * N;            // reals of a packed Hermitian matrix
    __host__ __device__ static constexpr int up(int a, int b) { return a * N - a * (a + 1) / 2 + (b - a - 1); }
};

// K~ = A + B / E of one species on one trajectory at one stage.
template <typename T, int N> struct SpeciesMat {
    T ad[N], bd[N];
    T au[Shape<N>::NU][2], bu[Shape<N>::NU][2];
};
template <typename T, int N> struct StageMat { SpeciesMat<T, N> sp[2]; };

// k = -i K~ y for one beam.  y, k: [2N] as (re, im) per component.
template <typename T, int N>
__device__ __forceinline__ void eval_k(const SpeciesMat<T, N>& M, T inv_e, const T* y, T* k)
{
    constexpr int NU = Shape<N>::NU;
    T kd[N], ku[NU][2];
#pragma unroll
    for (int a = 0; a < N; ++a) kd[a] = fma(M.bd[a], inv_e, M.ad[a]);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        ku[u][0] = fma(M.bu[u][0], inv_e, M.au[u][0]);
        ku[u][1] = fma(M.bu[u][1], inv_e, M.au[u][1]);
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
        k[2 * a] = q;       // -i (p + i q) = q - i p
        k[2 * a + 1] = -p;
    }
}

// Geometry of trajectory j at radius r (eq 3.14-3.15; single angle: c = 1,
// w = D(r/R) of eq 3.17).
__device__ __forceinline__ void traj_geometry(const RunConst& rc, int j, double r, double& c, double& w)
{
    // 1 - (R/r)^2 as (r - R)(r + R) / r^2: exact subtraction near the
    // neutrinosphere, where 1 - (R/r)^2 (1 - u^2) would cancel for small u.
    const double x = (rc.r_nu / r) * (rc.r_nu / r);
    const double y = (r - rc.r_nu) * (r + rc.r_nu) / (r * r);
    if (rc.ma) {
        const double du = 1.0 / (double)rc.na;
        const double u = ((double)j + 0.5) * du;
        c = sqrt(fma(1.0 - u * u, y, u * u));
        w = x * u * du / c;
    } else {
        c = 1.0;
        const double s = 1.0 - sqrt(y);
        w = 0.5 * s * s;
    }
}

__device__ __forceinline__ double matter(const RunConst& rc, double r)
{
    return rc.lambda0 * pow(rc.lambda_rref / r, rc.lambda_power);
}

// mu0 * traceless(J0 - c J1) from packed moments J (J0 then J1).
template <int N>
__device__ __forceinline__ void collective(const RunConst& rc, const double* J, double c, double* Cd, double (*Cu)[2])
{
    constexpr int NM = Shape<N>::NM, NU = Shape<N>::NU;
    double tr = 0.0;
    for (int a = 0; a < N; ++a) {
        Cd[a] = J[a] - c * J[NM + a];
        tr += Cd[a];
    }
    for (int a = 0; a < N; ++a) Cd[a] = rc.mu0 * (Cd[a] - tr / N);
    for (int u = 0; u < NU; ++u) {
        Cu[u][0] = rc.mu0 * (J[N + 2 * u] - c * J[NM + N + 2 * u]);
        Cu[u][1] = rc.mu0 * (J[N + 2 * u + 1] - c * J[NM + N + 2 * u + 1]);
    }
}

template <typename T> __device__ __forceinline__ T* psi_ptr(const RunConst& rc, int buf)
{
    return reinterpret_cast<T*>(rc.psi[buf]);
}

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

// Sum NV doubles over a workgroup of NW waves in a fixed order (butterfly in
// each wave, then waves in index order); result valid in thread 0.
template <int NV, int NW>
__device__ __forceinline__ void block_sum(double* v, double (*lds)[NW])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
        for (int i = 0; i < NV; ++i) lds[i][wave] = v[i];
    __syncthreads();
    // value i is combined by thread i (waves in index order), then gathered
    if ((int)threadIdx.x < NV) {
        const int i = threadIdx.x;
        double s = lds[i][0];
        for (int w = 1; w < NW; ++w) s += lds[i][w];
        lds[i][0] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < NV; ++i) v[i] = lds[i][0];
}

// Trajectories (wavefronts) per stage workgroup: their weighted sums are added
// in wave order into one partial, so the finalise launch reads na / 4 partials.
constexpr int kTrajPerBlock = 4;

// Radius of stage l of the current attempt (l == S: the new state).
template <typename TAB>
__device__ __forceinline__ double stage_radius(const RunConst& rc, const Control* ctl, double r, double h, int l)
{
    if (l < TAB::S) return r + TAB::C[l] * h;
    return (rc.integrator == 0) ? rc.r_start + (double)(ctl->istep + 1) * rc.h_fixed : r + h;
}

// ------------------------------------------------------------------ stage kernel
// One wavefront per trajectory j.  TS: amplitude type in HBM; T: arithmetic
// type of the stage update.  Launch I (1 <= I <= S) needs the Hamiltonian
// pieces of stages 0..I-1: those of stages < I-1 were built by earlier
// launches of this attempt and are read from rc.tab; stage I-1 is completed
// here from J_{I-1} (its geometry and phase were set by launch I-1); the
// output stage I gets its geometry and phase here.
template <typename TS, typename T, int N, bool MA, typename TAB, int I>
__global__ void __launch_bounds__(64 * kTrajPerBlock) k_stage(const RunConst rc)
{
    constexpr int S = TAB::S;
    constexpr bool FINAL = (I == S);
    constexpr int NU = Shape<N>::NU, NM = Shape<N>::NM;
    constexpr bool MOMENTS = !FINAL || !TAB::fsal;  // the last RK4 launch also forms J of y_{n+1}

    const Control* ctl = rc.ctrl;
    if (I > 0 && ctl->status != 0) return;  // run finished: attempts are no-ops
    const int cur = ctl->cur;
    const double r = ctl->r, h = ctl->h;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * kTrajPerBlock + wave;
    const bool active = j < rc.na;

    __shared__ StageMat<T, N> smat_all[kTrajPerBlock][I > 0 ? I : 1];
    __shared__ double sG_all[kTrajPerBlock][kMaxStages][N];
    __shared__ double spart[kTrajPerBlock][2 * NM + 1];
    StageMat<T, N>* smat = smat_all[wave];

    // ---- amplitudes stream through a two-deep register pipeline: the loads of
    //      the next two beams of this lane are in flight while one is computed
    //      (the first two are issued before the prologue).
    const TS* __restrict__ src = psi_ptr<TS>(rc, cur);
    TS* __restrict__ dst = psi_ptr<TS>(rc, cur ^ 1);
    const int64_t ld = rc.nb_pad;
    const int nbt = active ? 2 * rc.ne : 0;  // beams of this trajectory
    auto beam_index = [&](int t) {
        const int s = (t >= rc.ne) ? 1 : 0;
        return ((int64_t)s * rc.na + j) * rc.ne + (t - s * rc.ne);
    };
    auto fetch = [&](int t, TS* v) {
        if (t < nbt) {
            const int64_t b = beam_index(t);
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) v[q] = src[q * ld + b];
        }
    };
    TS ynext0[2 * N], ynext1[2 * N];
    fetch(lane, ynext0);
    fetch(lane + 64, ynext1);

    // ---- stored Hamiltonian pieces of stages 0..I-2 -> LDS (both species)
    if constexpr (I >= 2) {
        if (active) {
            constexpr int PER = 2 * NM;  // A then B, packed
            for (int idx = lane; idx < (I - 1) * PER; idx += 64) {
                const int l = idx / PER, q = idx - l * PER;
                const TrajStage& e = rc.tab[(size_t)l * rc.na + j];
                const int m = q < NM ? 0 : 1;       // 0: A, 1: B
                const int x = q - m * NM;
                const double v = m == 0 ? e.A[x] : e.B[x];
                SpeciesMat<T, N>& nu = smat[l].sp[0];
                SpeciesMat<T, N>& nb = smat[l].sp[1];
                if (x < N) {
                    if (m == 0) { nu.ad[x] = (T)v; nb.ad[x] = (T)(-v); }
                    else { nu.bd[x] = (T)v; nb.bd[x] = (T)v; }
                } else {
                    const int u = (x - N) >> 1, ri = (x - N) & 1;
                    // nubar: A -> -conj(A), B -> conj(B)
                    if (m == 0) { nu.au[u][ri] = (T)v; nb.au[u][ri] = (T)(ri ? v : -v); }
                    else { nu.bu[u][ri] = (T)v; nb.bu[u][ri] = (T)(ri ? -v : v); }
                }
            }
        }
    }

    // ---- lane 0: complete stage I-1, then geometry and phase of stage I (FP64)
    double zo[NU > 0 ? NU : 1][2], co = 1.0, wo = 0.0, pho[N];
    if (active && lane == 0) {
        const double* ph0 = rc.phase[cur] + (size_t)j * N;
        double (*G)[N] = sG_all[wave];
        for (int l = 0; l + 1 < I; ++l)
            for (int a = 0; a < N; ++a) G[l][a] = rc.tab[(size_t)l * rc.na + j].G[a];
        if constexpr (I >= 1) {
            constexpr int l = I - 1;
            TrajStage& e = rc.tab[(size_t)l * rc.na + j];
            const double rl = stage_radius<TAB>(rc, ctl, r, h, l);
            double c, w, phl[N], zl[NU > 0 ? NU : 1][2];
            if (l == 0) {
                traj_geometry(rc, j, rl, c, w);
                for (int a = 0; a < N; ++a) phl[a] = ph0[a];
                for (int a = 0; a < N; ++a)
                    for (int b = a + 1; b < N; ++b) {
                        const int u = Shape<N>::up(a, b);
                        sincos(phl[a] - phl[b], &zl[u][1], &zl[u][0]);
                    }
                e.c = c; e.w = w;
                for (int a = 0; a < N; ++a) e.phi[a] = phl[a];
                for (int u = 0; u < NU; ++u) { e.z[u][0] = zl[u][0]; e.z[u][1] = zl[u][1]; }
            } else {
                c = e.c;
                for (int u = 0; u < NU; ++u) { zl[u][0] = e.z[u][0]; zl[u][1] = e.z[u][1]; }
            }
            // Hamiltonian pieces of stage l in the co-rotating frame:
            //   A_ab = e^{i(Phi_a-Phi_b)} C_ab / c,  B_ab = e^{i(Phi_a-Phi_b)} V_ab / c   (a < b)
            //   A_aa = 0 (co-rotating) or (H_m + C)_aa / c (lab),  B_aa = V_aa / c
            double Cd[N], Cu[NU > 0 ? NU : 1][2];
            collective<N>(rc, rc.jhist + l * 2 * NM, c, Cd, Cu);
            const double lam = matter(rc, rl);
            const double ic = 1.0 / c;
            SpeciesMat<T, N>& nu = smat[l].sp[0];
            SpeciesMat<T, N>& nb = smat[l].sp[1];
            for (int a = 0; a < N; ++a) {
                const double hd = lam * ((a == 0 ? 1.0 : 0.0) - 1.0 / N) + Cd[a];
                const double gd = (rc.frame == 0) ? hd * ic : 0.0;
                G[l][a] = gd;
                e.G[a] = gd;
                const double ad = (rc.frame == 0) ? 0.0 : hd * ic;
                const double bd = rc.vac[a][a][0] * ic;
                e.A[a] = ad;
                e.B[a] = bd;
                nu.ad[a] = (T)ad; nb.ad[a] = (T)(-ad);
                nu.bd[a] = (T)bd; nb.bd[a] = (T)bd;
            }
            for (int u = 0; u < NU; ++u) {
                const double cs = zl[u][0], sn = zl[u][1];
                int a = 0, b = 1;
                for (int aa = 0; aa < N; ++aa)
                    for (int bb = aa + 1; bb < N; ++bb)
                        if (Shape<N>::up(aa, bb) == u) { a = aa; b = bb; }
                const double cr = Cu[u][0] * ic, ci = Cu[u][1] * ic;
                const double vr = rc.vac[a][b][0] * ic, vi = rc.vac[a][b][1] * ic;
                const double Ar = cs * cr - sn * ci, Ai = cs * ci + sn * cr;
                const double Br = cs * vr - sn * vi, Bi = cs * vi + sn * vr;
                e.A[N + 2 * u] = Ar; e.A[N + 2 * u + 1] = Ai;
                e.B[N + 2 * u] = Br; e.B[N + 2 * u + 1] = Bi;
                nu.au[u][0] = (T)Ar;  nu.au[u][1] = (T)Ai;
                nu.bu[u][0] = (T)Br;  nu.bu[u][1] = (T)Bi;
                nb.au[u][0] = (T)(-Ar); nb.au[u][1] = (T)Ai;
                nb.bu[u][0] = (T)Br;  nb.bu[u][1] = (T)(-Bi);
            }
        }
        // output stage (or new state): radius, geometry, phase, rotation
        const double ro = stage_radius<TAB>(rc, ctl, r, h, I);
        traj_geometry(rc, j, ro, co, wo);
        for (int a = 0; a < N; ++a) {
            double acc = 0.0;
            static_for<0, I>([&](auto Mc) {
                constexpr int m = decltype(Mc)::value;
                constexpr double coef = FINAL ? TAB::B[m] : TAB::A[I < S ? I : 0][m];
                if constexpr (coef != 0.0) acc += coef * G[m][a];
            });
            pho[a] = ph0[a] + h * acc;
        }
        for (int a = 0; a < N; ++a)
            for (int b = a + 1; b < N; ++b) {
                const int u = Shape<N>::up(a, b);
                sincos(pho[a] - pho[b], &zo[u][1], &zo[u][0]);
            }
        if constexpr (!FINAL && I >= 1) {
            TrajStage& e = rc.tab[(size_t)I * rc.na + j];
            e.c = co; e.w = wo;
            for (int a = 0; a < N; ++a) e.phi[a] = pho[a];
            for (int u = 0; u < NU; ++u) { e.z[u][0] = zo[u][0]; e.z[u][1] = zo[u][1]; }
        }
        if constexpr (FINAL) {
            double* ph1 = rc.phase[cur ^ 1] + (size_t)j * N;  // kept only if the attempt is accepted
            for (int a = 0; a < N; ++a) ph1[a] = pho[a];
        }
    }
    __syncthreads();

    // ---- per-beam work: lanes over the 2*NE beams of trajectory j
    // Stage states are y + h * (sum_m a_lm k_m): the tableau coefficients are
    // compile-time constants (scalar operands), only h is a runtime value.
    const T hT = (T)h;

    double macc[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) macc[i] = 0.0;
    double emax = 0.0;

#pragma unroll 1
    for (int t = lane; t < nbt; t += 64) {
        const int s = (t >= rc.ne) ? 1 : 0;
        const int k = t - s * rc.ne;
        const int64_t b = beam_index(t);
        T y[2 * N];
#pragma unroll
        for (int q = 0; q < 2 * N; ++q) {
            y[q] = (T)ynext0[q];
            ynext0[q] = ynext1[q];
        }
        fetch(t + 128, ynext1);
        // Compiler-only barrier: re-read the (wave-uniform) stage matrices from
        // LDS each iteration instead of keeping both species' copies in VGPRs.
        asm volatile("" ::: "memory");
        const T inv_e = (T)rc.inv_e[k];

        T kk[I > 0 ? I : 1][2 * N];
        static_for<0, I>([&](auto Lc) {
            constexpr int l = decltype(Lc)::value;
            T Y[2 * N];
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) {
                T acc = 0;
                static_for<0, l>([&](auto Mc) {
                    constexpr int m = decltype(Mc)::value;
                    if constexpr (TAB::A[l][m] != 0.0) acc = fma((T)TAB::A[l][m], kk[m][q], acc);
                });
                Y[q] = (l == 0) ? y[q] : fma(hT, acc, y[q]);
            }
            // keep only this stage's matrix live: no LDS reads hoisted across stages
            asm volatile("" ::: "memory");
            eval_k<T, N>(smat[l].sp[s], inv_e, Y, kk[l]);
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) pin(kk[l][q]);
        });

        // output state: Y_I (stage) or y_{n+1} (final)
        T Y[2 * N];
#pragma unroll
        for (int q = 0; q < 2 * N; ++q) {
            T acc = 0;
            static_for<0, I>([&](auto Mc) {
                constexpr int m = decltype(Mc)::value;
                constexpr double coef = FINAL ? TAB::B[m] : TAB::A[I < S ? I : 0][m];
                if constexpr (coef != 0.0) acc = fma((T)coef, kk[m][q], acc);
            });
            Y[q] = (I == 0) ? y[q] : fma(hT, acc, y[q]);
        }
        // FP32 amplitudes are renormalised whenever a new state is formed, and
        // the moments of the new state are those of its stored FP32 values.
        if constexpr (std::is_same<TS, float>::value && (FINAL || (TAB::fsal && I == S - 1))) {
            T nn = 0;
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) nn = fma(Y[q], Y[q], nn);
            const T sc = T(1) / sqrt(nn);
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) Y[q] = (T)(TS)(Y[q] * sc);
        }
        if constexpr (FINAL) {
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) dst[q * ld + b] = (TS)Y[q];
            bool bad = false;
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) bad |= !isfinite((double)Y[q]);
            if constexpr (TAB::embedded) {
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) {
                    double d = 0.0;
                    static_for<0, S>([&](auto Mc) {
                        constexpr int m = decltype(Mc)::value;
                        if constexpr (TAB::E[m] != 0.0) d = fma(TAB::E[m], (double)kk[m][q], d);
                    });
                    d = fabs(h * d);
                    bad |= !isfinite(d);
                    emax = fmax(emax, d);
                }
            }
            if (bad) emax = INFINITY;
        }
        if constexpr (MOMENTS) {
            // rotated-frame density sum: nu: +g psi_a conj(psi_b); nubar: -gbar conj(psi_a conj(psi_b))
            const double wt = s ? -rc.gbar[k] : rc.g[k];
            const double sg = s ? -1.0 : 1.0;
            double z[2 * N];
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) z[q] = (double)Y[q];
#pragma unroll
            for (int a = 0; a < N; ++a) macc[a] = fma(wt, fma(z[2 * a], z[2 * a], z[2 * a + 1] * z[2 * a + 1]), macc[a]);
#pragma unroll
            for (int a = 0; a < N; ++a)
#pragma unroll
                for (int c2 = a + 1; c2 < N; ++c2) {
                    const int u = Shape<N>::up(a, c2);
                    const double re = fma(z[2 * a], z[2 * c2], z[2 * a + 1] * z[2 * c2 + 1]);
                    const double im = fma(z[2 * a + 1], z[2 * c2], -z[2 * a] * z[2 * c2 + 1]);
                    macc[N + 2 * u] = fma(wt, re, macc[N + 2 * u]);
                    macc[N + 2 * u + 1] = fma(wt * sg, im, macc[N + 2 * u + 1]);
                }
        }
    }

    // ---- wave reduction, per-trajectory weighting, then the block's trajectories
    //      in wave order (fixed) into one partial per block
    if constexpr (MOMENTS) {
#pragma unroll
        for (int i = 0; i < NM; ++i) macc[i] = wave_sum(macc[i]);
        if (lane == 0) {
            for (int v = 0; v < 2 * NM; ++v) spart[wave][v] = 0.0;
        }
        if (active && lane == 0) {
            // lab frame: S_ab = 2 e^{-i(Phi_a - Phi_b)} S~_ab ; S_aa = 2 S~_aa
            double Sl[NM];
            for (int a = 0; a < N; ++a) Sl[a] = 2.0 * macc[a];
            for (int u = 0; u < NU; ++u) {
                const double cs = zo[u][0], sn = zo[u][1];
                const double xr = macc[N + 2 * u], xi = macc[N + 2 * u + 1];
                Sl[N + 2 * u] = 2.0 * (cs * xr + sn * xi);
                Sl[N + 2 * u + 1] = 2.0 * (cs * xi - sn * xr);
            }
            const double w0 = wo, w1 = MA ? wo * co : 0.0;
            for (int v = 0; v < NM; ++v) {
                spart[wave][v] = w0 * Sl[v];
                spart[wave][NM + v] = w1 * Sl[v];
            }
        }
    }
    if constexpr (FINAL) {
        const double e = wave_max(emax);
        if (lane == 0) spart[wave][2 * NM] = e;
    }
    __syncthreads();
    if (threadIdx.x < 2 * NM + 1) {
        const int v = threadIdx.x;
        const bool is_err = (v == 2 * NM);
        if ((MOMENTS && !is_err) || (FINAL && is_err)) {
            double acc = spart[0][v];
            for (int w = 1; w < kTrajPerBlock; ++w) acc = is_err ? fmax(acc, spart[w][v]) : acc + spart[w][v];
            if (is_err) rc.errpart[blockIdx.x] = acc;
            else rc.partial[(size_t)blockIdx.x * 2 * NM + v] = acc;
        }
    }
}

// Finalisation of launch I: one workgroup adds the per-trajectory partials
// of all trajectories in a fixed order into J_I (deterministic), and for the
// final launch reduces the step error and runs the step controller.  Running
// it as its own launch (instead of a last-workgroup handoff inside k_stage)
// avoids a device-scope fence in every workgroup: on gfx950 such a fence
// writes back and invalidates the XCD's L2.
constexpr int kFinBlock = 1024;

template <int N, typename TAB, int I>
__global__ void __launch_bounds__(kFinBlock) k_finalize(const RunConst rc)
{
    constexpr int S = TAB::S;
    constexpr bool FINAL = (I == S);
    constexpr int NM = Shape<N>::NM;
    constexpr int NV = 2 * NM;
    constexpr int NW = kFinBlock / 64;
    constexpr bool MOMENTS = !FINAL || !TAB::fsal;
    __shared__ double sred[NV + 1][NW];

    const Control* ctl = rc.ctrl;
    if (I > 0 && ctl->status != 0) return;
    const double h = ctl->h;
    // one partial per stage block; contiguous ranges summed in ascending order
    const int nparts = (rc.na + kTrajPerBlock - 1) / kTrajPerBlock;
    const int per = (nparts + kFinBlock - 1) / kFinBlock;
    const int j0 = min(nparts, (int)threadIdx.x * per), j1 = min(nparts, j0 + per);

    double* Jout = rc.jhist + (FINAL ? S : I) * NV;
    if constexpr (MOMENTS) {
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
        for (int jj = j0; jj < j1; ++jj) {
            const double* src = rc.partial + (size_t)jj * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += src[v];
        }
        block_sum<NV, NW>(acc, sred);
        if (threadIdx.x == 0)
            for (int v = 0; v < NV; ++v) Jout[v] = acc[v];
    }
    if constexpr (FINAL) {
        double m = 0.0;
        for (int jj = j0; jj < j1; ++jj) m = fmax(m, rc.errpart[jj]);
        m = wave_max(m);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) sred[0][threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < NW; ++w) m = fmax(m, sred[0][w]);
            Control& C = *rc.ctrl;
            C.attempts += 1;
            const double* Jnext = rc.jhist + (TAB::fsal ? (S - 1) : S) * NV;
            if constexpr (!TAB::embedded) {
                // fixed step: always accepted
                if (!(m <= 1.0e300)) { C.status = -4; }
                else {
                    C.istep += 1;
                    C.nacc += 1;
                    C.cur ^= 1;
                    C.r = rc.r_start + (double)C.istep * rc.h_fixed;
                    C.h = rc.h_fixed;
                    for (int v = 0; v < NV; ++v) rc.jhist[v] = Jnext[v];
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
                        rn = C.r + h;
                        C.r = rn;
                        C.nacc += 1;
                        C.cur ^= 1;
                        for (int v = 0; v < NV; ++v) rc.jhist[v] = Jnext[v];
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
        }
    }
}

// ------------------------------------------------------------------ small kernels
template <typename T, int N>
__global__ void k_probabilities(const RunConst rc, double* __restrict__ p)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= rc.nb) return;
    const T* src = psi_ptr<T>(rc, rc.ctrl->cur);
    const double re = (double)src[0 * rc.nb_pad + b], im = (double)src[1 * rc.nb_pad + b];
    p[b] = re * re + im * im;
}

template <typename T, int N>
__global__ void k_init(const RunConst rc)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < rc.nb_pad) {
        T* dst = psi_ptr<T>(rc, rc.ctrl->cur);
        for (int q = 0; q < 2 * N; ++q) dst[q * rc.nb_pad + b] = (q == 0 && b < rc.nb) ? T(1) : T(0);
    }
    if (b < (int64_t)rc.na * N) rc.phase[rc.ctrl->cur][b] = 0.0;
}

// ------------------------------------------------------------------ dispatch
using StageFn = void (*)(const RunConst);

template <typename TS, typename T, int N, bool MA, typename TAB>
struct StageTable {
    template <int... Is>
    static constexpr std::array<StageFn, kMaxStages> make(std::integer_sequence<int, Is...>)
    {
        return {{(Is <= TAB::S ? (StageFn)&k_stage<TS, T, N, MA, TAB, (Is <= TAB::S ? Is : 0)> : nullptr)...}};
    }
    static constexpr std::array<StageFn, kMaxStages> fns = make(std::make_integer_sequence<int, kMaxStages>{});
};

template <int N, typename TAB>
struct FinTable {
    template <int... Is>
    static constexpr std::array<StageFn, kMaxStages> make(std::integer_sequence<int, Is...>)
    {
        return {{(Is <= TAB::S ? (StageFn)&k_finalize<N, TAB, (Is <= TAB::S ? Is : 0)> : nullptr)...}};
    }
    static constexpr std::array<StageFn, kMaxStages> fns = make(std::make_integer_sequence<int, kMaxStages>{});
};

StageFn pick_finalize(int n, int integrator, int stage)
{
    if (n == 2) return integrator == 0 ? FinTable<2, TabRK4>::fns[stage] : FinTable<2, TabDP54>::fns[stage];
    return integrator == 0 ? FinTable<3, TabRK4>::fns[stage] : FinTable<3, TabDP54>::fns[stage];
}

template <typename TS, typename T, int N, bool MA>
StageFn pick_tab(int integrator, int stage)
{
    return integrator == 0 ? StageTable<TS, T, N, MA, TabRK4>::fns[stage]
                           : StageTable<TS, T, N, MA, TabDP54>::fns[stage];
}
template <typename TS, typename T, int N>
StageFn pick_ma(int ma, int integrator, int stage)
{
    return ma ? pick_tab<TS, T, N, true>(integrator, stage) : pick_tab<TS, T, N, false>(integrator, stage);
}
template <typename TS, typename T>
StageFn pick_n(int n, int ma, int integrator, int stage)
{
    return n == 2 ? pick_ma<TS, T, 2>(ma, integrator, stage) : pick_ma<TS, T, 3>(ma, integrator, stage);
}

}  // namespace

int num_stages(int integrator) { return integrator == 0 ? TabRK4::S : TabDP54::S; }

hipError_t launch_stage(const RunConst& rc, int stage, hipStream_t s)
{
    if (stage < 0 || stage > num_stages(rc.integrator)) return hipErrorInvalidValue;
    StageFn fn = nullptr;
    switch (rc.precision) {
    case 0: fn = pick_n<double, double>(rc.n, rc.ma, rc.integrator, stage); break;   // FP64
    case 1: fn = pick_n<float, float>(rc.n, rc.ma, rc.integrator, stage); break;     // FP32 amplitudes
    case 2: fn = pick_n<float, double>(rc.n, rc.ma, rc.integrator, stage); break;    // FP32 amplitudes, FP64 math
    default: break;
    }
    StageFn fin = pick_finalize(rc.n, rc.integrator, stage);
    if (!fn || !fin) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((rc.na + kTrajPerBlock - 1) / kTrajPerBlock), dim3(64 * kTrajPerBlock), 0, s, rc);
    hipLaunchKernelGGL(fin, dim3(1), dim3(kFinBlock), 0, s, rc);
    return hipGetLastError();
}

hipError_t launch_probabilities(const RunConst& rc, double* p, hipStream_t s)
{
    const unsigned grid = (unsigned)((rc.nb + 255) / 256);
    if (rc.precision == 0) {
        if (rc.n == 2) hipLaunchKernelGGL((k_probabilities<double, 2>), dim3(grid), dim3(256), 0, s, rc, p);
        else hipLaunchKernelGGL((k_probabilities<double, 3>), dim3(grid), dim3(256), 0, s, rc, p);
    } else {
        if (rc.n == 2) hipLaunchKernelGGL((k_probabilities<float, 2>), dim3(grid), dim3(256), 0, s, rc, p);
        else hipLaunchKernelGGL((k_probabilities<float, 3>), dim3(grid), dim3(256), 0, s, rc, p);
    }
    return hipGetLastError();
}

hipError_t launch_init_state(const RunConst& rc, hipStream_t s)
{
    int64_t work = rc.nb_pad > (int64_t)rc.na * rc.n ? rc.nb_pad : (int64_t)rc.na * rc.n;
    const unsigned grid = (unsigned)((work + 255) / 256);
    if (rc.precision == 0) {
        if (rc.n == 2) hipLaunchKernelGGL((k_init<double, 2>), dim3(grid), dim3(256), 0, s, rc);
        else hipLaunchKernelGGL((k_init<double, 3>), dim3(grid), dim3(256), 0, s, rc);
    } else {
        if (rc.n == 2) hipLaunchKernelGGL((k_init<float, 2>), dim3(grid), dim3(256), 0, s, rc);
        else hipLaunchKernelGGL((k_init<float, 3>), dim3(grid), dim3(256), 0, s, rc);
    }
    return hipGetLastError();
}

}  // namespace nuosc
