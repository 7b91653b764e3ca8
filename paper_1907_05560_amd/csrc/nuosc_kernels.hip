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

// Runtime-indexed copies for the per-trajectory prologue (few lanes).
struct TabConst {
    double C[8];
    double A[8][8];
    double B[8];
};
template <typename TAB>
constexpr TabConst make_tab()
{
    TabConst t{};
    for (int i = 0; i < 8; ++i) {
        t.C[i] = TAB::C[i];
        t.B[i] = TAB::B[i];
        for (int j = 0; j < 8; ++j) t.A[i][j] = TAB::A[i][j];
    }
    return t;
}
__constant__ TabConst c_tab[2] = {make_tab<TabRK4>(), make_tab<TabDP54>()};

template <typename TAB> struct TabIndex;
template <> struct TabIndex<TabRK4> { static constexpr int v = 0; };
template <> struct TabIndex<TabDP54> { static constexpr int v = 1; };

// ------------------------------------------------------------------ helpers
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
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

// FP64 per-trajectory data of one stage, built by one lane.
template <int N> struct StageGeo {
    double r, c, w;
    double G[N];      // d Phi / dr of the co-rotating frame
    double phi[N];    // stage phase
};

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

// Sum NV doubles over the workgroup in a fixed order; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double* v, double (*lds)[kBlock / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
        for (int i = 0; i < NV; ++i) lds[i][wave] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < NV; ++i) {
            double s = lds[i][0];
            for (int w = 1; w < kBlock / 64; ++w) s += lds[i][w];
            v[i] = s;
        }
}

// ------------------------------------------------------------------ stage kernel
// TS: type of the amplitudes in HBM; T: arithmetic type of the stage update.
template <typename TS, typename T, int N, bool MA, typename TAB, int I>
__global__ void __launch_bounds__(kBlock) k_stage(const RunConst rc)
{
    constexpr int S = TAB::S;
    constexpr bool FINAL = (I == S);
    constexpr int NST = FINAL ? S : I;          // stages whose derivative is needed
    constexpr int NU = Shape<N>::NU, NM = Shape<N>::NM;
    constexpr bool MOMENTS = !FINAL || !TAB::fsal;  // final launch of RK4 also forms J of y_{n+1}
    constexpr int TABI = TabIndex<TAB>::v;

    const Control* ctl = rc.ctrl;
    if (I > 0 && ctl->status != 0) return;  // run finished: attempts are no-ops
    const int cur = ctl->cur;
    const double r = ctl->r, h = ctl->h;
    const int j = blockIdx.x;

    __shared__ StageMat<T, N> smat[NST > 0 ? NST : 1];
    __shared__ StageGeo<N> sgeo[kMaxStages];
    __shared__ double sred[2 * NM + 1][kBlock / 64];

    // ---- per-trajectory prologue (FP64): stage radii, geometry, frame rates
    const int nprol = NST + 1;  // stages 0..NST-1 plus the output stage
    if ((int)threadIdx.x < nprol) {
        const int l = threadIdx.x;
        StageGeo<N>& g = sgeo[l];
        double rl;
        if (l < NST) rl = r + c_tab[TABI].C[l] * h;
        else if (FINAL) rl = (rc.integrator == 0) ? rc.r_start + (double)(ctl->istep + 1) * rc.h_fixed : r + h;
        else rl = r + c_tab[TABI].C[I] * h;
        g.r = rl;
        traj_geometry(rc, j, rl, g.c, g.w);
        if (l < NST && rc.frame == 0) {
            double Cd[N], Cu[NU > 0 ? NU : 1][2];
            collective<N>(rc, rc.jhist + l * 2 * NM, g.c, Cd, Cu);
            const double lam = matter(rc, rl);
            for (int a = 0; a < N; ++a) g.G[a] = (lam * ((a == 0 ? 1.0 : 0.0) - 1.0 / N) + Cd[a]) / g.c;
        } else {
            for (int a = 0; a < N; ++a) g.G[a] = 0.0;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nprol) {
        const int l = threadIdx.x;
        StageGeo<N>& g = sgeo[l];
        const double* ph0 = rc.phase[cur] + (size_t)j * N;
        for (int a = 0; a < N; ++a) {
            double acc = 0.0;
            if (l < NST || !FINAL) {
                const int row = (l < NST) ? l : I;
                for (int m = 0; m < row; ++m) acc += c_tab[TABI].A[row][m] * sgeo[m].G[a];
            } else {
                for (int m = 0; m < S; ++m) acc += c_tab[TABI].B[m] * sgeo[m].G[a];
            }
            g.phi[a] = ph0[a] + h * acc;
        }
        if (l < NST) {
            // Hamiltonian pieces of stage l in the co-rotating frame:
            //   nu:    A_ab = e^{i(Phi_a-Phi_b)} C_ab / c,  B_ab = e^{i(Phi_a-Phi_b)} V_ab / c
            //          A_aa = 0 (co-rotating) or (H_m + C)_aa / c (lab),  B_aa = V_aa / c
            //   nubar: A -> -conj(A), B -> conj(B)   (eq 3.4 map, Phibar = -Phi)
            double Cd[N], Cu[NU > 0 ? NU : 1][2];
            collective<N>(rc, rc.jhist + l * 2 * NM, g.c, Cd, Cu);
            const double lam = matter(rc, g.r);
            const double ic = 1.0 / g.c;
            SpeciesMat<T, N>& nu = smat[l].sp[0];
            SpeciesMat<T, N>& nb = smat[l].sp[1];
            for (int a = 0; a < N; ++a) {
                const double vd = rc.vac[a][a][0] * ic;
                const double ad = (rc.frame == 0) ? 0.0 : (lam * ((a == 0 ? 1.0 : 0.0) - 1.0 / N) + Cd[a]) * ic;
                nu.ad[a] = (T)ad;
                nb.ad[a] = (T)(-ad);
                nu.bd[a] = nb.bd[a] = (T)vd;
            }
            for (int a = 0; a < N; ++a)
                for (int b = a + 1; b < N; ++b) {
                    const int u = Shape<N>::up(a, b);
                    double sn, cs;
                    sincos(g.phi[a] - g.phi[b], &sn, &cs);
                    const double cr = Cu[u][0] * ic, ci = Cu[u][1] * ic;
                    const double vr = rc.vac[a][b][0] * ic, vi = rc.vac[a][b][1] * ic;
                    const double Ar = cs * cr - sn * ci, Ai = cs * ci + sn * cr;
                    const double Br = cs * vr - sn * vi, Bi = cs * vi + sn * vr;
                    nu.au[u][0] = (T)Ar;  nu.au[u][1] = (T)Ai;
                    nu.bu[u][0] = (T)Br;  nu.bu[u][1] = (T)Bi;
                    nb.au[u][0] = (T)(-Ar); nb.au[u][1] = (T)Ai;
                    nb.bu[u][0] = (T)Br;  nb.bu[u][1] = (T)(-Bi);
                }
        }
    }
    __syncthreads();

    // ---- per-beam work
    T hA[NST > 0 ? NST + 1 : 1][NST > 0 ? NST : 1];
    static_for<0, NST + 1>([&](auto Lc) {
        constexpr int l = decltype(Lc)::value;
        static_for<0, (l < NST ? l : NST)>([&](auto Mc) {
            constexpr int m = decltype(Mc)::value;
            if constexpr (l < NST) hA[l][m] = (T)(h * TAB::A[l][m]);
            else if constexpr (FINAL) hA[l][m] = (T)(h * TAB::B[m]);
            else hA[l][m] = (T)(h * TAB::A[I][m]);
        });
    });

    const TS* __restrict__ src = psi_ptr<TS>(rc, cur);
    TS* __restrict__ dst = psi_ptr<TS>(rc, cur ^ 1);
    const int64_t ld = rc.nb_pad;
    double macc[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) macc[i] = 0.0;
    double emax = 0.0;

    for (int t = threadIdx.x; t < 2 * rc.ne; t += kBlock) {
        const int s = (t >= rc.ne) ? 1 : 0;
        const int k = t - s * rc.ne;
        const int64_t b = ((int64_t)s * rc.na + j) * rc.ne + k;
        T y[2 * N];
#pragma unroll
        for (int q = 0; q < 2 * N; ++q) y[q] = (T)src[q * ld + b];
        const T inv_e = (T)rc.inv_e[k];

        T kk[NST > 0 ? NST : 1][2 * N];
        static_for<0, NST>([&](auto Lc) {
            constexpr int l = decltype(Lc)::value;
            T Y[2 * N];
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) Y[q] = y[q];
            static_for<0, l>([&](auto Mc) {
                constexpr int m = decltype(Mc)::value;
                if constexpr (TAB::A[l][m] != 0.0) {
#pragma unroll
                    for (int q = 0; q < 2 * N; ++q) Y[q] = fma(hA[l][m], kk[m][q], Y[q]);
                }
            });
            eval_k<T, N>(smat[l].sp[s], inv_e, Y, kk[l]);
        });

        // output state: Y_I (stage) or y_{n+1} (final)
        T Y[2 * N];
#pragma unroll
        for (int q = 0; q < 2 * N; ++q) Y[q] = y[q];
        static_for<0, NST>([&](auto Mc) {
            constexpr int m = decltype(Mc)::value;
            constexpr double coef = FINAL ? TAB::B[m] : TAB::A[I < S ? I : 0][m];
            if constexpr (coef != 0.0) {
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) Y[q] = fma(hA[NST][m], kk[m][q], Y[q]);
            }
        });
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

    // ---- workgroup reduction and per-trajectory output
    if constexpr (MOMENTS) {
        block_sum<NM>(macc, sred);
        if (threadIdx.x == 0) {
            const StageGeo<N>& g = sgeo[NST];
            // lab frame: S_ab = 2 e^{-i(Phi_a - Phi_b)} S~_ab ; S_aa = 2 S~_aa
            double Sl[NM];
            for (int a = 0; a < N; ++a) Sl[a] = 2.0 * macc[a];
            for (int a = 0; a < N; ++a)
                for (int b = a + 1; b < N; ++b) {
                    const int u = Shape<N>::up(a, b);
                    double sn, cs;
                    sincos(g.phi[a] - g.phi[b], &sn, &cs);
                    const double xr = macc[N + 2 * u], xi = macc[N + 2 * u + 1];
                    Sl[N + 2 * u] = 2.0 * (cs * xr + sn * xi);
                    Sl[N + 2 * u + 1] = 2.0 * (cs * xi - sn * xr);
                }
            const double w0 = g.w, w1 = MA ? g.w * g.c : 0.0;
            for (int v = 0; v < NM; ++v) {
                rc.partial[(size_t)v * rc.na + j] = w0 * Sl[v];
                rc.partial[(size_t)(NM + v) * rc.na + j] = w1 * Sl[v];
            }
        }
    }
    if constexpr (FINAL) {
        __syncthreads();  // sred may still be read by the moment reduction
        double e = wave_max(emax);
        if ((threadIdx.x & 63) == 0) sred[0][threadIdx.x >> 6] = e;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = sred[0][0];
            for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, sred[0][w]);
            rc.errpart[j] = m;
            // new phases of this trajectory (kept only if the attempt is accepted)
            double* ph1 = rc.phase[cur ^ 1] + (size_t)j * N;
            for (int a = 0; a < N; ++a) ph1[a] = sgeo[NST].phi[a];
        }
    }

}

// Finalisation of launch I: one workgroup adds the per-trajectory partials
// of all trajectories in a fixed order into J_I (deterministic), and for the
// final launch reduces the step error and runs the step controller.  Running
// it as its own launch (instead of a last-workgroup handoff inside k_stage)
// avoids a device-scope fence in every workgroup: on gfx950 such a fence
// writes back and invalidates the XCD's L2.
template <int N, typename TAB, int I>
__global__ void __launch_bounds__(kBlock) k_finalize(const RunConst rc)
{
    constexpr int S = TAB::S;
    constexpr bool FINAL = (I == S);
    constexpr int NM = Shape<N>::NM;
    constexpr bool MOMENTS = !FINAL || !TAB::fsal;
    __shared__ double sred[2 * NM + 1][kBlock / 64];

    const Control* ctl = rc.ctrl;
    if (I > 0 && ctl->status != 0) return;
    const double h = ctl->h;

    double* Jout = rc.jhist + (FINAL ? S : I) * 2 * NM;
    if constexpr (MOMENTS) {
        double acc[2 * NM];
#pragma unroll
        for (int v = 0; v < 2 * NM; ++v) acc[v] = 0.0;
        for (int jj = threadIdx.x; jj < rc.na; jj += kBlock)
#pragma unroll
            for (int v = 0; v < 2 * NM; ++v) acc[v] += rc.partial[(size_t)v * rc.na + jj];
        block_sum<2 * NM>(acc, sred);
        if (threadIdx.x == 0)
            for (int v = 0; v < 2 * NM; ++v) Jout[v] = acc[v];
    }
    if constexpr (FINAL) {
        double m = 0.0;
        for (int jj = threadIdx.x; jj < rc.na; jj += kBlock) m = fmax(m, rc.errpart[jj]);
        m = wave_max(m);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) sred[0][threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, sred[0][w]);
            Control& C = *rc.ctrl;
            C.attempts += 1;
            const double* Jnext = rc.jhist + (TAB::fsal ? (S - 1) : S) * 2 * NM;
            if constexpr (!TAB::embedded) {
                // fixed step: always accepted
                if (!(m <= 1.0e300)) { C.status = -4; }
                else {
                    C.istep += 1;
                    C.nacc += 1;
                    C.cur ^= 1;
                    C.r = rc.r_start + (double)C.istep * rc.h_fixed;
                    C.h = rc.h_fixed;
                    for (int v = 0; v < 2 * NM; ++v) rc.jhist[v] = Jnext[v];
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
                        for (int v = 0; v < 2 * NM; ++v) rc.jhist[v] = Jnext[v];
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
    hipLaunchKernelGGL(fn, dim3(rc.na), dim3(kBlock), 0, s, rc);
    hipLaunchKernelGGL(fin, dim3(1), dim3(kBlock), 0, s, rc);
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
