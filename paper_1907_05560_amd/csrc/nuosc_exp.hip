// gfx950 kernels of the paper's own stepper: exponential steps
// psi(l + dl) = exp(-i H dl) psi(l) (eq 3.10-3.12) inside the half-step /
// full-step loop with averaging and a maximum-error control (Section 4.2.3
// and the evolution loop of Section 5), in the lab frame, FP64.
//
// One attempt from psi0 at radius r with step h, U(H; a, b) = exp(-i H dl) the
// exponential step from radius a to b, dl = dr / ((c_j(a) + c_j(b)) / 2) the
// trajectory's path length across it (dr = b - a, taken as the step h or h/2
// itself; mean cosine of the two ends, Appendix A.4.3; eq 3.3):
//   H0 from psi0 at r;       psi1 = U(H0; r, r+h) psi0,  psi4 = U(H0; r, r+h/2) psi0
//   H1 from psi1 at r + h;   H2 from psi4 at r + h/2
//   psi3 = (psi1 + U(H1; r, r+h) psi0) / 2             full-step estimate
//   psi5 = U(H2; r+h/2, r+h) psi4;  H3 from psi5 at r + h
//   psi7 = (psi1 + U(H3; r, r+h) psi0) / 2             two-half-step estimate
//   err = max over beams, components, re/im of |psi3 - psi7| / rtol;
//   an accepted attempt advances to psi7 (controller exponent 1/3).
// The two Hamiltonian reductions the paper fuses (H1 and H2 from the first
// two evolutions) are one reduction here too.  Per attempt: three beam
// launches, each followed by one small reduction launch:
//   k_exp_beam<1>: psi1, psi4 (both written); weighted density sums of both;
//   k_exp_reduce<1>: J of psi1 (at r + h) and of psi4 (at r + h/2);
//   k_exp_beam<2>: psi5 from psi4; its density sums;
//   k_exp_reduce<2>: J of psi5 (at r + h);
//   k_exp_beam<3>: U(H1) psi0, U(H3) psi0, psi3, psi7 (with psi1), the error;
//     writes psi7 and its density sums;
//   k_exp_reduce<3>: error maximum, step control, J of the next attempt's H0
//     (of psi7 if accepted, else unchanged).
// Launch 0 (k_exp_beam<0>, k_exp_reduce<0>) forms J of the current state.
// The kernels are bound by vector-ALU issue, with HBM mostly idle: launch 1
// stores psi1 and psi4 (FP64) for launches 3 and 2 rather than have them
// recompute the two exponentials; launch 2 reads psi4 only, launch 3 psi0
// and psi1, and writes psi7.
//
// Beams: one wavefront per trajectory j, lanes over its 2 N_E beam slots,
// four trajectories per workgroup (one partial density sum per workgroup).
// Antineutrino amplitudes are held complex-conjugated on the device, so one
// matrix pair per trajectory serves both species: H = A + u B with A = H_m + H_nunu, B = V, H_vac(E) = V / E,
// and u = +1/E (neutrinos) or -1/E (antineutrinos).
//
// 3x3 exponential: for traceless Hermitian Q with c0 = det Q, c1 = tr(Q^2)/2,
// Cayley-Hamilton gives exp(iQ) = f0 + f1 Q + f2 Q^2 with closed-form f_j
// of the eigenvalue parametrisation q = 2u, -u +- w (Morningstar and
// Peardon, Phys. Rev. D 69, 054501 (2004)), evaluated for c0 >= 0
// and mapped to c0 < 0 by Q -> -Q.  Two flavors: eq 3.11.  Steps of different
// length with the same H share its spectrum (u and w scale with the length).
#include "nuosc_internal.hpp"
#include "nuosc_device.hpp"

#include <math.h>

namespace nuosc {
namespace {

constexpr int kExpTraj = kExpTrajPerBlock;  // trajectories (wavefronts) per workgroup
constexpr int kExpBlock = 64 * kExpTraj;

// wavefront sums and maxima: the DPP row reductions of nuosc_device.hpp
// (cross-lane moves of the vector ALU, no LDS permutes)
__device__ __forceinline__ double xwave_sum(double v) { return wave_sum_rows(v); }
__device__ __forceinline__ double xwave_max(double v) { return wave_max_rows(v); }

// Geometry of trajectory j at radius r (eq 3.14-3.15; single angle: c = 1,
// w = D(r/R) of eq 3.17); the same formulas as the Runge-Kutta stage kernels.
__device__ __forceinline__ void xgeometry(const RunConst& rc, int j, double r, double& c, double& w)
{
    const double x = (rc.r_nu / r) * (rc.r_nu / r);
    const double y = (r - rc.r_nu) * (r + rc.r_nu) / (r * r);
    if (rc.ma) {
        const double du = 1.0 / (double)rc.nth;
        const double u = ((double)j + 0.5) * du;
        c = sqrt(fma(1.0 - u * u, y, u * u));
        w = x * u * du / c;
    } else {
        c = 1.0;
        const double s = 1.0 - sqrt(y);
        w = 0.5 * s * s;
    }
}

__device__ __forceinline__ double xmatter(const RunConst& rc, double r)
{
    const double x = rc.lambda_rref / r, p = rc.lambda_power;
    if (p == 3.0) return rc.lambda0 * (x * x * x);
    return rc.lambda0 * pow(x, p);
}

// ------------------------------------------------------------------ complex helpers
struct cd { double re, im; };
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.re, -a.im}; }

// y = K x for packed Hermitian K (N real diagonal entries, then the upper
// pairs a < b as (re, im)); x, y: N complex amplitudes as (re, im).
template <int N>
__device__ __forceinline__ void herm_apply(const double* K, const double* x, double* y)
{
#pragma unroll
    for (int a = 0; a < N; ++a) {
        y[2 * a] = K[a] * x[2 * a];
        y[2 * a + 1] = K[a] * x[2 * a + 1];
    }
    int u = 0;
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = a + 1; b < N; ++b, ++u) {
            const double kr = K[N + 2 * u], ki = K[N + 2 * u + 1];
            // y_a += k x_b ; y_b += conj(k) x_a
            y[2 * a] += kr * x[2 * b] - ki * x[2 * b + 1];
            y[2 * a + 1] += kr * x[2 * b + 1] + ki * x[2 * b];
            y[2 * b] += kr * x[2 * a] + ki * x[2 * a + 1];
            y[2 * b + 1] += kr * x[2 * a + 1] - ki * x[2 * a];
        }
}


// 1 / d: the hardware reciprocal refined by two Newton steps r <- r (2 - d r)
// (each squares the relative error), for d away from 0 and overflow.
__device__ __forceinline__ double xrcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
}

// sin(w) / w (near 0 its Taylor series; the divisions by constants are
// written as products, which the compiler keeps as exact divisions otherwise)
__device__ __forceinline__ double sinc_of(double w, double sw)
{
    const double w2 = w * w;
    if (fabs(w) < 0.05)
        return 1.0 - w2 * (1.0 / 6.0) * (1.0 - w2 * (1.0 / 20.0) * (1.0 - w2 * (1.0 / 42.0)));
    return sw * xrcp(w);
}

// Spectrum of K, independent of the step length t: with Q = t K,
// u = t ub, w = t wb; neg: det K < 0 (then Q -> -Q); zero: K = 0.
struct Spec {
    double ub, wb;
    bool neg, zero;
};

template <int N>
__device__ __forceinline__ Spec spectrum_of(const double* K)
{
    Spec s;
    if constexpr (N == 2) {
        const double c1 = 0.5 * (K[0] * K[0] + K[1] * K[1]) + K[2] * K[2] + K[3] * K[3];
        s.ub = sqrt(c1);  // lambda of eq 3.12
        s.wb = 0.0;
        s.neg = false;
        s.zero = !(c1 > 0.0);
    } else {
        const double d0 = K[0], d1 = K[1], d2 = K[2];
        const cd a = {K[3], K[4]}, b = {K[5], K[6]}, c = {K[7], K[8]};  // K01, K02, K12
        const double na = a.re * a.re + a.im * a.im, nb = b.re * b.re + b.im * b.im, nc = c.re * c.re + c.im * c.im;
        const double c1 = 0.5 * (d0 * d0 + d1 * d1 + d2 * d2) + na + nb + nc;
        const cd acb = cmul(cmul(a, c), cconj(b));
        const double c0 = d0 * d1 * d2 - d0 * nc - d1 * nb - d2 * na + 2.0 * acb.re;
        s.zero = !(c1 > 0.0);
        s.neg = c0 < 0.0;
        // largest eigenvalue 2u of K for |c0|: the largest root of
        // q^3 - c1 q - |c0| = 0, by Newton's method from its upper bound
        // 2 sqrt(c1/3) (the cubic is convex there: monotone convergence);
        // then w^2 = c1 - 3u^2 (c1 = 3u^2 + w^2)
        const double ac0 = fabs(c0);
        double q = 2.0 * sqrt(c1 * (1.0 / 3.0));
        if (!s.zero) {
#pragma unroll
            for (int it = 0; it < 5; ++it) {
                const double q2 = q * q;
                // an approximate reciprocal leaves the fixed point unchanged and the
                // convergence quadratic down to its own relative error
                q -= fma(q, q2 - c1, -ac0) * __builtin_amdgcn_rcp(fma(3.0, q2, -c1));
            }
        }
        s.ub = 0.5 * q;
        s.wb = sqrt(fmax(fma(-3.0 * s.ub, s.ub, c1), 0.0));
    }
    return s;
}

// Angles of one step length: cos/sin of u (and of w, 3 flavors), sin(w)/w.
struct Angles {
    double t, u, w, cu, su, cw, sw, xi;
};

template <int N>
__device__ __forceinline__ Angles angles_of(const Spec& s, double t)
{
    Angles g;
    g.t = t;
    g.u = s.ub * t;
    g.w = s.wb * t;
    fast_sincos(g.u, g.su, g.cu);
    if constexpr (N == 3) {
        fast_sincos(g.w, g.sw, g.cw);
        g.xi = sinc_of(g.w, g.sw);
    } else {
        g.cw = 1.0;
        g.sw = 0.0;
        g.xi = sinc_of(g.u, g.su);
    }
    return g;
}

// exp(-i t K) = g0 + g1 K + g2 K^2 (g1, g2 carry the powers of t).
struct Coef {
    cd g0, g1, g2;
};

template <int N>
__device__ __forceinline__ Coef coef_of(const Spec& s, const Angles& a)
{
    Coef k;
    if (s.zero) {
        k.g0 = {1.0, 0.0};
        k.g1 = k.g2 = {0.0, 0.0};
        return k;
    }
    if constexpr (N == 2) {
        // eq 3.11: exp(-i K t) = cos(lam t) - i t sinc(lam t) K
        k.g0 = {a.cu, 0.0};
        k.g1 = {0.0, -a.t * a.xi};
        k.g2 = {0.0, 0.0};
    } else {
        const double u = a.u, w = a.w, u2 = u * u, w2 = w * w;
        const cd e2 = {a.cu * a.cu - a.su * a.su, 2.0 * a.su * a.cu};  // e^{2iu}
        const cd em = {a.cu, -a.su};                                    // e^{-iu}
        const cd h0 = cadd(cscale(e2, u2 - w2), cmul(em, cd{8.0 * u2 * a.cw, 2.0 * u * (3.0 * u2 + w2) * a.xi}));
        const cd h1 = csub(cscale(e2, 2.0 * u), cmul(em, cd{2.0 * u * a.cw, -(3.0 * u2 - w2) * a.xi}));
        const cd h2 = csub(e2, cmul(em, cd{a.cw, 3.0 * u * a.xi}));
        const double inv = xrcp(9.0 * u2 - w2);  // >= 2 c1 t^2 > 0
        const cd f0 = cscale(h0, inv), f1 = cscale(h1, inv), f2 = cscale(h2, inv);
        const double t = a.t;
        if (!s.neg) {
            // exp(-iQ) = conj(f0) + conj(f1) Q + conj(f2) Q^2, f_j of exp(iQ)
            k.g0 = cconj(f0);
            k.g1 = cscale(cconj(f1), t);
            k.g2 = cscale(cconj(f2), t * t);
        } else {
            // det Q < 0: f_j of exp(-iQ) = exp(i(-Q)), in powers of -Q
            k.g0 = f0;
            k.g1 = cscale(f1, -t);
            k.g2 = cscale(f2, t * t);
        }
    }
    return k;
}

// y = g0 x + g1 Kx + g2 KKx
template <int N>
__device__ __forceinline__ void combine(const Coef& k, const double* x, const double* kx, const double* kkx, double* y)
{
#pragma unroll
    for (int a = 0; a < N; ++a) {
        cd v = cmul(k.g0, cd{x[2 * a], x[2 * a + 1]});
        v = cadd(v, cmul(k.g1, cd{kx[2 * a], kx[2 * a + 1]}));
        if constexpr (N == 3) v = cadd(v, cmul(k.g2, cd{kkx[2 * a], kkx[2 * a + 1]}));
        y[2 * a] = v.re;
        y[2 * a + 1] = v.im;
    }
}

// ------------------------------------------------------------------ per-trajectory tables
// Packed A = H_m(rs) + mu0 tl(J0 - c J1) and B = V of trajectory j (cosine c
// at radius rs), from the packed J0, J1 at jhist slot `set`: entry v of both,
// by lane v < N*N of the wavefront.
template <int N>
__device__ __forceinline__ void traj_tables(const RunConst& rc, int set, double rs, double c, int v, double* A,
                                            double* B)
{
    constexpr int NM = N * N;
    const double* J = rc.jhist + (size_t)set * 2 * NM;
    const double wc = rc.ma ? c : 0.0;  // single angle: J1 = 0
    if (v < N) {
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) tr += J[a] - wc * J[NM + a];
        const double lam = xmatter(rc, rs);
        const double hm = lam * ((v == 0 ? 1.0 : 0.0) - 1.0 / (double)N);
        const double hc = rc.mu0 * ((J[v] - wc * J[NM + v]) - tr / (double)N);
        A[v] = hm + hc;
        B[v] = rc.vac[v][v][0];
    } else if (v < NM) {
        const int q = v - N, p = q >> 1;  // upper pair p, re (q even) or im
        int a = 0, b = 1;
        if (N == 3) {
            a = p < 2 ? 0 : 1;
            b = p == 0 ? 1 : 2;
        }
        A[v] = rc.mu0 * (J[v] - wc * J[NM + v]);
        B[v] = rc.vac[a][b][q & 1];
    }
}

// Adds the weighted density matrix w x x^dagger (packed Hermitian) to acc.
template <int N>
__device__ __forceinline__ void add_density(double wt, const double* x, double* acc)
{
#pragma unroll
    for (int a = 0; a < N; ++a) acc[a] += wt * (x[2 * a] * x[2 * a] + x[2 * a + 1] * x[2 * a + 1]);
    int u = 0;
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = a + 1; b < N; ++b, ++u) {
            // x_a conj(x_b)
            acc[N + 2 * u] += wt * (x[2 * a] * x[2 * b] + x[2 * a + 1] * x[2 * b + 1]);
            acc[N + 2 * u + 1] += wt * (x[2 * a + 1] * x[2 * b] - x[2 * a] * x[2 * b + 1]);
        }
}

// Beam launch L (see the file header).
template <int N, int L>
// Launches 1 and 2: three wavefronts per SIMD (at most 168 VGPRs; a few
// spill): their evaluations are long FP64 dependency chains, and two
// wavefronts per SIMD leave the vector ALU idle more often than the spills
// cost.  Launch 3 (two full evaluations live) spills too much at that budget
// and runs two wavefronts per SIMD.
__global__ void __launch_bounds__(kExpBlock) __attribute__((amdgpu_waves_per_eu(L == 3 ? 2 : 3)))
k_exp_beam(const RunConst rc)
{
    constexpr int NM = N * N;
    constexpr int SETS = (L == 1) ? 2 : 1;           // density sums formed by this launch
    constexpr int NV = SETS * 2 * NM;                 // J0, J1 per set
    constexpr int NK = (L == 0) ? 0 : (L == 3 ? 2 : 1);  // Hamiltonians used
    __shared__ double sAB[kExpTraj][3][2][NM];
    __shared__ double sP[kExpTraj][NV];
    __shared__ double sE[kExpTraj];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = blockIdx.x * kExpTraj + wave;
    const bool live = j < rc.na;

    // attempt state: launch 1 reads the between-attempt copy and hands it on
    Control C;
    if constexpr (L == 0 || L == 1) {
        C = rc.ctrl[1];
        if (L == 1 && blockIdx.x == 0 && threadIdx.x == 0) rc.ctrl[0] = C;
    } else {
        C = rc.ctrl[0];
    }
    if (L != 0 && C.status != 0) return;
    const double r = C.r, h = C.h;

    // Hamiltonian k of this launch: J slot and radius
    //   L1: H0 (slot 0, r);  L2: H2 (slot 2, r + h/2);  L3: H1 (slot 1, r + h), H3 (slot 3, r + h)
    // cosines and weights at r, r + h/2, r + h; path lengths of the full step
    // and of the two half steps
    double cs[3] = {1.0, 1.0, 1.0}, ws[3] = {0.0, 0.0, 0.0};
    if (live) {
        xgeometry(rc, j, r, cs[0], ws[0]);
        xgeometry(rc, j, r + 0.5 * h, cs[1], ws[1]);
        xgeometry(rc, j, r + h, cs[2], ws[2]);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int set = L == 1 ? 0 : (L == 2 ? 2 : (k == 0 ? 1 : 3));
            const int at = L == 1 ? 0 : (L == 2 ? 1 : 2);
            const double rs = r + 0.5 * h * (double)at;
            if (lane < NM) traj_tables<N>(rc, set, rs, cs[at], lane, sAB[wave][k][0], sAB[wave][k][1]);
        }
    }
    const double dl_full = h / (0.5 * (cs[0] + cs[2]));
    const double dl_h1 = 0.5 * h / (0.5 * (cs[0] + cs[1]));
    const double dl_h2 = 0.5 * h / (0.5 * (cs[1] + cs[2]));
    // the density sums formed here are weighted at r (L0), r + h (L1: psi1;
    // L2, L3) and r + h/2 (L1: psi4)
    const double c0 = L == 0 ? cs[0] : cs[2], w0 = L == 0 ? ws[0] : ws[2];
    __syncthreads();

    double acc[SETS][NM];
#pragma unroll
    for (int s = 0; s < SETS; ++s)
#pragma unroll
        for (int v = 0; v < NM; ++v) acc[s][v] = 0.0;
    double emax = 0.0;

    const int cur = C.cur;
    const size_t ld = (size_t)rc.nb_pad;
    // launch 2 starts from psi4, the others from psi0
    const double* __restrict__ src = L == 2 ? rc.xbuf + 2 * N * ld : reinterpret_cast<const double*>(rc.psi[cur]);
    double* __restrict__ dst = reinterpret_cast<double*>(rc.psi[cur ^ 1]);
    double* __restrict__ x1 = rc.xbuf;            // psi1
    double* __restrict__ x4 = rc.xbuf + 2 * N * ld;  // psi4
    const int ne = rc.ne;
    if (live) {
        for (int t = lane; t < 2 * ne; t += 64) {
            const size_t b = (size_t)t + (size_t)j * ne + (t >= ne ? (size_t)(rc.na - 1) * ne : 0);
            const double u = rc.uinv64[t];
            const double wt = 2.0 * rc.wgt[t];
            double x0[2 * N];
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) x0[q] = src[q * ld + b];
            if constexpr (L == 0) {
                add_density<N>(wt, x0, acc[0]);
            } else if constexpr (L == 1) {
                double K[NM], kx[2 * N], kkx[2 * N];
#pragma unroll
                for (int v = 0; v < NM; ++v) K[v] = fma(u, sAB[wave][0][1][v], sAB[wave][0][0][v]);
                const Spec s0 = spectrum_of<N>(K);
                herm_apply<N>(K, x0, kx);
                if constexpr (N == 3) herm_apply<N>(K, kx, kkx);
                double p1[2 * N], p4[2 * N];
                combine<N>(coef_of<N>(s0, angles_of<N>(s0, dl_full)), x0, kx, kkx, p1);
                add_density<N>(wt, p1, acc[0]);
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) __builtin_nontemporal_store(p1[q], &x1[q * ld + b]);
                __builtin_amdgcn_sched_barrier(0);  // one exponential at a time
                combine<N>(coef_of<N>(s0, angles_of<N>(s0, dl_h1)), x0, kx, kkx, p4);
                add_density<N>(wt, p4, acc[SETS - 1]);
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) __builtin_nontemporal_store(p4[q], &x4[q * ld + b]);
            } else if constexpr (L == 2) {
                // x0 holds psi4 here
                double K[NM], kx[2 * N], kkx[2 * N], p5[2 * N];
#pragma unroll
                for (int v = 0; v < NM; ++v) K[v] = fma(u, sAB[wave][0][1][v], sAB[wave][0][0][v]);
                const Spec s2 = spectrum_of<N>(K);
                herm_apply<N>(K, x0, kx);
                if constexpr (N == 3) herm_apply<N>(K, kx, kkx);
                combine<N>(coef_of<N>(s2, angles_of<N>(s2, dl_h2)), x0, kx, kkx, p5);
                add_density<N>(wt, p5, acc[0]);
            } else {
                // one exponential at a time (interleaved, they spill); psi1 (stored
                // by launch 1) and the full-step estimate psi3 stay live between them
                double K[NM], kx[2 * N], kkx[2 * N];
                double p1[2 * N], p3[2 * N], pk[2 * N];
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) p1[q] = __builtin_nontemporal_load(&x1[q * ld + b]);
#pragma unroll
                for (int v = 0; v < NM; ++v) K[v] = fma(u, sAB[wave][0][1][v], sAB[wave][0][0][v]);
                const Spec s1 = spectrum_of<N>(K);
                herm_apply<N>(K, x0, kx);
                if constexpr (N == 3) herm_apply<N>(K, kx, kkx);
                combine<N>(coef_of<N>(s1, angles_of<N>(s1, dl_full)), x0, kx, kkx, pk);
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) p3[q] = 0.5 * (p1[q] + pk[q]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int v = 0; v < NM; ++v) K[v] = fma(u, sAB[wave][1][1][v], sAB[wave][1][0][v]);
                const Spec s3 = spectrum_of<N>(K);
                herm_apply<N>(K, x0, kx);
                if constexpr (N == 3) herm_apply<N>(K, kx, kkx);
                combine<N>(coef_of<N>(s3, angles_of<N>(s3, dl_full)), x0, kx, kkx, pk);
                double p7[2 * N];
#pragma unroll
                for (int q = 0; q < 2 * N; ++q) {
                    p7[q] = 0.5 * (p1[q] + pk[q]);
                    emax = fmax(emax, fabs(p3[q] - p7[q]));
                    __builtin_nontemporal_store(p7[q], &dst[q * ld + b]);
                }
                add_density<N>(wt, p7, acc[0]);
            }
        }
    }

    // workgroup partial: angle-weighted sums of the wavefronts' trajectories, in wavefront order
    double wJ[SETS][2];
    wJ[0][0] = w0;
    wJ[0][1] = rc.ma ? w0 * c0 : 0.0;
    if constexpr (SETS == 2) {
        wJ[1][0] = ws[1];
        wJ[1][1] = rc.ma ? ws[1] * cs[1] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < SETS; ++s)
#pragma unroll
        for (int v = 0; v < NM; ++v) {
            const double S = xwave_sum(acc[s][v]);
            if (lane == 0) {
                sP[wave][s * 2 * NM + v] = live ? wJ[s][0] * S : 0.0;
                sP[wave][s * 2 * NM + NM + v] = live ? wJ[s][1] * S : 0.0;
            }
        }
    if constexpr (L == 3) {
        emax = xwave_max(emax);
        if (lane == 0) sE[wave] = emax;
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double sum = sP[0][threadIdx.x];
        for (int w = 1; w < kExpTraj; ++w) sum += sP[w][threadIdx.x];
        rc.partial[(size_t)threadIdx.x * rc.nblk + blockIdx.x] = sum;
    }
    if (L == 3 && threadIdx.x == 0) {
        double m = sE[0];
        for (int w = 1; w < kExpTraj; ++w) m = fmax(m, sE[w]);
        rc.errpart[blockIdx.x] = m;
    }
}

// Controller of the adaptive attempt (readings J, K of the Runge-Kutta path
// with the exponent of a third-order local error).  Returns acceptance.
__device__ bool exp_control(const RunConst& rc, Control& C, double m)
{
    C.attempts += 1;
    bool accepted = false;
    const double h = C.h;
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
            fac = (err == 0.0) ? f_hi : rc.safety * pow(err, -1.0 / 3.0);
            fac = fmin(fmax(fac, f_lo), f_hi);
            if (C.last_rejected && fac > 1.0) fac = 1.0;
            C.last_rejected = 0;
        } else {
            C.nrej += 1;
            fac = fmax(rc.safety * pow(err, -1.0 / 3.0), f_lo);
            C.last_rejected = 1;
        }
        double hn = fmin(h * fac, rc.dr_max);
        C.h_prop = hn;
        if (rn >= C.r_end) {
            C.status = 1;
        } else if (hn < 1e-14 * rn) {
            C.status = -5;
        } else if (rn + hn > C.r_end) {
            hn = C.r_end - rn;
        }
        C.h = hn;
    }
    if (C.status == 0 && rc.max_steps > 0 && C.attempts >= rc.max_steps) C.status = -6;
    return accepted;
}

// Reduction launch L: J of the density sums of beam launch L, summed over the
// workgroups' partials in one fixed order (thread (v, c) adds partials c,
// c + CH, ... of value v; one thread per value adds the CH chunk sums), into
// jhist slots L0: 0;  L1: 1 (psi1), 2 (psi4);  L2: 3 (psi5);  L3: the next
// attempt's slot 0 if accepted, with the error maximum and the controller.
constexpr int kExpRed = 1024;  // threads of a reduction launch

template <int N, int L>
__global__ void __launch_bounds__(kExpRed) k_exp_reduce(const RunConst rc)
{
    constexpr int NM = N * N;
    constexpr int NV = (L == 1 ? 2 : 1) * 2 * NM;
    constexpr int CH = kExpRed / NV;
    __shared__ double sred[NV][CH];
    __shared__ double sJ[NV];
    __shared__ double serr[kExpRed / 64];
    if (L != 0 && rc.ctrl[0].status != 0) return;
    const int t = threadIdx.x;
    const int nblk = rc.nblk;
    if (t < NV * CH) {
        const int v = t / CH, c = t - v * CH;
        const double* pv = rc.partial + (size_t)v * nblk;
        double acc = 0.0;
        int p = c;
        for (; p + 3 * CH < nblk; p += 4 * CH) {  // four loads in flight, added in order
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
        sJ[t] = sum;
    }
    __syncthreads();
    if constexpr (L == 0) {
        if (t < NV) rc.jhist[t] = sJ[t];
    } else if constexpr (L == 1) {
        if (t < NV) rc.jhist[2 * NM + t] = sJ[t];  // slots 1 and 2 are adjacent
    } else if constexpr (L == 2) {
        if (t < NV) rc.jhist[3 * 2 * NM + t] = sJ[t];
    } else {
        double m = 0.0;
        for (int p = t; p < nblk; p += kExpRed) m = fmax(m, rc.errpart[p]);
        m = xwave_max(m);
        if ((t & 63) == 0) serr[t >> 6] = m;
        __syncthreads();
        if (t == 0) {
            for (int w = 1; w < kExpRed / 64; ++w) m = fmax(m, serr[w]);
            Control c = rc.ctrl[0];
            if (exp_control(rc, c, m))
                for (int v = 0; v < NV; ++v) rc.jhist[v] = sJ[v];
            rc.ctrl[1] = c;
        }
    }
}

template <int N>
hipError_t launch_n(const RunConst& rc, int stage, hipStream_t s, hipEvent_t* ev)
{
    using Fn = void (*)(const RunConst);
    Fn beam, red;
    switch (stage) {
    case 0: beam = &k_exp_beam<N, 0>; red = &k_exp_reduce<N, 0>; break;
    case 1: beam = &k_exp_beam<N, 1>; red = &k_exp_reduce<N, 1>; break;
    case 2: beam = &k_exp_beam<N, 2>; red = &k_exp_reduce<N, 2>; break;
    case 3: beam = &k_exp_beam<N, 3>; red = &k_exp_reduce<N, 3>; break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(beam, dim3((unsigned)rc.nblk), dim3(kExpBlock), 0, s, rc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(red, dim3(1), dim3(kExpRed), 0, s, rc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace

hipError_t launch_exp_stage(const RunList& runs, int stage, hipStream_t s, hipEvent_t* ev)
{
    if (runs.count != 1) return hipErrorInvalidValue;
    const RunConst& rc = *runs.rc[0];
    // one wavefront per trajectory, eight per workgroup: nblk must cover na
    if (rc.precision != 0 || rc.nj != 2 || (long long)rc.nblk * kExpTraj < rc.na || rc.nblk < 1)
        return hipErrorInvalidValue;
    return rc.n == 2 ? launch_n<2>(rc, stage, s, ev) : launch_n<3>(rc, stage, s, ev);
}

}  // namespace nuosc
