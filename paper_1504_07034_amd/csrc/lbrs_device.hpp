// Device-side building blocks of the LBRS step kernels (gfx950, FP64).
//
// Physics follows Sec. II of Raghurama Rao, Deshmukh & Kotnala (arXiv
// 1504.07034): gamma-law Euler fluxes (Sec. II.C, the 2D form by the standard
// equations), algebraic equilibria of the diagonal relaxation system (D1Q2 and
// D1Q3, Sec. II.C; D2Q4, Sec. II.D), BGK relaxation with omega = dt/epsilon
// and exact hopping (Sec. II.A), the Jin-Xin wave-speed bound in 1D
// (Sec. II.C) and the Bouchut bound in 2D (Sec. II.D, "sqrt(2a)" read as
// sqrt(2)*a), and the specular free-slip wall (Sec. II.E).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbrs {

enum : int { D1Q2 = 0, D1Q3 = 1, D2Q4 = 2 };
enum : int { BC_TRANSMISSIVE = 0, BC_PERIODIC = 1, BC_WALL = 2, BC_DIRICHLET = 3 };
enum : int { LAM_PER_STEP = 0, LAM_FROZEN = 1, LAM_USER = 2 };

// ---------------------------------------------------------------- time state
// One launch of a step kernel reads slot (p & 1) and the reduction slot p % 3
// (p = host launch counter), accumulates the next bound into slot (p+1) % 3,
// clears slot (p+2) % 3, and block 0 writes the next time state into slot
// (p+1) & 1.  No slot is ever read and written by the same launch, so every
// workgroup of a launch sees the same t, lambda* and status without a grid
// barrier, and captured sequences of launches replay with period 6.
struct Slot {
    double t;          // time at the start of the next step
    long long n;       // completed steps
    double lam_used;   // lattice speed of the step that produced this state
    int cur;           // which population buffer holds f^n (0: f0, 1: f1)
    int pad;
};

struct DevState {
    Slot s[2];
    unsigned long long lam[3];   // lambda* accumulators: bit patterns of doubles >= 0
    unsigned int bad[3];         // non-physical flags, slotted like lam
    unsigned int status;         // sticky report: bit 0 = non-physical met
    unsigned long long fail_step;// first non-physical state (ULLONG_MAX = none)
    double lam_fixed;            // lattice speed of FROZEN / USER modes
    unsigned long long lam_init; // lambda*(U0) accumulator used by init
    double J;                    // objective accumulator
    unsigned long long lam_bc;   // bound of the prescribed (Dirichlet) side states
};

struct LaunchSlots {
    int sr, sw;        // time-state slot read / written
    int lr, la, lz;    // reduction slot read / accumulated / cleared
};

__host__ __device__ inline LaunchSlots slots_for(long long p) {
    LaunchSlots s;
    int p6 = (int)(p % 6);
    s.sr = p6 & 1;
    s.sw = s.sr ^ 1;
    s.lr = p6 % 3;
    s.la = (p6 + 1) % 3;
    s.lz = (p6 + 2) % 3;
    return s;
}

// Time control of one step (identical in every thread of a launch).
struct StepCtl {
    bool active;
    double lam;     // lattice speed of this step
    double t_new;
    int cur;
    long long n;
};

// dt = min(cfl*dx/lambda*, t_end - t) with the lattice speed dx/dt in the
// per-step mode; the fixed lattice speed and dt = dx/lambda otherwise.
__device__ inline StepCtl step_control(const DevState* st, LaunchSlots ls, int lam_mode,
                                       double dx, double cfl, double t_end) {
    StepCtl c;
    const Slot s = st->s[ls.sr];
    c.cur = s.cur;
    c.n = s.n;
    double t = s.t;
    bool bad = st->bad[ls.lr] != 0u;
    c.active = !bad && (t < t_end);
    if (lam_mode == LAM_PER_STEP) {
        // the ghost cells of Dirichlet sides count like interior cells
        double lam_star = __longlong_as_double((long long)(st->lam[ls.lr] > st->lam_bc
                                                               ? st->lam[ls.lr]
                                                               : st->lam_bc));
        double dt = cfl * dx / lam_star;
        double rem = t_end - t;
        bool last = false;
        if (dt >= rem) {
            dt = rem;
            last = true;
        }
        c.lam = dx / dt;
        c.t_new = last ? t_end : t + dt;
    } else {
        c.lam = st->lam_fixed;
        c.t_new = t + dx / c.lam;
    }
    return c;
}

// Block 0, thread 0 publishes the next time state and rotates the slots.
__device__ inline void publish_state(DevState* st, LaunchSlots ls, const StepCtl& c) {
    Slot s = st->s[ls.sr];
    if (c.active) {
        s.t = c.t_new;
        s.n = c.n + 1;
        s.lam_used = c.lam;
        s.cur = c.cur ^ 1;
    } else {
        // carry the bound and the flag unchanged into the slot the next launch reads
        st->lam[ls.la] = st->lam[ls.lr];
        st->bad[ls.la] = st->bad[ls.lr];
    }
    st->s[ls.sw] = s;
    st->lam[ls.lz] = 0ull;
    st->bad[ls.lz] = 0u;
}

// ----------------------------------------------------------- 2D Euler, D2Q4
// Conserved U = (rho, m, n, E) with m = rho u, n = rho v, E = rho e_total.
struct Euler2 {
    double u, v, p, H;  // velocity, pressure, E + p
};

// The per-cell arithmetic below is written with the multiply-adds the kernels
// take spelled out (fma_rn) and contraction off inside: the compiler may not
// fuse a product into a sum on its own, so every inlined copy of a step (a
// tile's first rows and its loop, the fused and single kernels, the
// prediction of the next bound) rounds every cell alike, bit for bit.
__device__ inline double fma_rn(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ inline Euler2 euler2(const double U[4], double gm1) {
#pragma clang fp contract(off)
    Euler2 e;
    double ir = 1.0 / U[0];
    e.u = U[1] * ir;
    e.v = U[2] * ir;
    // (m u + n v) / 2, symmetric in x and y
    double ke = 0.5 * (U[1] * e.u + U[2] * e.v);
    e.p = gm1 * (U[3] - ke);
    e.H = U[3] + e.p;
    return e;
}

// Fluxes G1 = F(U), G2 = G(U) of the 2D Euler equations.
__device__ inline void fluxes_d2q4(const double U[4], const Euler2& e, double G1[4],
                                   double G2[4]) {
#pragma clang fp contract(off)
    G1[0] = U[1];
    G1[1] = fma_rn(U[1], e.u, e.p);
    G1[2] = U[1] * e.v;
    G1[3] = e.u * e.H;
    G2[0] = U[2];
    G2[1] = U[2] * e.u;
    G2[2] = fma_rn(U[2], e.v, e.p);
    G2[3] = e.v * e.H;
}

// (1-omega) f + omega x.
__device__ inline double relax(double om1, double f, double omega, double x) {
#pragma clang fp contract(off)
    return fma_rn(om1, f, omega * x);
}

// Post-collision populations of one cell, fs = (1-omega) f + omega f^eq, with
// f^eq_i = U/4 + (s_ix G1 + s_iy G2)/(4 lambda); the four sign patterns are
// folded into a = G1 + G2 and b = G1 - G2.  f and fs: [i][k], 16 values.
__device__ inline void collide_d2q4(const double f[16], const double U[4], const Euler2& e,
                                    double c4lam, double omega, double fs[16]) {
#pragma clang fp contract(off)
    double G1[4], G2[4];
    fluxes_d2q4(U, e, G1, G2);
    const double om1 = 1.0 - omega;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double q = 0.25 * U[k];
        double a = (G1[k] + G2[k]) * c4lam;
        double b = (G1[k] - G2[k]) * c4lam;
        fs[0 * 4 + k] = relax(om1, f[0 * 4 + k], omega, q - a);
        fs[1 * 4 + k] = relax(om1, f[1 * 4 + k], omega, q + b);
        fs[2 * 4 + k] = relax(om1, f[2 * 4 + k], omega, q + a);
        fs[3 * 4 + k] = relax(om1, f[3 * 4 + k], omega, q - b);
    }
}

// Equilibria alone, f^eq_i = U/4 + (s_ix G1 + s_iy G2)/(4 lambda), in the same
// folded form as the collision (the populations of a Dirichlet ghost cell).
__device__ inline void equilibria_d2q4(const double U[4], const Euler2& e, double c4lam,
                                       double feq[16]) {
#pragma clang fp contract(off)
    double G1[4], G2[4];
    fluxes_d2q4(U, e, G1, G2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double q = 0.25 * U[k];
        double a = (G1[k] + G2[k]) * c4lam;
        double b = (G1[k] - G2[k]) * c4lam;
        feq[0 * 4 + k] = q - a;
        feq[1 * 4 + k] = q + b;
        feq[2 * 4 + k] = q + a;
        feq[3 * 4 + k] = q - b;
    }
}

// U = sum_i f_i, summed as (f1 + f3) + (f2 + f4) for every component.
__device__ inline void moments_d2q4(const double f[16], double U[4]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < 4; ++k) U[k] = (f[k] + f[8 + k]) + (f[4 + k] + f[12 + k]);
}

// Local bound max(|u+v|, |u+v +- sqrt2 a|, |u-v|, |u-v -+ sqrt2 a|), which for
// a >= 0 is max(|u+v|, |u-v|) + sqrt2 a exactly.  Returns false (and 0) for a
// non-physical state.
// An admissible state: positive density and pressure, every value finite.
__device__ inline bool admissible_d2q4(const double U[4], const Euler2& e) {
    return (U[0] > 0.0) && (e.p > 0.0) && isfinite(U[0]) && isfinite(U[1]) && isfinite(U[2]) &&
           isfinite(U[3]) && isfinite(e.p);
}

__device__ inline bool bound_d2q4(const double U[4], double gamma, double* lam) {
#pragma clang fp contract(off)
    double gm1 = gamma - 1.0;
    Euler2 e = euler2(U, gm1);
    bool ok = admissible_d2q4(U, e);
    double a = sqrt(gamma * e.p / U[0]);
    double l = fma_rn(1.4142135623730951, a, fmax(fabs(e.u + e.v), fabs(e.u - e.v)));
    *lam = ok ? l : 0.0;
    return ok;
}

// A1(U)^T hx + A2(U)^T hy for the 2D Euler fluxes, with
// dp/dU = (gamma-1) (|u|^2/2, -u, -v, 1) and H = (E + p)/rho:
//   A1^T h = h0 e_m + h1 (2u e_m - u^2 e_rho + dp) + h2 (v e_m + u e_n - uv e_rho)
//            + h3 (H e_m - H u e_rho + u e_E + u dp)
//   A2^T g = g0 e_n + g1 (v e_m + u e_n - uv e_rho) + g2 (2v e_n - v^2 e_rho + dp)
//            + g3 (H e_n - H v e_rho + v e_E + v dp)
__device__ inline void flux_vjp_2d(const double U[4], double gamma, const double hx[4],
                                   const double hy[4], double out[4]) {
    const double gm1 = gamma - 1.0;
    const double ir = 1.0 / U[0];
    const double u = U[1] * ir, v = U[2] * ir;
    const double q2 = u * u + v * v;
    const double p = gm1 * (U[3] - 0.5 * U[0] * q2);
    const double H = (U[3] + p) * ir;
    const double al = hx[1] + u * hx[3];
    const double be = hy[2] + v * hy[3];
    const double ab = gm1 * (al + be);
    out[0] = -u * (u * hx[1] + v * hx[2] + H * hx[3]) - v * (u * hy[1] + v * hy[2] + H * hy[3]) +
             ab * 0.5 * q2;
    out[1] = hx[0] + 2.0 * u * hx[1] + v * hx[2] + H * hx[3] + v * hy[1] - ab * u;
    out[2] = u * hx[2] + hy[0] + u * hy[1] + 2.0 * v * hy[2] + H * hy[3] - ab * v;
    out[3] = u * hx[3] + v * hy[3] + ab;
}

// fbar^n of one cell (D2Q4 fixed-speed step) from the reverse-streamed
// fbar*_i = fbar^{n+1}_i(x + s_i) (fb, [i][k]) and the step's input U^n:
//   Ubar = omega [ (1/4) sum_i fbar*_i + (A1^T h_x + A2^T h_y)/(4 lambda) ],
//   h_d = sum_i s_{i,d} fbar*_i,   fbar^n_i = (1 - omega) fbar*_i + Ubar.
__device__ inline void adjoint_cell_d2q4(const double fb[16], const double U[4], double gamma,
                                         double omega, double lam, double out[16]) {
    double sum[4], hx[4], hy[4], vjp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sum[k] = (fb[k] + fb[8 + k]) + (fb[4 + k] + fb[12 + k]);
        hx[k] = (fb[4 + k] + fb[8 + k]) - (fb[k] + fb[12 + k]);
        hy[k] = (fb[8 + k] + fb[12 + k]) - (fb[k] + fb[4 + k]);
    }
    flux_vjp_2d(U, gamma, hx, hy, vjp);
    const double c4 = 1.0 / (4.0 * lam);
    const double om1 = 1.0 - omega;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double Ub = omega * (0.25 * sum[k] + c4 * vjp[k]);
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i * 4 + k] = om1 * fb[i * 4 + k] + Ub;
    }
}

// Ubar0 = sum_i (df_i^eq/dU)^T fbar0_i at U0 (adjoint of f^0 = f^eq(U0)).
__device__ inline void adjoint_init_cell_d2q4(const double fb[16], const double U[4], double gamma,
                                              double lam, double out[4]) {
    double sum[4], hx[4], hy[4], vjp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sum[k] = (fb[k] + fb[8 + k]) + (fb[4 + k] + fb[12 + k]);
        hx[k] = (fb[4 + k] + fb[8 + k]) - (fb[k] + fb[12 + k]);
        hy[k] = (fb[8 + k] + fb[12 + k]) - (fb[k] + fb[4 + k]);
    }
    flux_vjp_2d(U, gamma, hx, hy, vjp);
    const double c4 = 1.0 / (4.0 * lam);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = 0.25 * sum[k] + c4 * vjp[k];
}

// ----------------------------------------------------------- 1D Euler
__device__ inline void euler1(const double U[3], double gm1, double* u, double* p, double* H) {
#pragma clang fp contract(off)
    double ir = 1.0 / U[0];
    *u = U[1] * ir;
    *p = gm1 * (U[2] - 0.5 * U[1] * (*u));
    *H = U[2] + *p;
}

// f^eq for D1Q2: U/2 -+ G/(2 lambda); D1Q3: U/3 -+ G/(2 lambda) and U/3.
template <int Q>
__device__ inline void collide_1d(const double* f, const double U[3], double gm1, double c2lam,
                                  double omega, double* fs) {
#pragma clang fp contract(off)
    double u, p, H;
    euler1(U, gm1, &u, &p, &H);
    const double G[3] = {U[1], U[1] * u + p, u * H};
    const double om1 = 1.0 - omega;
    const double w = (Q == 2) ? 0.5 : (1.0 / 3.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double q = w * U[k];
        double g = G[k] * c2lam;
        fs[0 * 3 + k] = relax(om1, f[0 * 3 + k], omega, q - g);
        if (Q == 2) {
            fs[1 * 3 + k] = relax(om1, f[1 * 3 + k], omega, q + g);
        } else {
            fs[1 * 3 + k] = relax(om1, f[1 * 3 + k], omega, q);
            fs[2 * 3 + k] = relax(om1, f[2 * 3 + k], omega, q + g);
        }
    }
}

template <int Q>
__device__ inline void moments_1d(const double* f, double U[3]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < 3; ++k) U[k] = (Q == 2) ? (f[k] + f[3 + k]) : ((f[k] + f[6 + k]) + f[3 + k]);
}

// Local bound max(|u-a|, |u|, |u+a|) = |u| + a for a >= 0 (Sec. II.C).
__device__ inline bool bound_1d(const double U[3], double gamma, double* lam) {
#pragma clang fp contract(off)
    double u, p, H;
    euler1(U, gamma - 1.0, &u, &p, &H);
    bool ok = (U[0] > 0.0) && (p > 0.0) && isfinite(U[0]) && isfinite(U[1]) && isfinite(U[2]) &&
              isfinite(p);
    double a = sqrt(gamma * p / U[0]);
    *lam = ok ? fabs(u) + a : 0.0;
    return ok;
}

// ----------------------------------------------------------- reductions
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Publish a wave's bound: skip the atomic when the slot already holds a value
// at least as large (the accumulator only grows during a launch).
__device__ inline void publish_max(unsigned long long* slot, double v) {
    unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    unsigned long long seen = __atomic_load_n(slot, __ATOMIC_RELAXED);
    if (bits > seen) atomicMax(slot, bits);
}

__device__ inline void publish_bad(DevState* st, LaunchSlots ls, long long step_index) {
    atomicOr(&st->bad[ls.la], 1u);
    atomicOr(&st->status, 1u);
    atomicMin(&st->fail_step, (unsigned long long)step_index);
}

// Index of a cell along an axis for a pull from outside [0, n): wrap for a
// periodic axis, clamp otherwise (a wall's out-of-range pull is overwritten by
// the reflection afterwards).  Always in [0, n), for any j.
__device__ inline int map_index(int j, int n, bool periodic) {
    if (j >= 0 && j < n) return j;
    if (periodic) {
        int m = j % n;
        return m < 0 ? m + n : m;
    }
    return j < 0 ? 0 : n - 1;
}

// Workgroup id remapped so that consecutive logical blocks run on the same
// XCD (blocks are dealt round-robin to the 8 XCDs): XCD k gets a contiguous
// range, and neighbouring tiles share that XCD's L2.
__device__ inline int xcd_remap(int b, int nblocks) {
    const int nx = 8;
    int xcd = b % nx, idx = b / nx;
    int per = nblocks / nx, rem = nblocks % nx;
    return xcd * per + min(xcd, rem) + idx;
}

}  // namespace lbrs
