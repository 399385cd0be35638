// LBRS oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, deliberately unoptimised FP64 CPU implementation of the
// Lattice Boltzmann Relaxation Scheme (LBRS) of Raghurama Rao, Deshmukh and
// Kotnala, "A Lattice Boltzmann Relaxation Scheme for Inviscid Compressible
// Flows" (arXiv 1504.07034).  It exists so that the GPU library can be checked
// against something that a reader can compare with the paper by eye.  Only the
// test-suite, the smoke check and the CPU-baseline leg of the benchmark may load
// it.  It shares no source, header, table or helper with the GPU library.
//
// Every time step is taken in the paper's order (Sec. II):
//   moments U = sum_i f_i                      (eq. "moments", "moments_system")
//   global lattice speed from U                (Sec. II.C lambda choice; Sec. II.D
//                                               Bouchut bound for D2Q4)
//   equilibria f_i^eq(U, G(U))                 (eq. "equilibrium", the D1Q2/D1Q3
//                                               Euler equilibria, the D2Q4 f^eq)
//   relaxation (1-omega) f + omega f^eq        (discrete LBRS update, Sec. II.A)
//   exact hopping one node along each link     (same equation, lambda_i dt = dx)
//   boundary populations                       (Sec. II.E specular wall; the
//                                               transmissive and periodic sides are
//                                               readings, not in the paper)
//
// Readings of points the paper leaves open (each listed in the design notes):
//   * the lattice speed is one global value per step: lambda* = max over cells
//     of the local bound, and the lattice speed is lambda_lat = dx/dt with
//     dt = min(cfl*dx/lambda*, t_end - t)   (exact hopping needs one speed);
//   * the 2D bound's garbled "sqrt(2a)" is read as sqrt(2)*a;
//   * the D1Q3 model uses the same lambda formula as D1Q2;
//   * 2D Euler: E = p/(rho(gamma-1)) + (u^2+v^2)/2 and the standard fluxes;
//   * transmissive side: the ghost population equals the nearest interior
//     post-collision population (index clamped per axis); periodic: wrap;
//   * the wall sits on a node row (column); its incoming populations are set
//     after streaming by specular reflection of the outgoing ones, with the
//     normal momentum component negated (Sec. II.E, upper wall written out
//     there; the other three sides by the same mirror rule);
//   * Dirichlet side (the inflow and top boundaries of the oblique-shock case,
//     Sec. III, are prescribed but not described): the ghost cells beyond it
//     hold the prescribed conserved state U_b in equilibrium at the step's
//     lattice speed, so a population pulled from across it is f^eq_i(U_b);
//     at a corner ghost the y-side decides; the prescribed states take part
//     in the global lambda* maximum like interior cells;
//   * f^0 = f^eq(U0) with the lattice speed lambda*(U0)/cfl (frozen / user
//     modes: the fixed speed);
//   * solid bodies (the step, the backward step and the ramp of the Sec. III
//     test cases, whose geometry the paper does not give) are a mask of solid
//     cells; the wall runs through the fluid nodes next to the body, as on a
//     wall side.  A solid cell holds no populations (zero), takes no part in
//     lambda* and is never checked.  A population whose pull source is solid
//     takes the same-node specular image that makes the wall's normal flux
//     vanish (Sec. II.E): across a face (source's x- or y-neighbour solid) the
//     mirror population with that momentum component negated; in a concave
//     corner (both neighbours solid) the opposite population with both
//     components negated (the two images combined); at a convex corner tip
//     (only the diagonal source solid) the opposite population reflected about
//     the corner's bisector, which swaps the two momentum components.  Beyond
//     a wall side every position is solid; elsewhere a position outside the
//     grid is wrapped (periodic) or clamped onto it and the mask decides.
//
// The core is templated on the scalar so that a forward-mode dual number gives
// exact directional derivatives (the reference for the adjoint).
//
// Built twice from this one source: serially (g++ -O2, the build the tests
// use) and with -O3 -march=native -fopenmp for timing on all host cores.  The
// OpenMP pragmas only split the loops over cells (every cell is computed by
// the same code) and take the global maximum and the first non-physical cell
// as reductions, which do not depend on the order; both builds give the same
// bits (no contraction of multiply-adds in either).

#include <cmath>
#include <cstdint>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <cstring>
#include <vector>
#include <algorithm>
#include <limits>

namespace orc {

// ----------------------------------------------------------------- parameters
enum { D1Q2 = 0, D1Q3 = 1, D2Q4 = 2 };
enum { FLUX_EULER = 0, FLUX_LINEAR = 1, FLUX_QUADRATIC = 2 };
enum { SIDE_TRANSMISSIVE = 0, SIDE_PERIODIC = 1, SIDE_WALL = 2, SIDE_DIRICHLET = 3 };
enum { LAM_PER_STEP = 0, LAM_FROZEN = 1, LAM_USER = 2 };
enum { ST_OK = 0, ST_INVAL = -1, ST_NONPHYSICAL = -4 };

// Mirrored field by field in oracle/__init__.py (ctypes).
struct Problem {
    int model;        // D1Q2, D1Q3, D2Q4
    int flux;         // FLUX_EULER, or a scalar law: FLUX_LINEAR, FLUX_QUADRATIC
    int nx, ny;       // ny = 1 in 1D
    double x0, x1, y0, y1;
    double gamma, omega, cfl;
    int side[4];      // xlo, xhi, ylo, yhi
    int lam_mode;
    double lam_user;  // lattice speed for LAM_USER
    double adv_x, adv_y;  // advection speed for FLUX_LINEAR
    // Dirichlet data per side (xlo, xhi, ylo, yhi): conserved states [K][n]
    // along the side, n = ny for the x-sides and nx for the y-sides.
    const double* dir[4];
    // FLUX_QUADRATIC: g1(u) = q[0] u + q[1] u^2/2, g2(u) = q[2] u + q[3] u^2/2
    // (Burgers, Sec. II.A: q = (0, 1, ., .); the 2D Burgers law of Sec. III:
    // q = (0, 1, 1, 0)).
    double q[4];
    // Solid cells [ny][nx] (nonzero = solid), or null: no body (D2Q4 Euler).
    const unsigned char* solid;
};

// ------------------------------------------------------------ dual numbers
// Forward-mode AD: value and one directional derivative.
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double a) : v(a), d(0) {}
    Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual sqrt(Dual a) {
    double s = std::sqrt(a.v);
    return Dual(s, a.d / (2.0 * s));
}
inline Dual pow(Dual a, double e) {
    double p = std::pow(a.v, e);
    return Dual(p, e * std::pow(a.v, e - 1.0) * a.d);
}
inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }
using std::sqrt;
using std::pow;

// ------------------------------------------------------------ the lattices
// Sign pattern s_i of each discrete velocity (c_i = lambda * s_i).
//   D1Q2: Lambda = diag(-lambda, +lambda)                       (Sec. II.A)
//   D1Q3: Lambda = diag(-lambda, 0, +lambda)                    (Sec. II.C)
//   D2Q4: Lambda_1 = diag(-,+,+,-) lambda, Lambda_2 = diag(-,-,+,+) lambda
//                                                               (Sec. II.D)
inline int nq(int model) { return model == D1Q2 ? 2 : (model == D1Q3 ? 3 : 4); }
inline int ndim(int model) { return model == D2Q4 ? 2 : 1; }
inline int sx(int model, int i) {
    static const int s12[2] = {-1, +1};
    static const int s13[3] = {-1, 0, +1};
    static const int s24[4] = {-1, +1, +1, -1};
    return model == D1Q2 ? s12[i] : (model == D1Q3 ? s13[i] : s24[i]);
}
inline int sy(int model, int i) {
    static const int s24[4] = {-1, -1, +1, +1};
    return model == D2Q4 ? s24[i] : 0;
}
inline bool scalar_law(const Problem& P) { return P.flux != FLUX_EULER; }
inline int ncomp(const Problem& P) {
    if (scalar_law(P)) return 1;
    return ndim(P.model) == 1 ? 3 : 4;
}

// --------------------------------------------------------- Euler equations
// 1D: U = (rho, rho u, rho E), G = (rho u, p + rho u^2, p u + rho u E),
//     E = p/(rho(gamma-1)) + u^2/2                                (Sec. II.C)
template <class T>
void euler_flux_1d(const T* U, double gamma, T* G) {
    T rho = U[0];
    T u = U[1] / rho;
    T E = U[2] / rho;
    T p = (gamma - 1.0) * rho * (E - 0.5 * (u * u));
    G[0] = rho * u;
    G[1] = p + rho * u * u;
    G[2] = p * u + rho * u * E;
}

// 2D: U = (rho, rho u, rho v, rho E), E = p/(rho(gamma-1)) + (u^2+v^2)/2,
//     G1 = (rho u, p + rho u^2, rho u v, p u + rho u E),
//     G2 = (rho v, rho v u, p + rho v^2, p v + rho v E).
// The paper only names "the 2D Euler equations" (Sec. II.D); these are the
// standard gamma-law fluxes.
template <class T>
void euler_flux_2d(const T* U, double gamma, T* G1, T* G2) {
    T rho = U[0];
    T u = U[1] / rho;
    T v = U[2] / rho;
    T E = U[3] / rho;
    T p = (gamma - 1.0) * rho * (E - 0.5 * (u * u + v * v));
    G1[0] = rho * u;
    G1[1] = p + rho * u * u;
    G1[2] = rho * u * v;
    G1[3] = p * u + rho * u * E;
    G2[0] = rho * v;
    G2[1] = rho * v * u;
    G2[2] = p + rho * v * v;
    G2[3] = p * v + rho * v * E;
}

// Flux vectors of the conservation law being relaxed.  Gy is untouched in 1D.
template <class T>
void flux(const Problem& P, const T* U, T* Gx, T* Gy) {
    if (P.flux == FLUX_LINEAR) {  // scalar test mode: g1 = cx u, g2 = cy u
        Gx[0] = P.adv_x * U[0];
        if (ndim(P.model) == 2) Gy[0] = P.adv_y * U[0];
        return;
    }
    if (P.flux == FLUX_QUADRATIC) {  // g(u) = a u + b u^2/2 per direction
        const T& u = U[0];
        Gx[0] = P.q[0] * u + P.q[1] * (0.5 * (u * u));
        if (ndim(P.model) == 2) Gy[0] = P.q[2] * u + P.q[3] * (0.5 * (u * u));
        return;
    }
    if (ndim(P.model) == 1)
        euler_flux_1d(U, P.gamma, Gx);
    else
        euler_flux_2d(U, P.gamma, Gx, Gy);
}

// Pressure of an Euler state, from E = p/(rho(gamma-1)) + |u|^2/2.
template <class T>
T pressure(const Problem& P, const T* U) {
    T rho = U[0];
    if (ndim(P.model) == 1) {
        T u = U[1] / rho, E = U[2] / rho;
        return (P.gamma - 1.0) * rho * (E - 0.5 * (u * u));
    }
    T u = U[1] / rho, v = U[2] / rho, E = U[3] / rho;
    return (P.gamma - 1.0) * rho * (E - 0.5 * (u * u + v * v));
}

// Local bound on the wave speeds.
//  1D: lambda = max(|u - a|, |u|, |u + a|)        (Sec. II.C, Jin-Xin choice)
//  2D: lambda = max(|u+v|, |u+v +- sqrt(2) a|, |u-v|, |u-v -+ sqrt(2) a|)
//      (Sec. II.D, Bouchut's condition; "sqrt(2a)" read as sqrt(2)*a)
//  linear advection: |c| in 1D, |cx| + |cy| in 2D (the sub-characteristic
//  bound for the scalar D1Q2 model, Sec. II.A, and its D2Q4 analogue).
//  quadratic scalar law: |g'(u)| in 1D (Sec. II.A sub-characteristic
//  condition); in 2D the largest |s_x g1'(u) + s_y g2'(u)| over the four
//  diagonal directions, i.e. |g1'| + |g2'| (the D2Q4 equilibria are then
//  non-decreasing in u, the scalar form of the Sec. II.D condition).
inline double local_lambda(const Problem& P, const double* U) {
    if (P.flux == FLUX_LINEAR)
        return ndim(P.model) == 1 ? std::fabs(P.adv_x)
                                  : std::fabs(P.adv_x) + std::fabs(P.adv_y);
    if (P.flux == FLUX_QUADRATIC) {
        double d1 = P.q[0] + P.q[1] * U[0];
        if (ndim(P.model) == 1) return std::fabs(d1);
        double d2 = P.q[2] + P.q[3] * U[0];
        double m = 0.0;
        for (int sxv = -1; sxv <= 1; sxv += 2)
            for (int syv = -1; syv <= 1; syv += 2) m = std::max(m, std::fabs(sxv * d1 + syv * d2));
        return m;
    }
    double rho = U[0];
    double p = pressure(P, U);
    double a = std::sqrt(P.gamma * p / rho);
    if (ndim(P.model) == 1) {
        double u = U[1] / rho;
        return std::max(std::max(std::fabs(u - a), std::fabs(u)), std::fabs(u + a));
    }
    double u = U[1] / rho, v = U[2] / rho;
    double r2a = std::sqrt(2.0) * a;
    double cands[6] = {std::fabs(u + v), std::fabs(u + v + r2a), std::fabs(u + v - r2a),
                       std::fabs(u - v), std::fabs(u - v - r2a), std::fabs(u - v + r2a)};
    double m = cands[0];
    for (int j = 1; j < 6; ++j) m = std::max(m, cands[j]);
    return m;
}

// Equilibria of the diagonal relaxation system for one conserved component.
//  D1Q2: f1 = U/2 - G/(2 lambda),  f2 = U/2 + G/(2 lambda)
//  D1Q3: f1 = U/3 - G/(2 lambda),  f2 = U/3,  f3 = U/3 + G/(2 lambda)
//  D2Q4: f_i = U/4 + s_ix G1/(4 lambda) + s_iy G2/(4 lambda)
// (Sec. II.A "equilibrium", Sec. II.C D1Q2/D1Q3 Euler equilibria, Sec. II.D.)
template <class T>
T equilibrium(int model, int i, const T& U, const T& Gx, const T& Gy, double lam) {
    if (model == D1Q2) return U / 2.0 + sx(model, i) * (Gx / (2.0 * lam));
    if (model == D1Q3) return U / 3.0 + sx(model, i) * (Gx / (2.0 * lam));
    return U / 4.0 + sx(model, i) * (Gx / (4.0 * lam)) + sy(model, i) * (Gy / (4.0 * lam));
}

// Is an Euler state admissible (rho > 0, p > 0, all finite)?
inline bool physical(const Problem& P, const double* U) {
    int K = ncomp(P);
    for (int k = 0; k < K; ++k)
        if (!std::isfinite(U[k])) return false;
    if (scalar_law(P)) return true;
    if (!(U[0] > 0.0)) return false;
    double p = pressure(P, U);
    return p > 0.0 && std::isfinite(p);
}

// ------------------------------------------------------------ solid bodies
// Position j along an axis of n cells, brought onto the grid: wrapped on a
// periodic axis, clamped otherwise.
inline int onto_grid(int j, int n, bool periodic) {
    if (j >= 0 && j < n) return j;
    if (periodic) return ((j % n) + n) % n;
    return j < 0 ? 0 : n - 1;
}

inline bool is_solid_cell(const Problem& P, long c) { return P.solid && P.solid[c] != 0; }

// Is the position (xs, ys), possibly outside the grid, solid?  Everything
// beyond a wall side is; otherwise the mask at the position brought onto the
// grid decides.
inline bool solid_at(const Problem& P, int xs, int ys) {
    if ((ys < 0 && P.side[2] == SIDE_WALL) || (ys >= P.ny && P.side[3] == SIDE_WALL)) return true;
    if ((xs < 0 && P.side[0] == SIDE_WALL) || (xs >= P.nx && P.side[1] == SIDE_WALL)) return true;
    if (!P.solid) return false;
    int x = onto_grid(xs, P.nx, P.side[0] == SIDE_PERIODIC);
    int y = onto_grid(ys, P.ny, P.side[2] == SIDE_PERIODIC);
    return P.solid[(long)y * P.nx + x] != 0;
}

// D2Q4 population whose velocity is that of i with s_x (flipx) and/or s_y
// (flipy) reversed.
inline int flipped(int i, bool flipx, bool flipy) {
    int tx = flipx ? -sx(D2Q4, i) : sx(D2Q4, i);
    int ty = flipy ? -sy(D2Q4, i) : sy(D2Q4, i);
    for (int j = 0; j < 4; ++j)
        if (sx(D2Q4, j) == tx && sy(D2Q4, j) == ty) return j;
    return -1;
}

// How population i of the fluid node (x, y) is found when its pull source
// (x - s_ix, y - s_iy) is solid: the population j of the same node it is
// imaged from, and the kind of image.
enum { IMG_FACE_X, IMG_FACE_Y, IMG_CONCAVE, IMG_TIP };
inline int image_of(const Problem& P, int x, int y, int i, int* kind) {
    bool bx = solid_at(P, x - sx(D2Q4, i), y);
    bool by = solid_at(P, x, y - sy(D2Q4, i));
    if (bx && !by) { *kind = IMG_FACE_X; return flipped(i, true, false); }
    if (by && !bx) { *kind = IMG_FACE_Y; return flipped(i, false, true); }
    *kind = bx ? IMG_CONCAVE : IMG_TIP;
    return flipped(i, true, true);
}

// A mask is admissible when some cell is fluid and every imaged population's
// source population is itself pulled from a non-solid position (bodies and
// gaps at least two cells across).
inline bool mask_admissible(const Problem& P) {
    bool any_fluid = false;
    for (int y = 0; y < P.ny; ++y)
        for (int x = 0; x < P.nx; ++x) {
            if (is_solid_cell(P, (long)y * P.nx + x)) continue;
            any_fluid = true;
            for (int i = 0; i < 4; ++i) {
                if (!solid_at(P, x - sx(D2Q4, i), y - sy(D2Q4, i))) continue;
                int kind;
                int j = image_of(P, x, y, i, &kind);
                if (solid_at(P, x - sx(D2Q4, j), y - sy(D2Q4, j))) return false;
            }
        }
    return any_fluid;
}

// ---------------------------------------------------------- the simulation
template <class T>
struct Sim {
    Problem P;
    int Q, K, D;
    long ncell;
    double dx;
    std::vector<T> f, fs;  // f[(i*K + k)*ncell + y*nx + x]; fs = post-collision
    std::vector<T> U;      // U[k*ncell + cell]

    explicit Sim(const Problem& p) : P(p) {
        Q = nq(P.model);
        K = ncomp(P);
        D = ndim(P.model);
        ncell = (long)P.nx * P.ny;
        dx = (P.x1 - P.x0) / P.nx;
        f.assign((size_t)Q * K * ncell, T(0.0));
        fs.assign((size_t)Q * K * ncell, T(0.0));
        U.assign((size_t)K * ncell, T(0.0));
    }
    T& F(std::vector<T>& a, int i, int k, int x, int y) {
        return a[((size_t)(i * K + k)) * ncell + (size_t)y * P.nx + x];
    }

    // U = sum_i f_i in every cell                      (eq. "moments_system")
    void moments() {
        for (int k = 0; k < K; ++k)
#pragma omp parallel for schedule(static)
            for (long c = 0; c < ncell; ++c) {
                T s = T(0.0);
                for (int i = 0; i < Q; ++i) s = s + f[((size_t)(i * K + k)) * ncell + c];
                U[(size_t)k * ncell + c] = s;
            }
    }

    // Number of prescribed states along side s.
    int side_len(int s) const { return s < 2 ? P.ny : P.nx; }

    double max_local_lambda() {
        double m = 0.0;
#pragma omp parallel reduction(max : m)
        {
            std::vector<double> Uc(K);
#pragma omp for schedule(static)
            for (long c = 0; c < ncell; ++c) {
                if (is_solid_cell(P, c)) continue;
                for (int k = 0; k < K; ++k) Uc[k] = val(U[(size_t)k * ncell + c]);
                m = std::max(m, local_lambda(P, Uc.data()));
            }
        }
        std::vector<double> Uc(K);
        for (int s = 0; s < 4; ++s)  // the ghost cells of Dirichlet sides
            if (P.side[s] == SIDE_DIRICHLET)
                for (int j = 0; j < side_len(s); ++j) {
                    for (int k = 0; k < K; ++k) Uc[k] = P.dir[s][(size_t)k * side_len(s) + j];
                    m = std::max(m, local_lambda(P, Uc.data()));
                }
        return m;
    }

    bool all_physical(long* bad) {
        long first = ncell;  // the first non-physical cell
#pragma omp parallel reduction(min : first)
        {
            std::vector<double> Uc(K);
#pragma omp for schedule(static)
            for (long c = 0; c < ncell; ++c) {
                if (is_solid_cell(P, c)) continue;
                for (int k = 0; k < K; ++k) Uc[k] = val(U[(size_t)k * ncell + c]);
                if (!physical(P, Uc.data())) first = std::min(first, c);
            }
        }
        if (first == ncell) return true;
        if (bad) *bad = first;
        return false;
    }

    // f^0 = f^eq(U0) in every cell (Sec. II.A: the initial data are given to
    // the populations through their equilibria); solid cells hold zeros.
    void init_equilibrium(const T* U0, double lam) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < P.ny; ++y) {
            std::vector<T> Uc(K), Gx(K), Gy(K);
            for (int x = 0; x < P.nx; ++x) {
                long c = (long)y * P.nx + x;
                if (is_solid_cell(P, c)) continue;  // f stays zero
                for (int k = 0; k < K; ++k) Uc[k] = U0[(size_t)k * ncell + c];
                flux(P, Uc.data(), Gx.data(), Gy.data());
                for (int i = 0; i < Q; ++i)
                    for (int k = 0; k < K; ++k)
                        F(f, i, k, x, y) = equilibrium(P.model, i, Uc[k], Gx[k], Gy[k], lam);
            }
        }
    }

    // Collision: f* = (1 - omega) f + omega f^eq(U), with U from moments().
    // (Discrete LBRS update with omega = dt/epsilon, Sec. II.A and II.D.)
    void collide(double lam) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < P.ny; ++y) {
            std::vector<T> Uc(K), Gx(K), Gy(K);
            for (int x = 0; x < P.nx; ++x) {
                long c = (long)y * P.nx + x;
                if (is_solid_cell(P, c)) continue;  // never pulled from
                for (int k = 0; k < K; ++k) Uc[k] = U[(size_t)k * ncell + c];
                flux(P, Uc.data(), Gx.data(), Gy.data());
                for (int i = 0; i < Q; ++i)
                    for (int k = 0; k < K; ++k) {
                        T feq = equilibrium(P.model, i, Uc[k], Gx[k], Gy[k], lam);
                        F(fs, i, k, x, y) = (1.0 - P.omega) * F(f, i, k, x, y) + P.omega * feq;
                    }
            }
        }
    }

    // Source index along one axis for a pull from position j - s.  Returns -1
    // when the source lies beyond a wall (the population is set by reflection).
    int source(int j, int s, int n, int side_lo, int side_hi) {
        int src = j - s;
        if (src >= 0 && src < n) return src;
        int side = src < 0 ? side_lo : side_hi;
        if (side == SIDE_PERIODIC) return (src + n) % n;
        if (side == SIDE_TRANSMISSIVE) return src < 0 ? 0 : n - 1;
        return -1;  // wall
    }

    // Index along one axis into a Dirichlet side's array for a ghost position
    // j: wrapped on a periodic axis, clamped otherwise.
    static int along(int j, int n, int side_lo, int side_hi) {
        if (j >= 0 && j < n) return j;
        int side = j < 0 ? side_lo : side_hi;
        if (side == SIDE_PERIODIC) return ((j % n) + n) % n;
        return j < 0 ? 0 : n - 1;
    }

    // Prescribed state of the ghost cell (xs, ys) if it lies across a
    // Dirichlet side (the y-side first at a corner).
    bool ghost_state(int xs, int ys, double* Ub) {
        if (D == 2 && (ys < 0 || ys >= P.ny)) {
            int s = ys < 0 ? 2 : 3;
            if (P.side[s] == SIDE_DIRICHLET) {
                int j = along(xs, P.nx, P.side[0], P.side[1]);
                for (int k = 0; k < K; ++k) Ub[k] = P.dir[s][(size_t)k * P.nx + j];
                return true;
            }
        }
        if (xs < 0 || xs >= P.nx) {
            int s = xs < 0 ? 0 : 1;
            if (P.side[s] == SIDE_DIRICHLET) {
                int j = D == 2 ? along(ys, P.ny, P.side[2], P.side[3]) : 0;
                for (int k = 0; k < K; ++k) Ub[k] = P.dir[s][(size_t)k * P.ny + j];
                return true;
            }
        }
        return false;
    }

    // Streaming with exact hopping: f_i(x + s_i, t + dt) = f*_i(x, t)   (Sec. II.A)
    // written as a pull f_i^{n+1}(x) = f*_i(x - s_i), then the walls.  A pull
    // from a Dirichlet ghost cell takes its equilibrium at lattice speed lam.
    void stream(double lam) {
        if (P.solid) {
            stream_with_bodies(lam);
            return;
        }
        for (int i = 0; i < Q; ++i)
#pragma omp parallel for schedule(static)
            for (int y = 0; y < P.ny; ++y) {
                std::vector<double> Ub(K), Gx(K), Gy(K, 0.0);
                for (int x = 0; x < P.nx; ++x) {
                    int xsrc = x - sx(P.model, i), ysrc = D == 2 ? y - sy(P.model, i) : 0;
                    if (ghost_state(xsrc, ysrc, Ub.data())) {
                        flux(P, Ub.data(), Gx.data(), Gy.data());
                        for (int k = 0; k < K; ++k)
                            F(f, i, k, x, y) = T(equilibrium(P.model, i, Ub[k], Gx[k], Gy[k], lam));
                        continue;
                    }
                    int xs = source(x, sx(P.model, i), P.nx, P.side[0], P.side[1]);
                    int ys = D == 2 ? source(y, sy(P.model, i), P.ny, P.side[2], P.side[3]) : 0;
                    for (int k = 0; k < K; ++k)
                        F(f, i, k, x, y) = (xs < 0 || ys < 0) ? T(0.0) : F(fs, i, k, xs, ys);
                }
            }
        apply_walls();
    }

    // Streaming with solid bodies (and the wall sides folded into them):
    // first every population whose source position is not solid is pulled as
    // in stream(); then each population whose source is solid is set from
    // the node's own pulled populations by the specular image of its kind.
    void stream_with_bodies(double lam) {
        const int kx = 1, ky = 2;  // momentum components
#pragma omp parallel for schedule(static)
        for (int y = 0; y < P.ny; ++y) {
            std::vector<double> Ub(K), Gx(K), Gy(K, 0.0);
            for (int x = 0; x < P.nx; ++x) {
                bool solid = is_solid_cell(P, (long)y * P.nx + x);
                for (int i = 0; i < 4; ++i) {
                    int xsrc = x - sx(P.model, i), ysrc = y - sy(P.model, i);
                    if (solid || solid_at(P, xsrc, ysrc)) {
                        for (int k = 0; k < K; ++k) F(f, i, k, x, y) = T(0.0);
                        continue;
                    }
                    if (ghost_state(xsrc, ysrc, Ub.data())) {
                        flux(P, Ub.data(), Gx.data(), Gy.data());
                        for (int k = 0; k < K; ++k)
                            F(f, i, k, x, y) = T(equilibrium(P.model, i, Ub[k], Gx[k], Gy[k], lam));
                        continue;
                    }
                    int xs = source(x, sx(P.model, i), P.nx, P.side[0], P.side[1]);
                    int ys = source(y, sy(P.model, i), P.ny, P.side[2], P.side[3]);
                    for (int k = 0; k < K; ++k) F(f, i, k, x, y) = F(fs, i, k, xs, ys);
                }
            }
        }
#pragma omp parallel for schedule(static)
        for (int y = 0; y < P.ny; ++y)
            for (int x = 0; x < P.nx; ++x) {
                if (is_solid_cell(P, (long)y * P.nx + x)) continue;
                for (int i = 0; i < 4; ++i) {
                    if (!solid_at(P, x - sx(P.model, i), y - sy(P.model, i))) continue;
                    int kind;
                    int j = image_of(P, x, y, i, &kind);
                    for (int k = 0; k < K; ++k) {
                        T v = F(f, j, k, x, y);
                        if (kind == IMG_FACE_X && k == kx) v = -v;
                        if (kind == IMG_FACE_Y && k == ky) v = -v;
                        if (kind == IMG_CONCAVE && (k == kx || k == ky)) v = -v;
                        if (kind == IMG_TIP && (k == kx || k == ky)) {
                            // reflection about the bisector normal n ~ s_i:
                            // (m_x, m_y) -> -s_ix s_iy (m_y, m_x)
                            double c = -double(sx(P.model, i) * sy(P.model, i));
                            v = c * F(f, j, k == kx ? ky : kx, x, y);
                        }
                        F(f, i, k, x, y) = v;
                    }
                }
            }
    }

    // Specular reflection at a wall node row/column (Sec. II.E).  The paper
    // writes the upper wall: f1 = f4 and f2 = f3 for the mass, x-momentum and
    // energy components, f1 = -f4 and f2 = -f3 for the y-momentum component.
    // The other sides follow by the same mirror rule: the incoming population
    // takes the value of its mirror image with the normal momentum negated.
    void apply_walls() {
        if (D != 2) return;
        // component index of the momentum normal to a y-wall / an x-wall
        const int ky = 2, kx = 1;
        if (P.side[3] == SIDE_WALL) {  // upper wall, row ny-1: f1 <- f4, f2 <- f3
            int y = P.ny - 1;
            for (int x = 0; x < P.nx; ++x)
                for (int k = 0; k < K; ++k) {
                    double sgn = (k == ky) ? -1.0 : 1.0;
                    F(f, 0, k, x, y) = sgn * F(f, 3, k, x, y);
                    F(f, 1, k, x, y) = sgn * F(f, 2, k, x, y);
                }
        }
        if (P.side[2] == SIDE_WALL) {  // lower wall, row 0: f4 <- f1, f3 <- f2
            int y = 0;
            for (int x = 0; x < P.nx; ++x)
                for (int k = 0; k < K; ++k) {
                    double sgn = (k == ky) ? -1.0 : 1.0;
                    F(f, 3, k, x, y) = sgn * F(f, 0, k, x, y);
                    F(f, 2, k, x, y) = sgn * F(f, 1, k, x, y);
                }
        }
        if (P.side[0] == SIDE_WALL) {  // left wall, column 0: f2 <- f1, f3 <- f4
            int x = 0;
            for (int y = 0; y < P.ny; ++y)
                for (int k = 0; k < K; ++k) {
                    double sgn = (k == kx) ? -1.0 : 1.0;
                    F(f, 1, k, x, y) = sgn * F(f, 0, k, x, y);
                    F(f, 2, k, x, y) = sgn * F(f, 3, k, x, y);
                }
        }
        if (P.side[1] == SIDE_WALL) {  // right wall, column nx-1: f1 <- f2, f4 <- f3
            int x = P.nx - 1;
            for (int y = 0; y < P.ny; ++y)
                for (int k = 0; k < K; ++k) {
                    double sgn = (k == kx) ? -1.0 : 1.0;
                    F(f, 0, k, x, y) = sgn * F(f, 1, k, x, y);
                    F(f, 3, k, x, y) = sgn * F(f, 2, k, x, y);
                }
        }
    }
};

// Are the prescribed states of every Dirichlet side admissible?  (Checked with
// the initial state: a bad one is reported as non-physical at step 0.)
bool dirichlet_admissible(const Problem& P) {
    int K = ncomp(P);
    std::vector<double> Ub(K);
    for (int s = 0; s < 4; ++s) {
        if (P.side[s] != SIDE_DIRICHLET) continue;
        int n = s < 2 ? P.ny : P.nx;
        for (int j = 0; j < n; ++j) {
            for (int k = 0; k < K; ++k) Ub[k] = P.dir[s][(size_t)k * n + j];
            if (!physical(P, Ub.data())) return false;
        }
    }
    return true;
}

// Largest admissible CFL number of each model.  The lattice speed is
// lambda*/cfl; the equilibria are monotone in U (Bouchut's condition,
// Sec. II.D) when every eigenvalue of df_i^eq/dU is >= 0.  D1Q2:
// 1/2 - mu/(2 lambda) >= 0, i.e. lambda >= |mu| (cfl <= 1).  D1Q3 (the Sec. II.C
// equilibria U/3 -+ G/(2 lambda)): 1/3 - mu/(2 lambda) >= 0, i.e.
// lambda >= 1.5 |mu| (cfl <= 2/3).  D2Q4: 1/4 - (s . mu)/(4 lambda) >= 0 with
// the bound of Sec. II.D (cfl <= 1).  mu runs over the eigenvalues of the flux
// Jacobian (g'(u) for a scalar law).
inline double cfl_max(int model) { return model == D1Q3 ? 2.0 / 3.0 : 1.0; }

int validate(const Problem& P) {
    if (P.model < D1Q2 || P.model > D2Q4) return ST_INVAL;
    if (P.flux < FLUX_EULER || P.flux > FLUX_QUADRATIC) return ST_INVAL;
    if (scalar_law(P) && (P.side[0] == SIDE_WALL || P.side[1] == SIDE_WALL ||
                          P.side[2] == SIDE_WALL || P.side[3] == SIDE_WALL))
        return ST_INVAL;  // specular walls are defined for the Euler equations
    if (P.nx < 3 || P.ny < 1) return ST_INVAL;
    if (ndim(P.model) == 1 && P.ny != 1) return ST_INVAL;
    if (ndim(P.model) == 2 && P.ny < 3) return ST_INVAL;
    if (!(P.omega > 0.0 && P.omega < 2.0)) return ST_INVAL;  // Chapman-Enskog, Sec. II.B
    if (!(P.x1 > P.x0)) return ST_INVAL;
    if (ndim(P.model) == 2) {
        // diagonal hops need dx == dy
        double dx = (P.x1 - P.x0) / P.nx, dy = (P.y1 - P.y0) / P.ny;
        if (!(std::fabs(dx - dy) <= 1e-12 * dx)) return ST_INVAL;
    }
    for (int s = 0; s < 4; ++s)
        if (P.side[s] < 0 || P.side[s] > 3) return ST_INVAL;
    for (int s = 0; s < 4; ++s)
        if (P.side[s] == SIDE_DIRICHLET && (!P.dir[s] || (ndim(P.model) == 1 && s >= 2)))
            return ST_INVAL;
    if ((P.side[0] == SIDE_PERIODIC) != (P.side[1] == SIDE_PERIODIC)) return ST_INVAL;
    if (ndim(P.model) == 2 && (P.side[2] == SIDE_PERIODIC) != (P.side[3] == SIDE_PERIODIC))
        return ST_INVAL;
    if (ndim(P.model) == 1 && (P.side[0] == SIDE_WALL || P.side[1] == SIDE_WALL)) return ST_INVAL;
    if (ndim(P.model) == 2 && !P.solid) {  // walls meeting at a corner need the body rules
        bool xw = P.side[0] == SIDE_WALL || P.side[1] == SIDE_WALL;
        bool yw = P.side[2] == SIDE_WALL || P.side[3] == SIDE_WALL;
        if (xw && yw) return ST_INVAL;
    }
    if (P.solid && (P.model != D2Q4 || scalar_law(P) || !mask_admissible(P))) return ST_INVAL;
    if (P.lam_mode < LAM_PER_STEP || P.lam_mode > LAM_USER) return ST_INVAL;
    if (P.lam_mode == LAM_USER && !(P.lam_user > 0.0)) return ST_INVAL;
    if (P.lam_mode != LAM_USER && !(P.cfl > 0.0 && P.cfl <= cfl_max(P.model))) return ST_INVAL;
    return ST_OK;
}

}  // namespace orc

using namespace orc;

extern "C" {

// Threads of the cell loops: a build with OpenMP (the timing build of the CPU
// baseline) runs every loop over cells in parallel, the default build is
// serial.  n > 0 sets the count; returns the count in use (1 when serial).
int orc_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

// Flux vectors of one state.  Gx, Gy: K values each (Gy unused in 1D).
void orc_flux(const Problem* P, const double* U, double* Gx, double* Gy) {
    flux(*P, U, Gx, Gy);
}

// Local wave-speed bound of one state.
double orc_local_lambda(const Problem* P, const double* U) { return local_lambda(*P, U); }

// Equilibria of one state at lattice speed lam.  feq: Q*K values, [i][k].
void orc_equilibria(const Problem* P, const double* U, double lam, double* feq) {
    int Q = nq(P->model), K = ncomp(*P);
    std::vector<double> Gx(K), Gy(K, 0.0);
    flux(*P, U, Gx.data(), Gy.data());
    for (int i = 0; i < Q; ++i)
        for (int k = 0; k < K; ++k)
            feq[i * K + k] = equilibrium(P->model, i, U[k], Gx[k], Gy[k], lam);
}

// Primitive (rho, u, [v,] p) -> conserved (rho, rho u, [rho v,] rho E) per cell,
// SoA planes of ncell values.  E = p/(rho(gamma-1)) + |u|^2/2.
void orc_prim_to_cons(const Problem* P, const double* W, double* U) {
    long n = (long)P->nx * P->ny;
    int K = ncomp(*P);
    if (scalar_law(*P)) {
        std::memcpy(U, W, sizeof(double) * n);
        return;
    }
    for (long c = 0; c < n; ++c) {
        double rho = W[c];
        if (K == 3) {
            double u = W[n + c], p = W[2 * n + c];
            double E = p / (rho * (P->gamma - 1.0)) + 0.5 * (u * u);
            U[c] = rho;
            U[n + c] = rho * u;
            U[2 * n + c] = rho * E;
        } else {
            double u = W[n + c], v = W[2 * n + c], p = W[3 * n + c];
            double E = p / (rho * (P->gamma - 1.0)) + 0.5 * (u * u + v * v);
            U[c] = rho;
            U[n + c] = rho * u;
            U[2 * n + c] = rho * v;
            U[3 * n + c] = rho * E;
        }
    }
}

// Lattice speed the run starts from: lambda*(U0)/cfl (per-step and frozen
// modes) or the user's value.  Returns <= 0 on error.
double orc_initial_lattice_speed(const Problem* P, const double* U0) {
    if (validate(*P) != ST_OK) return -1.0;
    if (P->lam_mode == LAM_USER) return P->lam_user;
    Sim<double> S(*P);
    std::memcpy(S.U.data(), U0, sizeof(double) * S.K * S.ncell);
    if (!S.all_physical(nullptr) || !dirichlet_admissible(*P)) return -1.0;
    return S.max_local_lambda() / P->cfl;
}

// Run the scheme from U0 (SoA [K][ny][nx]) until t >= t_end or max_steps steps.
// Outputs (each optional, may be null):
//   U_out  [K][ny][nx]  moments of the final populations
//   f_out  [Q][K][ny][nx] final populations
//   dt_seq, lam_seq [max_steps]: dt_n and the lattice speed used at step n
//   nsteps, t_final, fail_step (step whose result was non-physical, or -1)
// Returns ST_OK, ST_INVAL or ST_NONPHYSICAL.
int orc_run(const Problem* Pp, const double* U0, double t_end, long max_steps, double* U_out,
            double* f_out, double* dt_seq, double* lam_seq, long* nsteps, double* t_final,
            long* fail_step) {
    const Problem& P = *Pp;
    if (nsteps) *nsteps = 0;
    if (t_final) *t_final = 0.0;
    if (fail_step) *fail_step = -1;
    int st = validate(P);
    if (st != ST_OK) return st;
    Sim<double> S(P);
    std::memcpy(S.U.data(), U0, sizeof(double) * S.K * S.ncell);
    if (!S.all_physical(nullptr) || !dirichlet_admissible(P)) {
        if (fail_step) *fail_step = 0;
        return ST_NONPHYSICAL;
    }
    double lam_fixed = P.lam_mode == LAM_USER ? P.lam_user : S.max_local_lambda() / P.cfl;
    S.init_equilibrium(U0, lam_fixed);

    double t = 0.0;
    long n = 0;
    int status = ST_OK;
    while (n < max_steps && t < t_end) {
        S.moments();
        double dt, lam;
        if (P.lam_mode == LAM_PER_STEP) {
            // Global bound of step n from U^n, then exact hopping lam*dt = dx,
            // with the last step clipped to land on t_end.
            double lam_star = S.max_local_lambda();
            dt = P.cfl * S.dx / lam_star;
            double rem = t_end - t;
            bool last = false;
            if (dt >= rem) {
                dt = rem;
                last = true;
            }
            lam = S.dx / dt;
            t = last ? t_end : t + dt;
        } else {
            lam = lam_fixed;
            dt = S.dx / lam;
            t = t + dt;
        }
        if (dt_seq) dt_seq[n] = dt;
        if (lam_seq) lam_seq[n] = lam;
        S.collide(lam);
        S.stream(lam);
        ++n;
        S.moments();
        if (!S.all_physical(nullptr)) {
            status = ST_NONPHYSICAL;
            if (fail_step) *fail_step = n;
            break;
        }
    }
    S.moments();
    if (U_out) std::memcpy(U_out, S.U.data(), sizeof(double) * S.K * S.ncell);
    if (f_out) std::memcpy(f_out, S.f.data(), sizeof(double) * S.Q * S.K * S.ncell);
    if (nsteps) *nsteps = n;
    if (t_final) *t_final = t;
    return status;
}

// One step at a fixed lattice speed lam, from given populations f (no lambda
// reduction, no time bookkeeping), with its tangent: (f, df) -> (f', df').
// df / df_out may be null for a plain step.
int orc_step_fixed(const Problem* Pp, const double* f, const double* df, double lam,
                   double* f_out, double* df_out) {
    const Problem& P = *Pp;
    int st = validate(P);
    if (st != ST_OK) return st;
    Sim<Dual> S(P);
    size_t nf = (size_t)S.Q * S.K * S.ncell;
    for (size_t j = 0; j < nf; ++j) S.f[j] = Dual(f[j], df ? df[j] : 0.0);
    S.moments();
    S.collide(lam);
    S.stream(lam);
    for (size_t j = 0; j < nf; ++j) {
        f_out[j] = S.f[j].v;
        if (df_out) df_out[j] = S.f[j].d;
    }
    return ST_OK;
}

// Tangent of the initialisation f^0 = f^eq(U0) at lattice speed lam along dU0
// (both [K][ny][nx]); writes f0 and df0 ([Q][K][ny][nx]).
int orc_init_tangent(const Problem* Pp, const double* U0, const double* dU0, double lam,
                     double* f0, double* df0) {
    const Problem& P = *Pp;
    int st = validate(P);
    if (st != ST_OK) return st;
    Sim<Dual> S(P);
    std::vector<Dual> U((size_t)S.K * S.ncell);
    for (size_t j = 0; j < U.size(); ++j) U[j] = Dual(U0[j], dU0[j]);
    S.init_equilibrium(U.data(), lam);
    for (size_t j = 0; j < S.f.size(); ++j) {
        f0[j] = S.f[j].v;
        df0[j] = S.f[j].d;
    }
    return ST_OK;
}

// Directional derivative of a whole fixed-speed run with respect to the initial
// primitive state: W0 + eps*dW0 -> (U(T), dU(T)/deps), after nsteps steps at the
// lattice speed lam (frozen or user mode).  W0/dW0: SoA primitive planes.
// If isentropic != 0 the pressure plane is ignored and p = rho^gamma/gamma.
int orc_run_tangent(const Problem* Pp, const double* W0, const double* dW0, int isentropic,
                    double lam, long nsteps, double* U_out, double* dU_out) {
    const Problem& P = *Pp;
    int st = validate(P);
    if (st != ST_OK) return st;
    if (P.flux != FLUX_EULER) return ST_INVAL;
    Sim<Dual> S(P);
    long n = S.ncell;
    std::vector<Dual> U0((size_t)S.K * n);
    for (long c = 0; c < n; ++c) {
        // conserved variables of the primitive state, differentiated
        Dual rho(W0[c], dW0[c]);
        if (S.K == 3) {
            Dual u(W0[n + c], dW0[n + c]);
            Dual p = isentropic ? pow(rho, P.gamma) / P.gamma : Dual(W0[2 * n + c], dW0[2 * n + c]);
            Dual E = p / (rho * (P.gamma - 1.0)) + 0.5 * (u * u);
            U0[c] = rho;
            U0[n + c] = rho * u;
            U0[2 * n + c] = rho * E;
        } else {
            Dual u(W0[n + c], dW0[n + c]), v(W0[2 * n + c], dW0[2 * n + c]);
            Dual p = isentropic ? pow(rho, P.gamma) / P.gamma : Dual(W0[3 * n + c], dW0[3 * n + c]);
            Dual E = p / (rho * (P.gamma - 1.0)) + 0.5 * (u * u + v * v);
            U0[c] = rho;
            U0[n + c] = rho * u;
            U0[2 * n + c] = rho * v;
            U0[3 * n + c] = rho * E;
        }
    }
    S.init_equilibrium(U0.data(), lam);
    for (long s = 0; s < nsteps; ++s) {
        S.moments();
        S.collide(lam);
        S.stream(lam);
    }
    S.moments();
    for (size_t j = 0; j < (size_t)S.K * n; ++j) {
        U_out[j] = S.U[j].v;
        dU_out[j] = S.U[j].d;
    }
    return ST_OK;
}

}  // extern "C"
