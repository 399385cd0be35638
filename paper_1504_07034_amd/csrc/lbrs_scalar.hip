// LBRS for scalar conservation laws u_t + g1(u)_x [+ g2(u)_y] = 0 (gfx950, FP64).
//
// The relaxation scheme the paper builds first for a scalar law (Sec. II.A:
// the Jin-Xin system read as the two-velocity D1Q2 model; the three-velocity
// form by the same moment conditions) and in two dimensions (Sec. II.D, the
// isotropic D2Q4 model), for the quadratic fluxes
//   g1(u) = c0 u + c1 u^2/2,   g2(u) = c2 u + c3 u^2/2,
// which hold Burgers' equation (c = (0, 1)), the 2D Burgers law of the
// Sec. III test cases (c = (0, 1, 1, 0)) and linear advection (c1 = c3 = 0).
// Equilibria match the moments u = sum f_i, g = sum lambda_i f_i:
//   D1Q2  f = u/2 -+ g/(2 lambda)            D1Q3  f = u/3 -+ g/(2 lambda), u/3
//   D2Q4  f_i = u/4 + (s_ix g1 + s_iy g2)/(4 lambda).
// Local bound: |g'(u)| in 1D (the sub-characteristic condition of Sec. II.A);
// |g1'(u)| + |g2'(u)| in 2D, the largest |s . g'(u)| over the four diagonals,
// which keeps every D2Q4 equilibrium non-decreasing in u.
//
// The 2D kernel marches rows of strips like the Euler step (one HBM pass per
// step: 4 populations in, 4 out, DPP lane shifts for the x hops, a two-row
// register pipeline for the y hops, the next bound reduced from the new u;
// the waves of a workgroup march adjacent strips of one segment in lockstep;
// a ring of three row buffers keeps two rows of loads in flight);
// the 1D kernel stages a 1024-cell tile of post-collision values in LDS.  Side
// conditions: transmissive, periodic and DIRICHLET (ghost cells hold the
// prescribed u in equilibrium at the step's lattice speed; the y-side decides
// at a corner).  The time-state and reduction-slot protocol is the Euler
// step's.
#include "lbrs_launch.hpp"
#include "lbrs_rowops.hpp"

namespace lbrs {

static constexpr int STILE1D = 1024;

__device__ inline double sflux(const double c[4], int axis, double u) {
    return c[2 * axis] * u + c[2 * axis + 1] * (0.5 * (u * u));
}

// Local bound of the state u (see the header comment).
__device__ inline double sbound(const double c[4], bool two_d, double u) {
    const double d1 = fabs(c[0] + c[1] * u);
    if (!two_d) return d1;
    return d1 + fabs(c[2] + c[3] * u);
}

// D2Q4: post-collision values (1-omega) f + omega f^eq(u), folded like the
// Euler collision with a = (g1 + g2)/(4 lambda), b = (g1 - g2)/(4 lambda).
__device__ inline void scalar_collide_d2q4(const double f[4], double u, const double c[4],
                                           double c4lam, double omega, double fs[4]) {
    const double g1 = sflux(c, 0, u), g2 = sflux(c, 1, u);
    const double q = 0.25 * u, a = (g1 + g2) * c4lam, b = (g1 - g2) * c4lam;
    const double om1 = 1.0 - omega;
    fs[0] = om1 * f[0] + omega * (q - a);
    fs[1] = om1 * f[1] + omega * (q + b);
    fs[2] = om1 * f[2] + omega * (q + a);
    fs[3] = om1 * f[3] + omega * (q - b);
}
__device__ inline void scalar_eq_d2q4(double u, const double c[4], double c4lam, double fe[4]) {
    const double g1 = sflux(c, 0, u), g2 = sflux(c, 1, u);
    const double q = 0.25 * u, a = (g1 + g2) * c4lam, b = (g1 - g2) * c4lam;
    fe[0] = q - a;
    fe[1] = q + b;
    fe[2] = q + a;
    fe[3] = q - b;
}

// 1D equilibria f^eq(u) for Q = 2 (-, +) or Q = 3 (-, 0, +).
template <int Q>
__device__ inline void scalar_eq_1d(double u, const double c[4], double c2lam, double fe[Q]) {
    const double a = sflux(c, 0, u) * c2lam;
    if (Q == 2) {
        const double q = 0.5 * u;
        fe[0] = q - a;
        fe[Q - 1] = q + a;
    } else {
        const double q = u / 3.0;
        fe[0] = q - a;
        fe[1] = q;
        fe[Q - 1] = q + a;
    }
}

template <int Q>
__device__ inline double scalar_sum(const double f[Q]) {
    return Q == 2 ? f[0] + f[1] : (Q == 3 ? (f[0] + f[1]) + f[2] : (f[0] + f[2]) + (f[1] + f[3]));
}

// ------------------------------------------------------------------ 2D step
template <int WPB>
__global__ __launch_bounds__(64 * WPB) void scalar2d_step(ScalarArgs a) {
    constexpr int NB = 3;
    const LaunchSlots ls = slots_for(a.launch);
    DevState* st = a.st;
    const StepCtl c = step_control(st, ls, a.lam_mode, a.dx, a.cfl, a.t_end);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_state(st, ls, c);
    if (!c.active) return;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double* __restrict__ fin = c.cur ? a.f1 : a.f0;
    double* __restrict__ fout = c.cur ? a.f0 : a.f1;
    const double c4lam = 1.0 / (4.0 * c.lam), omega = a.omega;
    const int nx = a.nx, ny = a.ny;
    const long long ps = a.ps, rs = a.rs;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    const int row_bytes = nx * 8;
    double lmax = 0.0;
    bool bad = false;
    const int total_waves = gridDim.x * WPB;
    for (int tile = xcd_remap(blockIdx.x, gridDim.x) * WPB + wave; tile < a.ntiles;
         tile += total_waves) {
        const int strip = tile % a.nstrips, seg = tile / a.nstrips;
        const int y0 = (int)(((long long)seg * ny) / a.nseg);
        const int y1 = (int)(((long long)(seg + 1) * ny) / a.nseg);
        const int x = strip * a.strip - 1 + lane;
        const int xl = map_index(x, nx, px);
        const bool out_lane = lane >= 1 && lane <= a.strip && x < nx;
        const int voff = out_lane ? x * 8 : 0x7fffffff;
        const bool ghost_lane = (x < 0 && a.bc[0] == BC_DIRICHLET) ||
                                (x >= nx && a.bc[1] == BC_DIRICHLET);

        // post-collision values of row j (Dirichlet ghosts replaced), hopped
        double s1, s2, n3, n4;
        auto row = [&](int j, const double fr[4]) {
            const double u = scalar_sum<4>(fr);
            double fs[4];
            scalar_collide_d2q4(fr, u, a.sc, c4lam, omega, fs);
            const bool ghost_row = (j < 0 && a.bc[2] == BC_DIRICHLET) ||
                                   (j >= ny && a.bc[3] == BC_DIRICHLET);
            if (ghost_row || ghost_lane) {
                const double ub = ghost_row ? (j < 0 ? a.dir[2] : a.dir[3])[xl]
                                            : (x < 0 ? a.dir[0] : a.dir[1])[map_index(j, ny, py)];
                scalar_eq_d2q4(ub, a.sc, c4lam, fs);
            }
            s1 = lane_from_right(fs[0]);
            s2 = lane_from_left(fs[1]);
            n3 = lane_from_left(fs[2]);
            n4 = lane_from_right(fs[3]);
        };
        auto load = [&](double v[4], int j) {
            const long long off = (long long)map_index(j, ny, py) * rs + xl;
#pragma unroll
            for (int p = 0; p < 4; ++p) v[p] = fin[p * ps + off];
        };

        // output row r-1 from row r (populations fr): pops 1, 2 hop down from
        // row r, pops 3, 4 were produced two rows earlier
        double A3, A4, B3, B4;
        auto emit = [&](int r, const double fr[4]) {
            // lockstep with the workgroup's neighbouring strips (same segment,
            // same trip count): the cache lines two strips share are written
            // together
            if (WPB > 1) __builtin_amdgcn_s_barrier();
            row(r, fr);
            const double go[4] = {s1, s2, B3, B4};
            double* orow = fout + (long long)(r - 1) * rs;
#pragma unroll
            for (int p = 0; p < 4; ++p) store_row(orow + p * ps, row_bytes, voff, go[p]);
            const double un = scalar_sum<4>(go);
            bad |= out_lane && !isfinite(un);
            lmax = fmax(lmax, out_lane ? sbound(a.sc, true, un) : 0.0);
            B3 = A3;
            B4 = A4;
            A3 = n3;
            A4 = n4;
        };

        // prologue: rows y0-1 and y0 fill the pipeline; rows y0+1 ..
        // y0+NB-1 are prefetched into a ring of NB row buffers, so that NB-1
        // rows of loads stay in flight while a row is processed
        double buf[NB][4];
        load(buf[0], y0 - 1);
        load(buf[1], y0);
        row(y0 - 1, buf[0]);
        A3 = n3;
        A4 = n4;
        row(y0, buf[1]);
        B3 = A3;
        B4 = A4;
        A3 = n3;
        A4 = n4;
#pragma unroll
        for (int b = 0; b < NB - 1; ++b) load(buf[b], y0 + 1 + b);
        for (int r = y0 + 1; r <= y1; r += NB) {
            // buffer b holds row r + b (b < NB-1); buffer NB-1 is free
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (r + u > y1) break;
                load(buf[(u + NB - 1) % NB], r + u + NB - 1);
                emit(r + u, buf[u]);
            }
        }
    }
    if (a.lam_mode == LAM_PER_STEP) {
        const double wm = wave_max(lmax);
        if (lane == 0) publish_max(&st->lam[ls.la], wm);
    }
    if (__any(bad) && lane == 0) publish_bad(st, ls, c.n + 1);
}

// ------------------------------------------------------------------ 1D step
// A 256-lane workgroup owns STILE1D = 1024 output cells: the post-collision
// values of those cells and of one halo cell on each side go to LDS (lane t
// forms entries t, t + 256, ...), then every output cell pulls its streamed
// values from its neighbours' entries.
template <int Q, bool BLOCKED>
__global__ __launch_bounds__(256) void scalar1d_step(ScalarArgs a) {
    constexpr int E = STILE1D + 2;  // LDS entry e holds cell x0 - 1 + e
    __shared__ double fsl[Q][E];
    const LaunchSlots ls = slots_for(a.launch);
    DevState* st = a.st;
    const StepCtl c = step_control(st, ls, a.lam_mode, a.dx, a.cfl, a.t_end);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_state(st, ls, c);
    if (!c.active) return;

    const int t = threadIdx.x;
    const int nx = a.nx;
    const int x0 = blockIdx.x * STILE1D;
    const bool periodic = a.bc[0] == BC_PERIODIC;
    const double* __restrict__ fin = c.cur ? a.f1 : a.f0;
    double* __restrict__ fout = c.cur ? a.f0 : a.f1;
    const double c2lam = 1.0 / (2.0 * c.lam), om1 = 1.0 - a.omega;

    constexpr int PASSES = STILE1D / 256 + 1;  // the last pass covers the two halo entries
#pragma unroll
    for (int k = 0; k < PASSES; ++k) {
        const int e = t + 256 * k;
        if (k == PASSES - 1 && e >= E) break;
        const int x = x0 - 1 + e;
        const int xl = map_index(x, nx, periodic);
        double f[Q], fe[Q];
#pragma unroll
        for (int p = 0; p < Q; ++p) f[p] = fin[ofs1d(BLOCKED, a.ps, a.rs, p, xl)];
        const bool ghost = (x < 0 && a.bc[0] == BC_DIRICHLET) || (x >= nx && a.bc[1] == BC_DIRICHLET);
        if (ghost) {
            scalar_eq_1d<Q>((x < 0 ? a.dir[0] : a.dir[1])[0], a.sc, c2lam, fe);
#pragma unroll
            for (int p = 0; p < Q; ++p) fsl[p][e] = fe[p];
        } else {
            scalar_eq_1d<Q>(scalar_sum<Q>(f), a.sc, c2lam, fe);
#pragma unroll
            for (int p = 0; p < Q; ++p) fsl[p][e] = om1 * f[p] + a.omega * fe[p];
        }
    }
    __syncthreads();

    double lmax = 0.0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < STILE1D / 256; ++k) {
        const int j = t + 256 * k;
        const int x = x0 + j;
        if (x < nx) {
            double g[Q];
            g[0] = fsl[0][j + 2];           // s = -1: from x + 1
            if (Q == 3) g[1] = fsl[1][j + 1];  // rest
            g[Q - 1] = fsl[Q - 1][j];       // s = +1: from x - 1
#pragma unroll
            for (int p = 0; p < Q; ++p) fout[ofs1d(BLOCKED, a.ps, a.rs, p, x)] = g[p];
            const double un = scalar_sum<Q>(g);
            const bool b = !isfinite(un);
            bad |= b;
            lmax = fmax(lmax, b ? 0.0 : sbound(a.sc, false, un));
        }
    }
    if (a.lam_mode == LAM_PER_STEP) {
        const double wm = wave_max(lmax);
        if ((t & 63) == 0) publish_max(&st->lam[ls.la], wm);
    }
    if (__any(bad) && (t & 63) == 0) publish_bad(st, ls, c.n + 1);
}

// ------------------------------------------------------------ init & output
struct ScalarSides {
    const double* d[4];
};

__device__ inline int nq_model(int model) { return model == D1Q2 ? 2 : (model == D1Q3 ? 3 : 4); }

// Bounds of u0 into the initial accumulator (non-finite values flagged).
__global__ void scalar_bound_u_kernel(CellArgs a, const double* __restrict__ U, DevState* st) {
    const long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    bool bad = false;
    if (cidx < a.plane) {
        const double u = U[cidx];
        bad = !isfinite(u);
        l = bad ? 0.0 : sbound(a.sc, a.model == D2Q4, u);
    }
    const double wm = wave_max(l);
    if ((threadIdx.x & 63) == 0) publish_max(&st->lam_init, wm);
    if (__any(bad) && (threadIdx.x & 63) == 0) {
        atomicOr(&st->bad[0], 1u);
        atomicOr(&st->status, 1u);
        atomicMin(&st->fail_step, 0ull);
    }
}

// Bounds of the prescribed values of the Dirichlet sides (x-low, x-high: ny
// values each; y-low, y-high: nx each) into the initial bound and lam_bc.
__global__ void scalar_dirichlet_bound_kernel(CellArgs a, ScalarSides ds, DevState* st) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nxs = a.ny, nys = a.nx;
    int side = -1;
    long long pos = 0;
    if (j < nxs) { side = 0; pos = j; }
    else if (j < 2 * nxs) { side = 1; pos = j - nxs; }
    else if (j < 2 * nxs + nys) { side = 2; pos = j - 2 * nxs; }
    else if (j < 2 * nxs + 2 * nys) { side = 3; pos = j - 2 * nxs - nys; }
    double l = 0.0;
    bool bad = false;
    if (side >= 0 && ds.d[side]) {
        const double u = ds.d[side][pos];
        bad = !isfinite(u);
        l = bad ? 0.0 : sbound(a.sc, a.model == D2Q4, u);
    }
    const double wm = wave_max(l);
    if ((threadIdx.x & 63) == 0) {
        publish_max(&st->lam_init, wm);
        publish_max(&st->lam_bc, wm);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) {
        atomicOr(&st->bad[0], 1u);
        atomicOr(&st->status, 1u);
        atomicMin(&st->fail_step, 0ull);
    }
}

__device__ inline long long sofs(const CellArgs& a, int p, long long c) { return cell_ofs(a, p, c); }

// f^0 = f^eq(u0) at lambda*(u0)/cfl (or the user's speed); the bound of
// sum f^0 into reduction slot 0; time slot 0.
__global__ void scalar_init_eq_kernel(CellArgs a, const double* __restrict__ U0, double* __restrict__ f,
                                      DevState* st, int lam_mode, double lam_user, double cfl) {
    const long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double lam0 = lam_mode == LAM_USER
                            ? lam_user
                            : __longlong_as_double((long long)st->lam_init) / cfl;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->s[0].t = 0.0;
        st->s[0].n = 0;
        st->s[0].lam_used = lam0;
        st->s[0].cur = 0;
        st->lam_fixed = lam0;
    }
    double l = 0.0;
    if (cidx < a.plane) {
        const double u = U0[cidx];
        double fe[4];
        double un;
        if (a.model == D2Q4) {
            scalar_eq_d2q4(u, a.sc, 1.0 / (4.0 * lam0), fe);
            un = scalar_sum<4>(fe);
        } else if (a.model == D1Q2) {
            scalar_eq_1d<2>(u, a.sc, 1.0 / (2.0 * lam0), fe);
            un = scalar_sum<2>(fe);
        } else {
            scalar_eq_1d<3>(u, a.sc, 1.0 / (2.0 * lam0), fe);
            un = scalar_sum<3>(fe);
        }
        const int Q = nq_model(a.model);
        for (int p = 0; p < Q; ++p) f[sofs(a, p, cidx)] = fe[p];
        l = isfinite(un) ? sbound(a.sc, a.model == D2Q4, un) : 0.0;
    }
    const double wm = wave_max(l);
    if ((threadIdx.x & 63) == 0) publish_max(&st->lam[0], wm);
}

__device__ inline double scalar_u_of(const CellArgs& a, const double* __restrict__ f, long long c) {
    double v[4];
    const int Q = nq_model(a.model);
    for (int p = 0; p < Q; ++p) v[p] = f[sofs(a, p, c)];
    return Q == 4 ? scalar_sum<4>(v) : (Q == 3 ? scalar_sum<3>(v) : scalar_sum<2>(v));
}

// Bound of given populations into reduction slot 0 (after lbrs_set_f).
__global__ void scalar_bound_f_kernel(CellArgs a, const double* __restrict__ f, DevState* st) {
    const long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    bool bad = false;
    if (cidx < a.plane) {
        const double u = scalar_u_of(a, f, cidx);
        bad = !isfinite(u);
        l = bad ? 0.0 : sbound(a.sc, a.model == D2Q4, u);
    }
    const double wm = wave_max(l);
    if ((threadIdx.x & 63) == 0) publish_max(&st->lam[0], wm);
    if (__any(bad) && (threadIdx.x & 63) == 0) {
        atomicOr(&st->bad[0], 1u);
        atomicOr(&st->status, 1u);
    }
}

// u = sum_i f_i of the current populations (slot's buffer) into U [ny][nx].
__global__ void scalar_moments_kernel(CellArgs a, const double* __restrict__ f0,
                                      const double* __restrict__ f1, const DevState* st, int slot,
                                      double* __restrict__ U) {
    const long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cidx >= a.plane) return;
    const double* f = st->s[slot].cur ? f1 : f0;
    U[cidx] = scalar_u_of(a, f, cidx);
}

static inline dim3 sgrid(long long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t launch_scalar_init(const CellArgs& a, const double* U0, double* f0, DevState* st,
                              int lam_mode, double lam_user, double cfl,
                              const double* const dir[4], hipStream_t s) {
    hipLaunchKernelGGL(scalar_bound_u_kernel, sgrid(a.plane, 256), dim3(256), 0, s, a, U0, st);
    ScalarSides ds;
    bool any = false;
    for (int k = 0; k < 4; ++k) {
        ds.d[k] = dir ? dir[k] : nullptr;
        any = any || ds.d[k];
    }
    if (any)
        hipLaunchKernelGGL(scalar_dirichlet_bound_kernel, sgrid(2LL * (a.nx + a.ny), 256), dim3(256),
                           0, s, a, ds, st);
    hipLaunchKernelGGL(scalar_init_eq_kernel, sgrid(a.plane, 256), dim3(256), 0, s, a, U0, f0, st,
                       lam_mode, lam_user, cfl);
    return hipGetLastError();
}

hipError_t launch_scalar_bound_f(const CellArgs& a, const double* f, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(scalar_bound_f_kernel, sgrid(a.plane, 256), dim3(256), 0, s, a, f, st);
    return hipGetLastError();
}

hipError_t launch_scalar_moments(const CellArgs& a, const double* f0, const double* f1,
                                 const DevState* st, int slot, double* U, hipStream_t s) {
    hipLaunchKernelGGL(scalar_moments_kernel, sgrid(a.plane, 256), dim3(256), 0, s, a, f0, f1, st,
                       slot, U);
    return hipGetLastError();
}

#define LBRS_SCALAR_WPB(X) X(1) X(2) X(4) X(6) X(8) X(12) X(16)

hipError_t launch_scalar_step2d(const ScalarArgs& a, int wpb, int max_blocks, hipStream_t s) {
#define LBRS_CASE(W)                                                                  \
    if (wpb == W) {                                                                   \
        int nblocks = (a.ntiles + W - 1) / W;                                         \
        if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;             \
        hipLaunchKernelGGL(scalar2d_step<W>, dim3(nblocks), dim3(64 * W), 0, s, a);  \
        return hipGetLastError();                                                     \
    }
    LBRS_SCALAR_WPB(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

int scalar2d_blocks_per_cu(int wpb) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
#define LBRS_CASE(W) \
    if (wpb == W) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, scalar2d_step<W>, 64 * W, 0);
    LBRS_SCALAR_WPB(LBRS_CASE)
#undef LBRS_CASE
    return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_scalar_step1d(const ScalarArgs& a, int q, hipStream_t s) {
    const dim3 grid((unsigned)((a.nx + STILE1D - 1) / STILE1D));
    if (a.blocked) {
        if (q == 2) hipLaunchKernelGGL((scalar1d_step<2, true>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((scalar1d_step<3, true>), grid, dim3(256), 0, s, a);
    } else {
        if (q == 2) hipLaunchKernelGGL((scalar1d_step<2, false>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((scalar1d_step<3, false>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace lbrs
