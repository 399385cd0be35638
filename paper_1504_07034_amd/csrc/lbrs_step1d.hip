// Fused LBRS steps for the 1D Euler equations, D1Q2 and D1Q3 (gfx950, FP64).
//
// Two forms of the same step (Sec. II.A discrete update with exact hopping,
// Sec. II.C equilibria and the Jin-Xin wave-speed bound):
//
//  * step1d_tile: one launch per step for long domains (planar or blocked
//    1D population layout).  A 256-lane workgroup
//    owns 512 output cells (two per lane) plus one halo cell on each side; the
//    lanes form the post-collision populations of those cells, stage them in
//    LDS, and pull f_i^{n+1}(x) = f*_i(x - s_i) from the neighbours' entries.
//    The next step's bound is reduced from the new moments in the same pass.
//
//  * run1d_persistent: the whole time loop of a domain that fits in one
//    workgroup's LDS, in one launch.  Populations live in registers; each step
//    stages f* in LDS, pulls the streamed values back, and reduces the bound
//    across the workgroup (two barriers per step).  No HBM traffic between
//    steps.
#include "lbrs_launch.hpp"

namespace lbrs {

static constexpr int TILE1D = 512;  // output cells per workgroup (2 per lane)

template <int Q, bool BLOCKED>
__global__ __launch_bounds__(256) void step1d_tile(Step1DArgs a) {
    constexpr int QK = Q * 3;
    constexpr int E = TILE1D + 2;  // LDS entry e holds cell x0 - 1 + e
    __shared__ double fsl[QK][E];
    const LaunchSlots ls = slots_for(a.launch);
    DevState* st = a.st;
    const StepCtl c = step_control(st, ls, a.lam_mode, a.dx, a.cfl, a.t_end);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_state(st, ls, c);
    if (!c.active) return;

    const int t = threadIdx.x;
    const int x0 = blockIdx.x * TILE1D;
    const double* __restrict__ fin = c.cur ? a.f1 : a.f0;
    double* __restrict__ fout = c.cur ? a.f0 : a.f1;
    const double gm1 = a.gamma - 1.0, c2lam = 1.0 / (2.0 * c.lam);

    // post-collision values of the tile's cells and its two halo cells
    constexpr int PASSES = TILE1D / 256 + 1;  // the last pass covers the halo entries
#pragma unroll
    for (int k = 0; k < PASSES; ++k) {
        const int e = t + 256 * k;
        if (k == PASSES - 1 && e >= E) break;
        const int xl = map_index(x0 - 1 + e, a.nx, a.periodic != 0);
        double f[QK], U[3], fs[QK];
#pragma unroll
        for (int p = 0; p < QK; ++p) f[p] = fin[ofs1d(BLOCKED, a.plane, QK * BLOCK1D, p, xl)];
        moments_1d<Q>(f, U);
        collide_1d<Q>(f, U, gm1, c2lam, a.omega, fs);
#pragma unroll
        for (int p = 0; p < QK; ++p) fsl[p][e] = fs[p];
    }
    __syncthreads();

    double lmax = 0.0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < TILE1D / 256; ++k) {
        const int j = t + 256 * k;  // output cell x0 + j reads entries j, j+1, j+2
        const int x = x0 + j;
        if (x < a.nx) {
            double g[QK];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                g[0 * 3 + kk] = fsl[0 * 3 + kk][j + 2];          // s = -1: from x + 1
                if (Q == 2) {
                    g[1 * 3 + kk] = fsl[1 * 3 + kk][j];          // s = +1: from x - 1
                } else {
                    g[1 * 3 + kk] = fsl[1 * 3 + kk][j + 1];      // rest particle
                    g[2 * 3 + kk] = fsl[2 * 3 + kk][j];          // s = +1: from x - 1
                }
            }
#pragma unroll
            for (int p = 0; p < QK; ++p) fout[ofs1d(BLOCKED, a.plane, QK * BLOCK1D, p, x)] = g[p];
            double Un[3], l;
            moments_1d<Q>(g, Un);
            const bool ok = bound_1d(Un, a.gamma, &l);
            bad |= !ok;
            lmax = fmax(lmax, l);
        }
    }
    if (a.lam_mode == LAM_PER_STEP) {
        double wm = wave_max(lmax);
        if ((t & 63) == 0) publish_max(&st->lam[ls.la], wm);
    }
    if (__any(bad) && (t & 63) == 0) publish_bad(st, ls, c.n + 1);
}

// Whole run of one domain of nx <= CPT * blockDim.x cells in one workgroup.
// Dynamic LDS: Q*3*nx doubles (the staged post-collision populations).
template <int Q, int CPT>
__global__ __launch_bounds__(1024) void run1d_persistent(Step1DArgs a) {
    constexpr int QK = Q * 3;
    extern __shared__ double lds[];
    __shared__ double red[2][16];
    const LaunchSlots ls = slots_for(a.launch);
    DevState* st = a.st;
    const Slot s0 = st->s[ls.sr];
    double t = s0.t;
    long long n = s0.n;
    double lam_used = s0.lam_used;
    bool bad = st->bad[ls.lr] != 0u;
    double lam_star = __longlong_as_double((long long)st->lam[ls.lr]);
    const int N = a.nx;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nwaves = (nt + 63) >> 6;
    const double* __restrict__ fin = s0.cur ? a.f1 : a.f0;
    double* __restrict__ fout = s0.cur ? a.f0 : a.f1;
    const double gm1 = a.gamma - 1.0;

    double f[CPT][QK];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        int j = tid + c * nt;
        int jl = j < N ? j : N - 1;
#pragma unroll
        for (int p = 0; p < QK; ++p)
            f[c][p] = fin[ofs1d(a.blocked != 0, a.plane, QK * BLOCK1D, p, jl)];
    }

    int steps = 0;
    for (int it = 0; it < a.max_steps; ++it) {
        if (bad || !(t < a.t_end)) break;
        double lam, tn;
        if (a.lam_mode == LAM_PER_STEP) {
            double dt = a.cfl * a.dx / lam_star;
            double rem = a.t_end - t;
            bool last = false;
            if (dt >= rem) {
                dt = rem;
                last = true;
            }
            lam = a.dx / dt;
            tn = last ? a.t_end : t + dt;
        } else {
            lam = st->lam_fixed;
            tn = t + a.dx / lam;
        }
        const double c2lam = 1.0 / (2.0 * lam);
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            int j = tid + c * nt;
            if (j < N) {
                double U[3], fs[QK];
                moments_1d<Q>(f[c], U);
                collide_1d<Q>(f[c], U, gm1, c2lam, a.omega, fs);
#pragma unroll
                for (int p = 0; p < QK; ++p) lds[p * N + j] = fs[p];
            }
        }
        __syncthreads();
        double lmax = 0.0;
        bool lbad = false;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            int j = tid + c * nt;
            if (j < N) {
                const int jp = map_index(j + 1, N, a.periodic != 0);
                const int jm = map_index(j - 1, N, a.periodic != 0);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    f[c][0 * 3 + k] = lds[(0 * 3 + k) * N + jp];
                    if (Q == 2) {
                        f[c][1 * 3 + k] = lds[(1 * 3 + k) * N + jm];
                    } else {
                        f[c][1 * 3 + k] = lds[(1 * 3 + k) * N + j];
                        f[c][2 * 3 + k] = lds[(2 * 3 + k) * N + jm];
                    }
                }
                double Un[3], l;
                moments_1d<Q>(f[c], Un);
                lbad |= !bound_1d(Un, a.gamma, &l);
                lmax = fmax(lmax, l);
            }
        }
        double wm = wave_max(lmax);
        if ((tid & 63) == 0) red[it & 1][tid >> 6] = wm;
        int any_bad = __syncthreads_or(lbad ? 1 : 0);
        double m = 0.0;
        for (int w = 0; w < nwaves; ++w) m = fmax(m, red[it & 1][w]);
        t = tn;
        n += 1;
        lam_used = lam;
        ++steps;
        if (a.lam_mode == LAM_PER_STEP) lam_star = m;
        if (any_bad) bad = true;
    }

    if (steps > 0) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            int j = tid + c * nt;
            if (j < N) {
#pragma unroll
                for (int p = 0; p < QK; ++p)
                    fout[ofs1d(a.blocked != 0, a.plane, QK * BLOCK1D, p, j)] = f[c][p];
            }
        }
    }
    if (tid == 0) {
        Slot s = s0;
        s.t = t;
        s.n = n;
        s.lam_used = lam_used;
        if (steps > 0) s.cur = s0.cur ^ 1;
        st->s[ls.sw] = s;
        st->lam[ls.la] = (unsigned long long)__double_as_longlong(lam_star);
        st->bad[ls.la] = bad ? 1u : 0u;
        st->lam[ls.lz] = 0ull;
        st->bad[ls.lz] = 0u;
        if (bad && st->bad[ls.lr] == 0u) {
            atomicOr(&st->status, 1u);
            atomicMin(&st->fail_step, (unsigned long long)n);
        }
    }
}

hipError_t launch_step1d(const Step1DArgs& a, int Q, hipStream_t s) {
    int nblocks = (a.nx + TILE1D - 1) / TILE1D;
    if (a.blocked) {
        if (Q == 2) hipLaunchKernelGGL((step1d_tile<2, true>), dim3(nblocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((step1d_tile<3, true>), dim3(nblocks), dim3(256), 0, s, a);
    } else {
        if (Q == 2) hipLaunchKernelGGL((step1d_tile<2, false>), dim3(nblocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((step1d_tile<3, false>), dim3(nblocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

// Largest domain the persistent form accepts for Q populations, given the
// device's LDS limit per workgroup.
int persistent1d_max_cells(int Q, size_t lds_limit) {
    size_t by_lds = lds_limit / (sizeof(double) * 3 * Q);
    size_t by_regs = 2 * 1024;
    size_t m = by_lds < by_regs ? by_lds : by_regs;
    return (int)m;
}

hipError_t launch_run1d(const Step1DArgs& a, int Q, hipStream_t s) {
    int N = a.nx;
    int cpt = N <= 1024 ? 1 : 2;
    int threads = (N + cpt - 1) / cpt;
    threads = ((threads + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    size_t lds = sizeof(double) * 3 * Q * (size_t)N;
    hipError_t e = hipSuccess;
    if (Q == 2) {
        if (cpt == 1) {
            e = hipFuncSetAttribute((const void*)run1d_persistent<2, 1>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e == hipSuccess)
                hipLaunchKernelGGL((run1d_persistent<2, 1>), dim3(1), dim3(threads), lds, s, a);
        } else {
            e = hipFuncSetAttribute((const void*)run1d_persistent<2, 2>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e == hipSuccess)
                hipLaunchKernelGGL((run1d_persistent<2, 2>), dim3(1), dim3(threads), lds, s, a);
        }
    } else {
        if (cpt == 1) {
            e = hipFuncSetAttribute((const void*)run1d_persistent<3, 1>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e == hipSuccess)
                hipLaunchKernelGGL((run1d_persistent<3, 1>), dim3(1), dim3(threads), lds, s, a);
        } else {
            e = hipFuncSetAttribute((const void*)run1d_persistent<3, 2>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e == hipSuccess)
                hipLaunchKernelGGL((run1d_persistent<3, 2>), dim3(1), dim3(threads), lds, s, a);
        }
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace lbrs
