// Fused LBRS steps for the 1D Euler equations, D1Q2 and D1Q3 (gfx950, FP64).
//
// Two forms of the same step (Sec. II.A discrete update with exact hopping,
// Sec. II.C equilibria and the Jin-Xin wave-speed bound):
//
//  * step1d_march: one launch per step for long domains.  Each wave marches
//    a contiguous run of aligned 64-cell chunks; the hops are wavefront lane
//    shifts, the chunk-edge values are carried between consecutive chunks,
//    and the next step's bound is reduced from the new moments in the same
//    pass.
//
//  * run1d_persistent: the whole time loop of a domain that fits in one
//    workgroup's LDS, in one launch.  Populations live in registers; each step
//    stages f* in LDS, pulls the streamed values back, and reduces the bound
//    across the workgroup (two barriers per step).  No HBM traffic between
//    steps.
#include "lbrs_launch.hpp"
#include "lbrs_rowops.hpp"

namespace lbrs {

// One step for long domains without LDS: every wave marches a contiguous run
// of 64-cell chunks (aligned, lane l = cell 64 c + l) with the next chunk's
// populations prefetched.  The hops are one-lane wavefront shifts (DPP); the
// two values a chunk needs from outside it -- the post-collision population
// moving right from the cell before it and the one moving left from the cell
// after it -- come from the neighbouring chunks of the same march, carried in
// scalar registers (lane 63 of the previous chunk, lane 0 of the next).  Only
// the cell before the run and the cell after it are extra work (one cell each,
// loaded by every lane, so one cache line).  Stores are range-checked buffer
// stores, so the loop has no branch around memory instructions.  The next
// step's bound is reduced in the same pass, as in the 2D step.
static constexpr int CHUNK1D = 64;

// The value lane l holds, in every lane (wave-uniform).
__device__ inline double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

template <int Q>
__global__ __launch_bounds__(256) void step1d_march(Step1DArgs a) {
    constexpr int QK = Q * 3;
    constexpr int R = (Q - 1) * 3;  // first plane of the population moving right (s = +1)
    const LaunchSlots ls = slots_for(a.launch);
    DevState* st = a.st;
    const StepCtl c = step_control(st, ls, a.lam_mode, a.dx, a.cfl, a.t_end);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_state(st, ls, c);
    if (!c.active) return;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double* __restrict__ fin = c.cur ? a.f1 : a.f0;
    double* __restrict__ fout = c.cur ? a.f0 : a.f1;
    const double gm1 = a.gamma - 1.0, c2lam = 1.0 / (2.0 * c.lam);
    const bool per = a.periodic != 0;
    const int nx = a.nx;
    const long long nchunks = (nx + CHUNK1D - 1) / CHUNK1D;
    const long long nw = (long long)gridDim.x * 4;
    const long long w = (long long)xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    const long long c0 = w * nchunks / nw, c1 = (w + 1) * nchunks / nw;  // chunks [c0, c1)

    // populations of cell x0 + stride * lane (wrapped or clamped onto the grid)
    auto load = [&](double (&v)[QK], long long x0, int stride) {
        const int xl = map_index((int)(x0 + stride * lane), nx, per);
#pragma unroll
        for (int p = 0; p < QK; ++p) v[p] = fin[p * a.plane + xl];
    };
    // what completes chunk ch: chunk ch + 1, or past the run the one cell after it
    auto load_next = [&](double (&v)[QK], long long ch) {
        const long long nc = ch + 1 < c1 ? ch + 1 : c1;
        load(v, nc * CHUNK1D, ch + 1 < c1 ? 1 : 0);
    };
    auto collide = [&](const double (&f)[QK], double (&fs)[QK]) {
        double U[3];
        moments_1d<Q>(f, U);
        collide_1d<Q>(f, U, gm1, c2lam, a.omega, fs);
    };

    double lmax = 0.0;
    bool bad = false;
    if (c0 < c1) {
        double f[QK], fs[QK], fc[QK], nxt[QK];
        double from_left[3];  // s = +1 population of the cell before the current chunk
        load(f, c0 * CHUNK1D - 1, 0);  // the cell before the run
        load(nxt, c0 * CHUNK1D, 1);    // chunk c0
        collide(f, fs);
#pragma unroll
        for (int k = 0; k < 3; ++k) from_left[k] = lane_value(fs[R + k], 0);
#pragma unroll
        for (int p = 0; p < QK; ++p) f[p] = nxt[p];
        load_next(nxt, c0);
        collide(f, fc);
        for (long long ch = c0; ch < c1; ++ch) {
#pragma unroll
            for (int p = 0; p < QK; ++p) f[p] = nxt[p];
            load_next(nxt, ch + 1);  // the run's last iterations reload the cell after it
            collide(f, fs);          // chunk ch + 1 (or the cell after the run)
            double g[QK];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double after = lane_value(fs[k], 0);      // s = -1 from the next cell
                const double sl = lane_from_right(fc[k]);       // s = -1: from cell x + 1
                g[k] = lane == 63 ? after : sl;
                if (Q == 3) g[3 + k] = fc[3 + k];               // rest particle
                const double sr = lane_from_left(fc[R + k]);    // s = +1: from cell x - 1
                g[R + k] = lane == 0 ? from_left[k] : sr;
                from_left[k] = lane_value(fc[R + k], 63);
            }
            const long long x0 = ch * CHUNK1D;
            const long long rest = nx - x0;
            const int rec = (int)(rest < CHUNK1D ? rest : CHUNK1D) * 8;
            const bool out = lane < rest;
#pragma unroll
            for (int p = 0; p < QK; ++p) store_row(fout + p * a.plane + x0, rec, lane * 8, g[p]);
            double Un[3], l;
            moments_1d<Q>(g, Un);
            const bool ok = bound_1d(Un, a.gamma, &l);
            bad |= out && !ok;
            lmax = fmax(lmax, out ? l : 0.0);
#pragma unroll
            for (int p = 0; p < QK; ++p) fc[p] = fs[p];
        }
    }
    if (a.lam_mode == LAM_PER_STEP) {
        double wm = wave_max(lmax);
        if (lane == 0) publish_max(&st->lam[ls.la], wm);
    }
    if (__any(bad) && lane == 0) publish_bad(st, ls, c.n + 1);
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
        for (int p = 0; p < QK; ++p) f[c][p] = fin[p * a.plane + jl];
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
                for (int p = 0; p < QK; ++p) fout[p * a.plane + j] = f[c][p];
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

// Resident 256-lane workgroups of the marching kernel on the device (cached).
template <int Q>
static int march1d_max_blocks() {
    static int cached = 0;
    if (cached == 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, step1d_march<Q>, 256, 0) !=
                hipSuccess || per < 1)
            return 1024;
        cached = cus * per;
    }
    return cached;
}

hipError_t launch_step1d(const Step1DArgs& a, int Q, hipStream_t s) {
    // one chunk per wave on short domains; long ones fill the resident waves
    const long long chunks = (a.nx + CHUNK1D - 1) / CHUNK1D;
    const long long want = (chunks + 3) / 4;
    if (Q == 2) {
        const long long cap = march1d_max_blocks<2>();
        hipLaunchKernelGGL(step1d_march<2>, dim3((unsigned)(want < cap ? want : cap)), dim3(256), 0,
                           s, a);
    } else {
        const long long cap = march1d_max_blocks<3>();
        hipLaunchKernelGGL(step1d_march<3>, dim3((unsigned)(want < cap ? want : cap)), dim3(256), 0,
                           s, a);
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
