// Ragged batch of independent 1D LBRS problems (shock tubes) in one persistent
// launch (gfx950, FP64).
//
// Each unit runs the paper's 1D scheme (Sec. II.A update with exact hopping,
// Sec. II.C equilibria and wave-speed bound) with its own cell count, lattice
// speed, dt, t_end and side conditions, exactly as the plain single-domain
// kernels do it (same device functions, so results are bitwise equal).
//
// Work decomposition.  A unit of n cells is cut into g = ceil(n / C) chunks
// ("members"); chunk m is held in one workgroup's registers and LDS for the
// whole run, plus one halo cell on each side.  A step is
//   collide the chunk and its halo cells -> f* staged in LDS
//   pull the streamed f^{n+1} of the own cells, local bound, admissibility
//   publish the chunk's two edge cells and its bound -> team slot (parity n)
//   team barrier (one counter per unit), read the neighbours' edges into the
//   halo and the members' bounds -> lambda*_{n+1}.
// One team barrier per step; single-member units need none.
//
// Scheduling.  The grid is the resident workgroups (persistent).  The host
// assigns every member to a workgroup with a list schedule (earliest free
// workgroups first; teams start together), and each workgroup runs its jobs
// in order of scheduled start.  A team whose members are all present runs to
// completion, and the team with the earliest start among incomplete ones only
// waits for jobs that start earlier, so the schedule cannot deadlock.  Every
// spin is bounded: on the (never expected) limit the unit is flagged and the
// workgroup moves on, so every wave exits.
#include "lbrs_launch.hpp"

namespace lbrs {

static constexpr int QKMAX = 9;

struct TeamReduce {
    double lam;
    bool bad;
};

// Team exchange without cache flushes: slot data and the arrival counter are
// written and read with agent-scope atomics (coherent across XCDs, no L2
// write-back), and a writer waits for its stores' acknowledgement before its
// workgroup arrives, so arrival implies the data are visible.
__device__ inline unsigned load_counter(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_coherent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_coherent_u(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double load_relaxed(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned load_relaxed_u(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int Q, int CPT>
__device__ void run_job(const Batch1DArgs& a, const Job1D job, double* lds, double* red) {
    constexpr int QK = Q * 3;
    const Unit1D u = a.units[job.unit];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nwaves = (nt + 63) >> 6;
    const int C = job.c1 - job.c0;       // own cells; local halo cells -1 and C
    const int m = job.member, g = u.g;
    const double gm1 = u.gamma - 1.0;
    const bool transm = !u.periodic;
    EdgeSlot* my_slots = a.slots + a.slot_off[job.unit];
    unsigned* counter = a.counters + (long long)job.unit * COUNTER_STRIDE;
    const int W = C + 2;                 // local cells q = -1 .. C, stored at q + 1

    // f^n of the local cells (own cells and halo) in registers
    double f[CPT][QKMAX];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        int q = tid + k * nt - 1;
        int qc = q < 0 ? 0 : (q >= C ? C - 1 : q);  // halo starts as the edge cell
        long long cell = u.off + job.c0 + qc;
#pragma unroll
        for (int p = 0; p < QK; ++p) f[k][p] = (tid + k * nt < W) ? a.f[p * a.total + cell] : 0.0;
    }

    const UnitState1D s0 = a.states[job.unit];
    double t = s0.t, lam_used = s0.lam_used;
    long long n = s0.nsteps;
    bool bad = (s0.status & 1u) != 0u, timeout = false;
    double lam_star = 0.0;
    unsigned arrivals = 0;

    // Exchange of one step's edge cells and bounds.  Single-workgroup units
    // use LDS only; teams publish to their slots, meet at the barrier, and
    // read the members' bounds and the neighbours' edges in one round trip.
    auto exchange = [&](double lmax, bool lbad, int parity) {
        EdgeSlot* mine = my_slots + parity * g + m;
        double* edge = red + 64;             // [2][QKMAX]: own first and last cell
        double* mem = red + 96 + 2 * MAXTEAM * parity;  // members' bounds, then flags
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            int q = tid + k * nt - 1;
            if (q == 0) {
#pragma unroll
                for (int p = 0; p < QK; ++p) {
                    edge[p] = f[k][p];
                    if (g > 1) store_coherent(&mine->first[p], f[k][p]);
                }
            }
            if (q == C - 1) {
#pragma unroll
                for (int p = 0; p < QK; ++p) {
                    edge[QKMAX + p] = f[k][p];
                    if (g > 1) store_coherent(&mine->last[p], f[k][p]);
                }
            }
        }
        double wm = wave_max(lmax);
        bool wb = __any(lbad);
        if ((tid & 63) == 0) {
            red[2 * (tid >> 6)] = wm;
            red[2 * (tid >> 6) + 1] = wb ? 1.0 : 0.0;
        }
        __syncthreads();
        double mm = 0.0;
        bool bb = false;
        for (int w = 0; w < nwaves; ++w) {
            mm = fmax(mm, red[2 * w]);
            bb |= red[2 * w + 1] != 0.0;
        }
        if (g > 1) {
            if (tid == 0) {
                store_coherent(&mine->lam, mm);
                store_coherent_u(&mine->bad, bb ? 1u : 0u);
            }
            __builtin_amdgcn_s_waitcnt(0);  // this thread's slot stores acknowledged
            __syncthreads();
            if (tid == 0) {
                __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                arrivals += (unsigned)g;
                unsigned spins = 0;
                bool ok = true;
                while (load_counter(counter) < arrivals) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > a.spin_limit) {
                        ok = false;  // never expected: give up, flag the unit
                        break;
                    }
                }
                red[62] = ok ? 0.0 : 1.0;
            }
            __syncthreads();
            if (red[62] != 0.0) timeout = true;
            // members' bounds and flags, one member per thread
            if (tid < g) {
                const EdgeSlot* sl = my_slots + parity * g + tid;
                mem[tid] = load_relaxed(&sl->lam);
                mem[MAXTEAM + tid] = load_relaxed_u(&sl->bad) ? 1.0 : 0.0;
            }
        }
        // halo cells: the neighbours' edges, or the side condition at the ends
        const EdgeSlot* left = nullptr;
        const EdgeSlot* right = nullptr;
        if (m > 0) left = my_slots + parity * g + (m - 1);
        if (m < g - 1) right = my_slots + parity * g + (m + 1);
        if (g > 1 && !transm) {
            if (m == 0) left = my_slots + parity * g + (g - 1);
            if (m == g - 1) right = my_slots + parity * g;
        }
        // single-workgroup periodic unit: the halo wraps onto its own edges
        const bool wrap_self = g == 1 && !transm;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            int q = tid + k * nt - 1;
            if (q == -1) {
#pragma unroll
                for (int p = 0; p < QK; ++p)
                    f[k][p] = left ? load_relaxed(&left->last[p])
                                   : (wrap_self ? edge[QKMAX + p] : edge[p]);
            }
            if (q == C) {
#pragma unroll
                for (int p = 0; p < QK; ++p)
                    f[k][p] = right ? load_relaxed(&right->first[p])
                                    : (wrap_self ? edge[p] : edge[QKMAX + p]);
            }
        }
        __syncthreads();  // halo and member values in place; red/edge reusable
        if (g > 1) {
            mm = 0.0;
            bb = false;
            for (int j = 0; j < g; ++j) {
                mm = fmax(mm, mem[j]);
                bb |= mem[MAXTEAM + j] != 0.0;
            }
        }
        TeamReduce tr;
        tr.lam = mm;
        tr.bad = bb;
        return tr;
    };

    // lambda*_0 from U^0 of the own cells
    {
        double lmax = 0.0;
        bool lbad = false;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            int q = tid + k * nt - 1;
            if (q >= 0 && q < C) {
                double U[3], l;
                moments_1d<Q>(f[k], U);
                lbad |= !bound_1d(U, u.gamma, &l);
                lmax = fmax(lmax, l);
            }
        }
        TeamReduce r = exchange(lmax, lbad, 1);
        lam_star = r.lam;
        bad = bad || r.bad;
    }

    int it = 0;
    for (; it < a.max_steps && !timeout; ++it) {
        if (bad || !(t < u.t_end)) break;
        double lam, tn;
        if (u.lam_mode == LAM_PER_STEP) {
            double dt = u.cfl * u.dx / lam_star;
            double rem = u.t_end - t;
            bool last = false;
            if (dt >= rem) {
                dt = rem;
                last = true;
            }
            lam = u.dx / dt;
            tn = last ? u.t_end : t + dt;
        } else {
            lam = u.lam_fixed;
            tn = t + u.dx / lam;
        }
        const double c2lam = 1.0 / (2.0 * lam);
        // collide the local cells (own and halo); the two moving populations
        // go to LDS (slots 0..2: s = -1, 3..5: s = +1), D1Q3's rest
        // population stays in its cell's registers
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            int q = tid + k * nt - 1;
            if (q >= -1 && q <= C) {
                double U[3], fs[QKMAX];
                moments_1d<Q>(f[k], U);
                collide_1d<Q>(f[k], U, gm1, c2lam, u.omega, fs);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    lds[c * W + q + 1] = fs[c];
                    lds[(3 + c) * W + q + 1] = fs[(Q - 1) * 3 + c];
                    if (Q == 3) f[k][3 + c] = fs[3 + c];
                }
            }
        }
        __syncthreads();
        // stream into the own cells
        double lmax = 0.0;
        bool lbad = false;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            int q = tid + k * nt - 1;
            if (q >= 0 && q < C) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    f[k][c] = lds[c * W + q + 2];                          // s = -1: from q + 1
                    f[k][(Q - 1) * 3 + c] = lds[(3 + c) * W + q];          // s = +1: from q - 1
                }
                double U[3], l;
                moments_1d<Q>(f[k], U);
                lbad |= !bound_1d(U, u.gamma, &l);
                lmax = fmax(lmax, l);
            }
        }
        TeamReduce r = exchange(lmax, lbad, it & 1);
        t = tn;
        n += 1;
        lam_used = lam;
        if (u.lam_mode == LAM_PER_STEP) lam_star = r.lam;
        if (r.bad) bad = true;
    }

    // write back the own cells; member 0 records the unit's state
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        int q = tid + k * nt - 1;
        if (q >= 0 && q < C) {
            long long cell = u.off + job.c0 + q;
#pragma unroll
            for (int p = 0; p < QK; ++p) a.f[p * a.total + cell] = f[k][p];
        }
    }
    if (m == 0 && tid == 0) {
        UnitState1D s;
        s.t = t;
        s.nsteps = n;
        s.lam_used = lam_used;
        s.status = (bad ? 1u : 0u) | (timeout ? 2u : 0u) | s0.status;
        s.pad = 0;
        s.fail_step = (s0.status & 1u) ? s0.fail_step : (bad ? n : -1);
        a.states[job.unit] = s;
    }
}

// MAXT: the largest workgroup the instance is launched with.  Four cells per
// thread need more than the 128 registers a 1024-thread bound leaves (they
// spilled to scratch memory), so workgroups of up to 512 and of up to 768
// threads get instances of their own.
template <int Q, int CPT, int MAXT>
__global__ __launch_bounds__(MAXT) void batch1d_persistent(Batch1DArgs a) {
    extern __shared__ double lds[];
    // [0,32) wave partials, 62 barrier flag, [64,82) edge cells, then the
    // members' bounds and flags for the two step parities
    __shared__ double red[96 + 4 * MAXTEAM];
    const int w = blockIdx.x;
    for (int j = a.job_begin[w]; j < a.job_begin[w + 1]; ++j) {
        run_job<Q, CPT>(a, a.jobs[j], lds, red);
        __syncthreads();
    }
}

// f^0 = f^eq(U0) per unit at lambda*(U0)/cfl (or the unit's fixed speed):
// one workgroup per unit reduces the bound, then sets the populations.
template <int Q>
__global__ __launch_bounds__(256) void batch1d_init(const Unit1D* units, Unit1D* units_rw,
                                                    const double* __restrict__ U0, double* f,
                                                    long long total, UnitState1D* states) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const Unit1D u = units[b];
    double lmax = 0.0;
    for (int j = threadIdx.x; j < u.n; j += blockDim.x) {
        double U[3], l;
        for (int k = 0; k < 3; ++k) U[k] = U0[k * total + u.off + j];
        bound_1d(U, u.gamma, &l);
        lmax = fmax(lmax, l);
    }
    double wm = wave_max(lmax);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wm;
    __syncthreads();
    double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    double lam0 = u.lam_mode == LAM_USER ? u.lam_fixed : m / u.cfl;
    for (int j = threadIdx.x; j < u.n; j += blockDim.x) {
        double U[3], z[9], fs[9];
        for (int k = 0; k < 3; ++k) U[k] = U0[k * total + u.off + j];
        for (int p = 0; p < 9; ++p) z[p] = 0.0;
        collide_1d<Q>(z, U, u.gamma - 1.0, 1.0 / (2.0 * lam0), 1.0, fs);
        for (int p = 0; p < Q * 3; ++p) f[p * total + u.off + j] = fs[p];
    }
    if (threadIdx.x == 0) {
        units_rw[b].lam_fixed = lam0;
        UnitState1D st;
        st.t = 0.0;
        st.nsteps = 0;
        st.lam_used = lam0;
        st.status = 0u;
        st.pad = 0;
        st.fail_step = -1;
        states[b] = st;
    }
}

__global__ void zero_counters(unsigned* c, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[(long long)i * COUNTER_STRIDE] = 0u;
}

hipError_t launch_zero_counters(unsigned* c, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_counters, dim3((n + 255) / 256), dim3(256), 0, s, c, n);
    return hipGetLastError();
}

hipError_t launch_batch1d_init(const Unit1D* units, Unit1D* units_rw, int nunits, const double* U0,
                               double* f, long long total, UnitState1D* states, int Q, hipStream_t s) {
    if (Q == 2)
        hipLaunchKernelGGL(batch1d_init<2>, dim3(nunits), dim3(256), 0, s, units, units_rw, U0, f, total,
                           states);
    else
        hipLaunchKernelGGL(batch1d_init<3>, dim3(nunits), dim3(256), 0, s, units, units_rw, U0, f, total,
                           states);
    return hipGetLastError();
}

// (the dynamic LDS limit of the instance is raised by batch1d_blocks_per_cu,
// which the plan calls first, so nothing here is illegal under graph capture)
template <int Q, int CPT, int MAXT>
static hipError_t launch_b1(const Batch1DArgs& a, int grid, int threads, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((batch1d_persistent<Q, CPT, MAXT>), dim3(grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// The instance for (Q, cells per thread, workgroup size).
template <int Q>
static const void* b1_kernel(int cpt, int threads) {
    if (cpt <= 1) return (const void*)batch1d_persistent<Q, 1, 1024>;
    if (cpt <= 2) return (const void*)batch1d_persistent<Q, 2, 1024>;
    if (cpt <= 4)
        return threads <= 512 ? (const void*)batch1d_persistent<Q, 4, 512>
             : threads <= 768 ? (const void*)batch1d_persistent<Q, 4, 768>
                              : (const void*)batch1d_persistent<Q, 4, 1024>;
    return nullptr;
}

template <int Q>
static hipError_t launch_b1q(const Batch1DArgs& a, int grid, int threads, int cpt, size_t lds,
                             hipStream_t s) {
    if (cpt <= 1) return launch_b1<Q, 1, 1024>(a, grid, threads, lds, s);
    if (cpt <= 2) return launch_b1<Q, 2, 1024>(a, grid, threads, lds, s);
    if (cpt <= 4)
        return threads <= 512 ? launch_b1<Q, 4, 512>(a, grid, threads, lds, s)
             : threads <= 768 ? launch_b1<Q, 4, 768>(a, grid, threads, lds, s)
                              : launch_b1<Q, 4, 1024>(a, grid, threads, lds, s);
    return hipErrorInvalidValue;
}

// chunk = cells per member; threads per workgroup; the local cells (chunk + 2
// halo) are spread CPT per thread.
hipError_t launch_batch1d(const Batch1DArgs& a, int grid, int threads, int chunk, hipStream_t s) {
    const int W = chunk + 2;
    const int cpt = (W + threads - 1) / threads;
    size_t lds = batch1d_lds_bytes(chunk);
    if (threads < 1 || threads > 1024) return hipErrorInvalidValue;
    return a.Q == 2 ? launch_b1q<2>(a, grid, threads, cpt, lds, s)
                    : launch_b1q<3>(a, grid, threads, cpt, lds, s);
}

// Dynamic LDS of one workgroup: the two moving populations' post-collision
// values (3 components each) of the chunk's cells and its two halo cells.
size_t batch1d_lds_bytes(int chunk) { return sizeof(double) * 6 * (size_t)(chunk + 2); }

int batch1d_blocks_per_cu(int Q, int threads, int chunk) {
    const int W = chunk + 2;
    const int cpt = (W + threads - 1) / threads;
    size_t lds = batch1d_lds_bytes(chunk);
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    const void* k = Q == 2 ? b1_kernel<2>(cpt, threads) : b1_kernel<3>(cpt, threads);
    if (!k) return 0;
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, lds);
    return e == hipSuccess ? n : 0;
}

}  // namespace lbrs
