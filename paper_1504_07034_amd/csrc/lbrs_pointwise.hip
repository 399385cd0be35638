// Pointwise kernels around the LBRS step (gfx950, FP64): state reset,
// primitive -> conserved conversion, the initial equilibrium (Sec. II.A:
// f_i = f_i^eq(u0)), moments (eq. "moments_system"), population copies, the
// window objective and its seed, and the adjoint of one fixed-speed D2Q4 step
// and of the initialisation.
#include "lbrs_launch.hpp"

namespace lbrs {


__host__ __device__ inline int nq_of(int model) { return model == D1Q2 ? 2 : (model == D1Q3 ? 3 : 4); }
__host__ __device__ inline int nk_of(int model) { return model == D2Q4 ? 4 : 3; }

__global__ void reset_state_kernel(DevState* st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int i = 0; i < 2; ++i) {
            st->s[i].t = 0.0;
            st->s[i].n = 0;
            st->s[i].lam_used = 0.0;
            st->s[i].cur = 0;
            st->s[i].pad = 0;
        }
        for (int i = 0; i < 3; ++i) {
            st->lam[i] = 0ull;
            st->bad[i] = 0u;
        }
        st->status = 0u;
        st->fail_step = ~0ull;
        st->lam_fixed = 0.0;
        st->lam_init = 0ull;
        st->J = 0.0;
        st->lam_bc = 0ull;
    }
}

// E = p/(rho(gamma-1)) + |u|^2/2, U = (rho, rho u, [rho v,] rho E)
__global__ void prim_to_cons_kernel(CellArgs a, const double* __restrict__ W, double* __restrict__ U) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.plane) return;
    const long long P = a.plane;
    double rho = W[c];
    if (a.model == D2Q4) {
        double u = W[P + c], v = W[2 * P + c], p = W[3 * P + c];
        U[c] = rho;
        U[P + c] = rho * u;
        U[2 * P + c] = rho * v;
        U[3 * P + c] = p / (a.gamma - 1.0) + 0.5 * rho * (u * u + v * v);
    } else {
        double u = W[P + c], p = W[2 * P + c];
        U[c] = rho;
        U[P + c] = rho * u;
        U[2 * P + c] = p / (a.gamma - 1.0) + 0.5 * rho * u * u;
    }
}

// Adjoint of prim_to_cons: Wbar = (dU/dW)^T Ubar.
__global__ void prim_to_cons_adjoint_kernel(CellArgs a, const double* __restrict__ W,
                                            const double* __restrict__ Ub, double* __restrict__ Wb) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.plane) return;
    const long long P = a.plane;
    const double gm1 = a.gamma - 1.0;
    double rho = W[c];
    if (a.model == D2Q4) {
        double u = W[P + c], v = W[2 * P + c];
        double b0 = Ub[c], b1 = Ub[P + c], b2 = Ub[2 * P + c], b3 = Ub[3 * P + c];
        Wb[c] = b0 + u * b1 + v * b2 + 0.5 * (u * u + v * v) * b3;
        Wb[P + c] = rho * b1 + rho * u * b3;
        Wb[2 * P + c] = rho * b2 + rho * v * b3;
        Wb[3 * P + c] = b3 / gm1;
    } else {
        double u = W[P + c];
        double b0 = Ub[c], b1 = Ub[P + c], b2 = Ub[2 * P + c];
        Wb[c] = b0 + u * b1 + 0.5 * u * u * b2;
        Wb[P + c] = rho * b1 + rho * u * b2;
        Wb[2 * P + c] = b2 / gm1;
    }
}

// Gas at rest with p = rho^gamma/gamma: U = (rho, 0, [0,] rho^gamma/(gamma(gamma-1))).
__global__ void isentropic_to_cons_kernel(CellArgs a, const double* __restrict__ rho,
                                          double* __restrict__ U) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.plane) return;
    const long long P = a.plane;
    const int K = nk_of(a.model);
    double r = rho[c];
    U[c] = r;
    for (int k = 1; k < K - 1; ++k) U[k * P + c] = 0.0;
    U[(K - 1) * P + c] = pow(r, a.gamma) / (a.gamma * (a.gamma - 1.0));
}

// Its adjoint: rhobar = Ubar_rho + Ubar_E rho^(gamma-1)/(gamma-1).
__global__ void isentropic_to_cons_adjoint_kernel(CellArgs a, const double* __restrict__ rho,
                                                  const double* __restrict__ Ub,
                                                  double* __restrict__ rb) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.plane) return;
    const int K = nk_of(a.model);
    double r = rho[c];
    rb[c] = Ub[c] + Ub[(K - 1) * a.plane + c] * pow(r, a.gamma - 1.0) / (a.gamma - 1.0);
}

__device__ inline bool cell_bound(int model, const double* U, double gamma, double* l) {
    return model == D2Q4 ? bound_d2q4(U, gamma, l) : bound_1d(U, gamma, l);
}

// Is cell c solid (a body's codes are given and mark it)?
__device__ inline bool solid_cell(const CellArgs& a, long long c) {
    return a.code && (a.code[c] & CODE_SOLID);
}

// lambda*(U0) -> st->lam_init; a non-physical U0 sets the status (step 0).
// Solid cells take no part.
__global__ void bound_of_U_kernel(CellArgs a, const double* __restrict__ U, DevState* st) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    bool bad = false;
    if (c < a.plane && !solid_cell(a, c)) {
        const int K = nk_of(a.model);
        double Uc[4];
        for (int k = 0; k < K; ++k) Uc[k] = U[k * a.plane + c];
        bad = !cell_bound(a.model, Uc, a.gamma, &l);
    }
    double wm = wave_max(l);
    if ((threadIdx.x & 63) == 0) publish_max(&st->lam_init, wm);
    if (__any(bad) && (threadIdx.x & 63) == 0) {
        atomicOr(&st->bad[0], 1u);
        atomicOr(&st->status, 1u);
        atomicMin(&st->fail_step, 0ull);
    }
}

// Bounds of the prescribed states of the Dirichlet sides (D2Q4): into the
// initial bound (the ghost cells count like interior cells) and into lam_bc,
// which every later per-step bound includes.  A non-admissible prescribed
// state is reported like a non-admissible U0.  Thread j covers position j of
// the concatenated sides x-low, x-high (ny each), y-low, y-high (nx each).
struct DirSides {
    const double* d[4];
};
__global__ void dirichlet_bound_kernel(CellArgs a, DirSides ds, DevState* st) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    bool bad = false;
    const long long nxs = a.ny, nys = a.nx;
    int side = -1;
    long long pos = 0, n = 0;
    if (j < nxs) { side = 0; pos = j; n = nxs; }
    else if (j < 2 * nxs) { side = 1; pos = j - nxs; n = nxs; }
    else if (j < 2 * nxs + nys) { side = 2; pos = j - 2 * nxs; n = nys; }
    else if (j < 2 * nxs + 2 * nys) { side = 3; pos = j - 2 * nxs - nys; n = nys; }
    if (side >= 0 && ds.d[side]) {
        double U[4];
        for (int k = 0; k < 4; ++k) U[k] = ds.d[side][k * n + pos];
        bad = !bound_d2q4(U, a.gamma, &l);
    }
    double wm = wave_max(l);
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

// f^0 = f^eq(U0) at the lattice speed lambda*(U0)/cfl (or the user's), then
// lambda*_0 from U^0 = sum_i f^0_i into reduction slot 0.  Solid cells of a
// body hold zeros and take no part in the bound.
__global__ void init_eq_kernel(CellArgs a, const double* __restrict__ U0, double* __restrict__ f,
                               DevState* st, int lam_mode, double lam_user, double cfl) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double lam0 = lam_mode == LAM_USER
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
    if (c < a.plane) {
        const long long P = a.plane;
        if (a.model == D2Q4) {
            double U[4], z[16], fs[16];
            for (int k = 0; k < 4; ++k) U[k] = U0[k * P + c];
            for (int p = 0; p < 16; ++p) z[p] = 0.0;
            Euler2 e = euler2(U, a.gamma - 1.0);
            collide_d2q4(z, U, e, 1.0 / (4.0 * lam0), 1.0, fs);
            const bool solid = solid_cell(a, c);
            for (int p = 0; p < 16; ++p) f[cell_ofs(a, p, c)] = solid ? 0.0 : fs[p];
            double Un[4];
            moments_d2q4(fs, Un);
            bound_d2q4(Un, a.gamma, &l);
            if (solid) l = 0.0;
        } else {
            double U[3], z[9], fs[9];
            for (int k = 0; k < 3; ++k) U[k] = U0[k * P + c];
            for (int p = 0; p < 9; ++p) z[p] = 0.0;
            double Un[3];
            if (a.model == D1Q2) {
                collide_1d<2>(z, U, a.gamma - 1.0, 1.0 / (2.0 * lam0), 1.0, fs);
                for (int p = 0; p < 6; ++p) f[cell_ofs(a, p, c)] = fs[p];
                moments_1d<2>(fs, Un);
            } else {
                collide_1d<3>(z, U, a.gamma - 1.0, 1.0 / (2.0 * lam0), 1.0, fs);
                for (int p = 0; p < 9; ++p) f[cell_ofs(a, p, c)] = fs[p];
                moments_1d<3>(fs, Un);
            }
            bound_1d(Un, a.gamma, &l);
        }
    }
    double wm = wave_max(l);
    if ((threadIdx.x & 63) == 0) publish_max(&st->lam[0], wm);
}

// lambda* of given populations into reduction slot 0 (after lbrs_set_f);
// solid cells take no part.
__global__ void bound_of_f_kernel(CellArgs a, const double* __restrict__ f, DevState* st) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    bool bad = false;
    if (c < a.plane && !solid_cell(a, c)) {
        const int Q = nq_of(a.model), K = nk_of(a.model);
        double Uc[4] = {0.0, 0.0, 0.0, 0.0};
        double fc[16];
        for (int p = 0; p < Q * K; ++p) fc[p] = f[cell_ofs(a, p, c)];
        if (a.model == D2Q4) moments_d2q4(fc, Uc);
        else if (a.model == D1Q2) moments_1d<2>(fc, Uc);
        else moments_1d<3>(fc, Uc);
        bad = !cell_bound(a.model, Uc, a.gamma, &l);
    }
    double wm = wave_max(l);
    if ((threadIdx.x & 63) == 0) publish_max(&st->lam[0], wm);
    if (__any(bad) && (threadIdx.x & 63) == 0) {
        atomicOr(&st->bad[0], 1u);
        atomicOr(&st->status, 1u);
    }
}

__global__ void set_slot0_kernel(DevState* st, double t, long long n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->s[0].t = t;
        st->s[0].n = n;
        st->s[0].lam_used = st->lam_fixed;
        st->s[0].cur = 0;
        for (int i = 0; i < 3; ++i) {
            st->lam[i] = 0ull;
            st->bad[i] = 0u;
        }
        st->status = 0u;
        st->fail_step = ~0ull;
    }
}

// U = sum_i f_i of the current buffer (slot `slot` of the time state).
__global__ void moments_kernel(CellArgs a, const double* __restrict__ f0, const double* __restrict__ f1,
                               const DevState* st, int slot, double* __restrict__ U) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.plane) return;
    const double* f = st->s[slot].cur ? f1 : f0;
    const int Q = nq_of(a.model), K = nk_of(a.model);
    double fc[16], Uc[4];
    for (int p = 0; p < Q * K; ++p) fc[p] = f[cell_ofs(a, p, c)];
    if (a.model == D2Q4) moments_d2q4(fc, Uc);
    else if (a.model == D1Q2) moments_1d<2>(fc, Uc);
    else moments_1d<3>(fc, Uc);
    for (int k = 0; k < K; ++k) U[k * a.plane + c] = Uc[k];
}

// U = sum_i f_i of a population pool (no time state: one buffer).
__global__ void pool_moments_kernel(CellArgs a, const double* __restrict__ f, double* __restrict__ U) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.plane) return;
    const int Q = nq_of(a.model), K = nk_of(a.model);
    double fc[16], Uc[4];
    for (int p = 0; p < Q * K; ++p) fc[p] = f[cell_ofs(a, p, c)];
    if (a.model == D2Q4) moments_d2q4(fc, Uc);
    else if (a.model == D1Q2) moments_1d<2>(fc, Uc);
    else moments_1d<3>(fc, Uc);
    for (int k = 0; k < K; ++k) U[k * a.plane + c] = Uc[k];
}

// Copy between the current buffer and an external one (dir 0: out, 1: in to f0).
__global__ void copy_f_kernel(long long count, double* __restrict__ f0, double* __restrict__ f1,
                              const DevState* st, int slot, double* __restrict__ ext, int dir) {
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    if (dir == 0) {
        const double* f = st->s[slot].cur ? f1 : f0;
        ext[j] = f[j];
    } else {
        f0[j] = ext[j];
    }
}

// Density of the current populations at cell c.
__device__ inline double density_at(const CellArgs& a, const double* f, long long c) {
    const int Q = nq_of(a.model), K = nk_of(a.model);
    if (Q == 4)
        return (f[cell_ofs(a, 0 * K, c)] + f[cell_ofs(a, 2 * K, c)]) +
               (f[cell_ofs(a, 1 * K, c)] + f[cell_ofs(a, 3 * K, c)]);
    double rho = 0.0;
    for (int i = 0; i < Q; ++i) rho += f[cell_ofs(a, i * K, c)];
    return rho;
}

// Seed of the adjoint: fbar_{i,rho} = 2 rho inside the window, zero elsewhere
// and in the other components (dJ/df for J = sum_window rho^2, rho = sum_i f_i).
__global__ void window_seed_kernel(CellArgs a, const double* __restrict__ f0,
                                   const double* __restrict__ f1, const DevState* st, int slot,
                                   int ix0, int ix1, int iy0, int iy1, double* __restrict__ fbar) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.plane) return;
    const double* f = st->s[slot].cur ? f1 : f0;
    const int Q = nq_of(a.model), K = nk_of(a.model);
    const int x = (int)(c % a.nx), y = (int)(c / a.nx);
    const bool in = x >= ix0 && x < ix1 && y >= iy0 && y < iy1;
    const double g = in ? 2.0 * density_at(a, f, c) : 0.0;
    for (int i = 0; i < Q; ++i)
        for (int k = 0; k < K; ++k) fbar[cell_ofs(a, i * K + k, c)] = k == 0 ? g : 0.0;
}

// J = sum over the window of rho^2, by one workgroup in a fixed order (the
// result is bitwise reproducible, which finite differences of J rely on).
__global__ __launch_bounds__(1024) void window_sum_kernel(CellArgs a, const double* __restrict__ f0,
                                                          const double* __restrict__ f1,
                                                          const DevState* st, int slot, int ix0,
                                                          int ix1, int iy0, int iy1, double* J) {
    __shared__ double part[16];
    const double* f = st->s[slot].cur ? f1 : f0;
    const long long w = ix1 - ix0, cells = w * (long long)(iy1 - iy0);
    double acc = 0.0;
    for (long long j = threadIdx.x; j < cells; j += blockDim.x) {
        long long c = (long long)(iy0 + j / w) * a.nx + (ix0 + j % w);
        double rho = density_at(a, f, c);
        acc += rho * rho;
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += part[i];
        *J = t;
    }
}

// fbar^n from fbar^{n+1} and U^n (D2Q4, periodic sides):
//   fbar*_i(x) = fbar^{n+1}_i(x + s_i)
//   Ubar = omega [ (1/4) sum_i fbar*_i + (A1^T h_x + A2^T h_y)/(4 lambda) ]
//   fbar^n_i = (1 - omega) fbar*_i + Ubar
__global__ __launch_bounds__(256) void adjoint_step_d2q4(AdjArgs a, const double* __restrict__ Un,
                                                         const double* __restrict__ gn,
                                                         double* __restrict__ g) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.nx) return;
    const long long P = a.plane;
    const int xp = x + 1 < a.nx ? x + 1 : 0, xm = x > 0 ? x - 1 : a.nx - 1;
    const int yp = y + 1 < a.ny ? y + 1 : 0, ym = y > 0 ? y - 1 : a.ny - 1;
    // s1 = (-,-), s2 = (+,-), s3 = (+,+), s4 = (-,+)
    const long long src[4] = {(long long)ym * a.rs + xm, (long long)ym * a.rs + xp,
                              (long long)yp * a.rs + xp, (long long)yp * a.rs + xm};
    double fb[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) fb[i * 4 + k] = gn[(i * 4 + k) * a.ps + src[i]];
    const long long c = (long long)y * a.nx + x;
    double U[4], out[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) U[k] = Un[k * P + c];
    adjoint_cell_d2q4(fb, U, a.gamma, a.omega, a.st->lam_fixed, out);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) g[(i * 4 + k) * a.ps + (long long)y * a.rs + x] = out[i * 4 + k];
}

// Ubar0 = sum_i (df_i^eq/dU)^T fbar0_i at U0 (D2Q4).
__global__ void adjoint_init_d2q4(AdjArgs a, const double* __restrict__ fb0,
                                  const double* __restrict__ U0, double* __restrict__ Ub) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.plane) return;
    const long long P = a.plane;
    double fb[16], U[4], out[4];
    for (int p = 0; p < 16; ++p) fb[p] = fb0[p * a.ps + (c / a.nx) * a.rs + c % a.nx];
    for (int k = 0; k < 4; ++k) U[k] = U0[k * P + c];
    adjoint_init_cell_d2q4(fb, U, a.gamma, a.st->lam_fixed, out);
    for (int k = 0; k < 4; ++k) Ub[k * P + c] = out[k];
}

// ------------------------------------------------------------ launchers
static inline dim3 grid1(long long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

// The time state a sequence of launches left (slot `slot`), as doubles:
// t, completed steps, lattice speed of the last step, status, first
// non-physical step (-1: none).
__global__ void export_state_kernel(const DevState* st, int slot, double* out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const Slot sl = st->s[slot];
        out[0] = sl.t;
        out[1] = (double)sl.n;
        out[2] = sl.lam_used;
        out[3] = (double)st->status;
        out[4] = st->fail_step == ~0ull ? -1.0 : (double)st->fail_step;
    }
}

hipError_t launch_export_state(const DevState* st, int slot, double* out, hipStream_t s) {
    hipLaunchKernelGGL(export_state_kernel, dim3(1), dim3(64), 0, s, st, slot, out);
    return hipGetLastError();
}

hipError_t launch_reset(DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(reset_state_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}
hipError_t launch_prim_to_cons(const CellArgs& a, const double* W, double* U, hipStream_t s) {
    hipLaunchKernelGGL(prim_to_cons_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, W, U);
    return hipGetLastError();
}
hipError_t launch_prim_to_cons_adjoint(const CellArgs& a, const double* W, const double* Ub,
                                       double* Wb, hipStream_t s) {
    hipLaunchKernelGGL(prim_to_cons_adjoint_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, W, Ub, Wb);
    return hipGetLastError();
}
hipError_t launch_isentropic_to_cons(const CellArgs& a, const double* rho, double* U, hipStream_t s) {
    hipLaunchKernelGGL(isentropic_to_cons_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, rho, U);
    return hipGetLastError();
}
hipError_t launch_isentropic_to_cons_adjoint(const CellArgs& a, const double* rho, const double* Ub,
                                             double* rb, hipStream_t s) {
    hipLaunchKernelGGL(isentropic_to_cons_adjoint_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, rho,
                       Ub, rb);
    return hipGetLastError();
}
hipError_t launch_init(const CellArgs& a, const double* U0, double* f0, DevState* st, int lam_mode,
                       double lam_user, double cfl, const double* const dir[4], hipStream_t s) {
    hipLaunchKernelGGL(bound_of_U_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, U0, st);
    DirSides ds;
    bool any = false;
    for (int k = 0; k < 4; ++k) {
        ds.d[k] = dir ? dir[k] : nullptr;
        any = any || ds.d[k];
    }
    if (any)
        hipLaunchKernelGGL(dirichlet_bound_kernel, grid1(2LL * (a.nx + a.ny), 256), dim3(256), 0, s, a,
                           ds, st);
    hipLaunchKernelGGL(init_eq_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, U0, f0, st, lam_mode,
                       lam_user, cfl);
    return hipGetLastError();
}
hipError_t launch_set_f(const CellArgs& a, double* f0, double* f1, DevState* st, const double* ext,
                        double t, long long n, bool per_step, hipStream_t s) {
    const int Q = nq_of(a.model), K = a.law == LAW_SCALAR ? 1 : nk_of(a.model);
    long long cnt = (long long)Q * K * (a.fcells > 0 ? a.fcells : a.plane);
    hipLaunchKernelGGL(set_slot0_kernel, dim3(1), dim3(64), 0, s, st, t, n);
    hipLaunchKernelGGL(copy_f_kernel, grid1(cnt, 256), dim3(256), 0, s, cnt, f0, f1, st, 0,
                       const_cast<double*>(ext), 1);
    if (per_step) {
        if (a.law == LAW_SCALAR) return launch_scalar_bound_f(a, f0, st, s);
        hipLaunchKernelGGL(bound_of_f_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, f0, st);
    }
    return hipGetLastError();
}
hipError_t launch_get_f(const CellArgs& a, double* f0, double* f1, const DevState* st, int slot,
                        double* ext, hipStream_t s) {
    const int Q = nq_of(a.model), K = a.law == LAW_SCALAR ? 1 : nk_of(a.model);
    long long cnt = (long long)Q * K * (a.fcells > 0 ? a.fcells : a.plane);
    hipLaunchKernelGGL(copy_f_kernel, grid1(cnt, 256), dim3(256), 0, s, cnt, f0, f1, st, slot, ext, 0);
    return hipGetLastError();
}
hipError_t launch_moments(const CellArgs& a, const double* f0, const double* f1, const DevState* st,
                          int slot, double* U, hipStream_t s) {
    hipLaunchKernelGGL(moments_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, f0, f1, st, slot, U);
    return hipGetLastError();
}
hipError_t launch_window_objective(const CellArgs& a, const double* f0, const double* f1,
                                   DevState* st, int slot, int ix0, int ix1, int iy0, int iy1,
                                   double* J, double* fbar, hipStream_t s) {
    hipLaunchKernelGGL(window_sum_kernel, dim3(1), dim3(1024), 0, s, a, f0, f1, st, slot, ix0, ix1,
                       iy0, iy1, J);
    hipLaunchKernelGGL(window_seed_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, f0, f1, st, slot,
                       ix0, ix1, iy0, iy1, fbar);
    return hipGetLastError();
}
hipError_t launch_pool_moments(const CellArgs& a, const double* f, double* U, hipStream_t s) {
    hipLaunchKernelGGL(pool_moments_kernel, grid1(a.plane, 256), dim3(256), 0, s, a, f, U);
    return hipGetLastError();
}
hipError_t launch_adjoint_step(const AdjArgs& a, const double* Un, const double* gn, double* g,
                               hipStream_t s) {
    dim3 grid((a.nx + 255) / 256, a.ny);
    hipLaunchKernelGGL(adjoint_step_d2q4, grid, dim3(256), 0, s, a, Un, gn, g);
    return hipGetLastError();
}
hipError_t launch_adjoint_init(const AdjArgs& a, const double* fb0, const double* U0, double* Ub,
                               hipStream_t s) {
    hipLaunchKernelGGL(adjoint_init_d2q4, grid1(a.plane, 256), dim3(256), 0, s, a, fb0, U0, Ub);
    return hipGetLastError();
}

}  // namespace lbrs
