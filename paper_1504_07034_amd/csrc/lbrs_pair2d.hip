// Fused LBRS launches of up to four steps for the 2D Euler equations (D2Q4,
// gfx950).
//
// The single-step kernel reads f^n and writes f^{n+1} once per step: 256 B of
// HBM traffic per cell and step, which bounds it.  Here a wavefront feeds
// every row of f^{n+1} it has just streamed straight into the next collision
// and streaming, k times, so f^n is read once and f^{n+k} written once: 256/k
// B per cell and step.  Every step is the scheme of Sec. II.D unchanged
// (moments, the folded equilibria, relaxation, exact diagonal hops, Sec. II.E
// walls, transmissive and periodic sides); nothing but the order of the work
// differs.
//
// Lanes and rows.  Lane l holds column x0 - k + l; step s (0-based) is valid
// on lanes s+1 .. 62-s, so a strip has <= 64 - 2k output columns.  A tile
// reads rows y0-k .. y1+k-1 of f^n; step s completes rows from y0-k+1+s on,
// the last step rows y0 .. y1-1 of f^{n+k}.  Pipelines: the upward hops of
// the last two rows of each step (the older one in LDS for three or more
// steps), and the next row of f^n in flight.  Between steps every
// intermediate state obeys the side rules: beyond a clamped (transmissive or
// wall) side the next step pulls from the edge cell of that state itself
// (the edge column's values copied into the halo lane, the edge row's hops
// reused), in every strip and segment whose lanes or rows reach the side.
//
// Lattice speeds of the later steps.  With a fixed speed they are known.
// With the per-step speed each is the global bound over the state before it,
// which no workgroup has before the launch ends.  The launch then guesses
// them (the predictions the launch before left, else the current bound while
// it keeps repeating), reduces the true bound of every intermediate state on
// the side, and leaves its result tentative.  The next launch checks every
// guess: all equal bit for bit (and the states admissible) means the k steps
// are exactly those of k single steps, and it continues from f^{n+k};
// otherwise f^n, still intact in the other buffer, is current again, and
// that launch redoes the steps with the bounds now known (up to the first
// wrong guess; up to a non-physical state).  Where nothing can be guessed a
// launch first reduces the bound of f^{n+1} alone.  Every workgroup of a
// launch takes the same decisions from the same slots, so no grid barrier is
// needed.  The last launch of a call never leaves a tentative result, so
// every other call sees an ordinary time state.  The predictions: after each
// launch, one small kernel per predicted step evaluates the exact bound of
// the next states on patches around the cells where the bound peaks.
//
// Also here: the taped form (U of every step's input for the gradients'
// recompute) and the 2D batch's form over all domains (fixed speeds).
#include "lbrs_launch.hpp"
#include "lbrs_rowops.hpp"

namespace lbrs {

namespace {

// Post-collision values of one row moved one lane along their diagonal:
// populations 0 (-,-) and 1 (+,-) travel to the row below, 2 (+,+) and
// 3 (-,+) to the row above.
struct Hops {
    double d0[4], d1[4];  // f0*(x+1, r), f1*(x-1, r): pulled by row r-1
    double u2[4], u3[4];  // f2*(x-1, r), f3*(x+1, r): pulled by row r+1
};

// Collision of one row (moments U given) and its hops.
__device__ inline void collide_hops(const double f[16], const double U[4], double gm1, double c4lam,
                                    double omega, Hops& h) {
    const Euler2 e = euler2(U, gm1);
    double fs[16];
    collide_d2q4(f, U, e, c4lam, omega, fs);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        h.d0[k] = lane_from_right(fs[0 * 4 + k]);
        h.d1[k] = lane_from_left(fs[1 * 4 + k]);
        h.u2[k] = lane_from_left(fs[2 * 4 + k]);
        h.u3[k] = lane_from_right(fs[3 * 4 + k]);
    }
}

// Free-slip wall on a node row or column (Sec. II.E): the populations that
// would come from beyond the wall are the mirror images of the outgoing ones,
// normal momentum negated.
__device__ inline void wall_images(double g[16], bool top, bool bot, bool xlo, bool xhi) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double ry = k == 2 ? -1.0 : 1.0, rx = k == 1 ? -1.0 : 1.0;
        if (top) {
            g[0 * 4 + k] = ry * g[3 * 4 + k];
            g[1 * 4 + k] = ry * g[2 * 4 + k];
        }
        if (bot) {
            g[3 * 4 + k] = ry * g[0 * 4 + k];
            g[2 * 4 + k] = ry * g[1 * 4 + k];
        }
        if (xlo) {
            g[1 * 4 + k] = rx * g[0 * 4 + k];
            g[2 * 4 + k] = rx * g[3 * 4 + k];
        }
        if (xhi) {
            g[0 * 4 + k] = rx * g[1 * 4 + k];
            g[3 * 4 + k] = rx * g[2 * 4 + k];
        }
    }
}

struct PairGeom {
    const double* fin;
    double* fout;
    long long ps, rs;
    int nx, ny, strip;
    double c4lam[KMAX_STEPS];  // 1/(4 lambda) of each step
    double omega, gamma;
    int bc[4];
    double* tape[KMAX_STEPS];  // TAPE: U^{n+s} of step s's input, element (k, y, x) at
    long long tape_ps;         // k*tape_ps + y*nx + x
    // CAND: the floor of the candidates' bounds, this launch's header and
    // where candidates go
    double t0;
    PredHeader* ph;
    PredCand* cand;
};

// A wave-uniform double, moved to scalar registers.
__device__ inline double uniform(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ inline void load_row(double v[16], const double* __restrict__ fin, long long ps,
                                long long rs, int j, int xl) {
    const double* __restrict__ row = fin + (long long)j * rs;
#pragma unroll
    for (int p = 0; p < 16; ++p) v[p] = row[p * ps + xl];
}

__device__ inline void store_full_row(double* row, long long ps, int row_bytes, int voff,
                                      const double g[16]) {
#pragma unroll
    for (int p = 0; p < 16; ++p) store_row(row + p * ps, row_bytes, voff, g[p]);
}

// Moments of row j of a tape (rows [y0, y1) of the tile only: other rows
// and lanes carry an out-of-range offset, so the store is unconditional).
__device__ inline void tape_row(double* tape, long long tape_ps, int nx, int j, int y0, int y1,
                                int voff, const double U[4]) {
    const bool own = j >= y0 && j < y1;
    double* row = tape + (long long)(own ? j : y0) * nx;
#pragma unroll
    for (int k = 0; k < 4; ++k) store_row(row + k * tape_ps, nx * 8, own ? voff : 0x7fffffff, U[k]);
}

// K fused steps of rows y0..y1-1 of one strip (K = 1: a single step).  Lane
// l holds column x0 - K + l; step s (0-based) is valid on lanes s+1 .. 62-s,
// so a strip has <= 64 - 2K output columns.  Row r of f^n (read once)
// enters step 0; step s takes row j = r - s of f^{n+s} and completes row
// j - 1 of f^{n+s+1}, which goes straight into step s+1: the downward hops
// (populations 0, 1) come from row j, the upward hops (2, 3) from row j - 2,
// kept in the step's two-row register pipeline.  Rows y0-K .. y1+K-1 of f^n
// are read, so step s produces rows y0-K+s .. y1+K-2-s; the first rows of
// each pipeline start as zeros and only feed rows that are never used.
// After step s < K-1, at a clamped (transmissive or wall) side, the next
// step must pull from the edge cell of f^{n+s+1} itself, not from a ghost
// that this step would make up: the halo lane beyond a clamped x side takes
// the edge column's values; at a clamped bottom, row -1 is row 0 again (its
// upward hops stand in), at a clamped top row ny is row ny-1 again (its
// downward hops are kept for the virtual row).  Walls overwrite the pulls
// across them.  lm[s]/bad[s] gather the bound and admissibility of this
// tile's cells of f^{n+s+1}; TAPE stores U^{n+s} of every step's input;
// CAND lists candidates from the last step's output (see PredCand).  One
// copy of the step code serves every row and step of a kernel's path, so
// all cells round alike.  EARLY: a wave sends the next row's loads before it
// waits at the workgroup barrier (else after).
template <int WPB, int K, bool TAPE, bool CAND = false, bool LPB = false, bool EARLY = true>
__device__ __forceinline__ void march_k(const PairGeom& g, int strip, int y0, int y1, int lane,
                                        double (&lm)[KMAX_STEPS], bool (&bad)[KMAX_STEPS],
                                        bool store = true, double* pbl = nullptr) {
    static_assert(K >= 1 && K <= KMAX_STEPS, "steps per launch");
    static_assert(!CAND || !TAPE, "candidates ride on plain launches");
    const int nx = g.nx, ny = g.ny;
    const bool px = g.bc[0] == BC_PERIODIC, py = g.bc[2] == BC_PERIODIC;
    const double gm1 = g.gamma - 1.0;
    const int row_bytes = nx * 8;
    const int x0 = strip * g.strip;
    const int x = x0 - K + lane;
    const int xl = map_index(x, nx, px);
    const bool out_lane = lane >= K && lane <= g.strip + K - 1 && x < nx;
    const int voff = out_lane ? x * 8 : 0x7fffffff;
    const bool wxlo = g.bc[0] == BC_WALL && x == 0;
    const bool wxhi = g.bc[1] == BC_WALL && x == nx - 1;
    const bool wlo = g.bc[2] == BC_WALL, whi = g.bc[3] == BC_WALL;
    // Wave-uniform: the strip's lanes (halo lanes included) hold a wall
    // column; they hold the ghost column x = -1 or x = nx of a clamped x
    // side.  Every column and row a tile computes is a true cell of its
    // state (halo ones feed the next steps), so the side rules apply to each,
    // also in a strip or segment that does not begin at the side.
    const bool xwall = (g.bc[0] == BC_WALL && x0 - K <= 0) ||
                       (g.bc[1] == BC_WALL && x0 + 63 - K >= nx - 1);
    const bool xfix = K > 1 && !px && (x0 - K < 0 || x0 + 63 - K >= nx);
    const bool clamp_lo = K > 1 && !py;
    const bool clamp_hi = K > 1 && !py;

    // per step: upward hops (u2, u3) of the last input row (PA) and of the
    // one before (PB); at a clamped top PA keeps row ny-1's downward hops.
    // LPB: PB lives in the wave's LDS area pbl instead of registers, element
    // k of step st at pbl[(st*8 + k)*64 + lane] (each lane reads and writes
    // only its own elements, in program order: no barrier)
    double PA[K][8], PB[LPB ? 1 : K][8];
#pragma unroll
    for (int st = 0; st < K; ++st)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            PA[st][k] = 0.0;
            if (LPB) pbl[(st * 8 + k) * 64 + lane] = 0.0;
            else PB[st][k] = 0.0;
        }

    // CAND: candidates for the prediction of the next launch's bounds (see
    // PredCand).  A row's cells are decided when the row after it is known:
    // l of rows o-1 (lp, pending) and o-2 (lpp) in this lane, -1 outside the
    // tile; the wave's largest bound so far, the threshold CAND_REL below it
    // (at least the launch's floor), and the first lane of the pending row
    // that raised the largest bound (-1: none) -- wave-uniform, in scalar
    // registers.  Each lane keeps the largest cell of its column that
    // qualified (cbest, row crow; -1: none) and lists it when the tile ends:
    // nothing but selects in the row loop.
    double thr = CAND ? g.t0 : 0.0, wmax = 0.0, lp = -1.0, lpp = -1.0, cbest = -1.0;
    int rec_prev = -1, crow = 0;
    auto candidates = [&](double lc, int o) {
        int rec_cur = -1;
        if (__any(lc > thr)) {
            const double rowmax = uniform(wave_max(lc));
            if (rowmax > wmax) {
                rec_cur = __builtin_amdgcn_readfirstlane(
                    __ffsll((long long)__ballot(lc == rowmax)) - 1);
                wmax = rowmax;
                thr = uniform(fmax(g.t0, wmax * (1.0 - CAND_REL)));
            }
        }
        // row o-1: a cell qualifies when its bound is above the threshold and
        // no neighbour's exceeds it (a neighbour outside the tile is
        // ignored), except inside a flat region, which leaves only the cell
        // that first reached its value
        if (__any(lp > thr)) {
            const double ll = lane_from_left(lp), lr = lane_from_right(lp);
            const bool top = (ll < 0.0 || lp >= ll) && (lr < 0.0 || lp >= lr) &&
                             (lpp < 0.0 || lp >= lpp) && (lc < 0.0 || lp >= lc);
            const bool flat = (ll < 0.0 || lp == ll) && (lr < 0.0 || lp == lr) &&
                              (lpp < 0.0 || lp == lpp) && (lc < 0.0 || lp == lc);
            const bool take = lp > thr && top && (!flat || lane == rec_prev) && lp > cbest;
            cbest = take ? lp : cbest;
            crow = take ? o - 1 : crow;
        }
        rec_prev = rec_cur;
        lpp = lp;
        lp = lc;
    };
    auto list_candidates = [&]() {
        const bool emit = cbest > thr;
        const unsigned long long m = __ballot(emit);
        if (m) {
            unsigned base = 0;
            if (lane == 0) base = atomicAdd(&g.ph->ncand, (unsigned)__popcll(m));
            base = __shfl(base, 0, 64);
            if (emit) {
                const unsigned idx = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
                if (idx < (unsigned)PRED_CAP) {
                    g.cand[idx].cell = (long long)crow * nx + x;
                    g.cand[idx].l = cbest;
                }
            }
        }
    };

    // Lockstep with the workgroup's neighbouring strips (equal trip counts
    // and the same rows, so every wave meets the same barriers): a barrier
    // at every row, or every second row with four steps per launch, where
    // the longer rows make the looser lockstep faster while the strips still
    // share the halo columns' reads in cache (with no barrier at all the
    // reads from HBM triple).  The barrier carries no memory order (the
    // waves exchange nothing), so a wave's next-row loads can go out before
    // it waits there: faster for every form measured but the batch's three
    // steps, which passes EARLY = false.
    constexpr int ROW_SYNC = K >= 4 ? 2 : 1;
    double cur[16], nxt[16], Uc[4];
    load_row(nxt, g.fin, g.ps, g.rs, map_index(y0 - K, ny, py), xl);
    for (int r = y0 - K; r <= y1 + K - 1; ++r) {
        const bool sync = WPB > 1 && (r & (ROW_SYNC - 1)) == 0;
        if (!EARLY && sync) __builtin_amdgcn_s_barrier();
#pragma unroll
        for (int p = 0; p < 16; ++p) cur[p] = nxt[p];
        // row r+1 in flight while row r is computed
        load_row(nxt, g.fin, g.ps, g.rs, map_index(r + 1, ny, py), xl);
        if (EARLY && sync) __builtin_amdgcn_s_barrier();
        moments_d2q4(cur, Uc);
        if (TAPE) tape_row(g.tape[0], g.tape_ps, nx, r, y0, y1, voff, Uc);  // U^n of row r
#pragma unroll
        for (int st = 0; st < K; ++st) {
            const int j = r - st;  // input row of step st
            const int o = j - 1;   // its output row
            const Euler2 e = euler2(Uc, gm1);
            double fs[16];
            collide_d2q4(cur, Uc, e, g.c4lam[st], g.omega, fs);
            double d0[4], d1[4], u2[4], u3[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                d0[k] = lane_from_right(fs[0 * 4 + k]);
                d1[k] = lane_from_left(fs[1 * 4 + k]);
                u2[k] = lane_from_left(fs[2 * 4 + k]);
                u3[k] = lane_from_right(fs[3 * 4 + k]);
            }
            // output row o: the downward movers of row j (at a clamped top,
            // for the virtual row ny, those kept from row ny-1), the upward
            // movers of row j-2
            const bool topv = st > 0 && clamp_hi && j == ny;
            const bool lo_edge = st > 0 && clamp_lo && j == 0;
            const bool hi_edge = st > 0 && clamp_hi && j == ny - 1;
            const bool wtop = whi && o == ny - 1, wbot = wlo && o == 0;
            // the rows at a clamped side or a wall and the strips with a wall
            // column take the general form; the others (wave-uniform branch)
            // plain hops with no selects
            double gq[16];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                gq[0 * 4 + k] = d0[k];
                gq[1 * 4 + k] = d1[k];
            }
            double b23[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) b23[k] = PA[st][k];
            if (topv || lo_edge || hi_edge) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    gq[0 * 4 + k] = topv ? PA[st][k] : gq[0 * 4 + k];
                    gq[1 * 4 + k] = topv ? PA[st][4 + k] : gq[1 * 4 + k];
                    b23[k] = lo_edge ? u2[k] : b23[k];
                    b23[4 + k] = lo_edge ? u3[k] : b23[4 + k];
                    u2[k] = hi_edge ? d0[k] : u2[k];
                    u3[k] = hi_edge ? d1[k] : u3[k];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (LPB) {
                    double* e2 = pbl + (st * 8 + k) * 64 + lane;
                    double* e3 = pbl + (st * 8 + 4 + k) * 64 + lane;
                    gq[2 * 4 + k] = *e2;
                    gq[3 * 4 + k] = *e3;
                    *e2 = b23[k];
                    *e3 = b23[4 + k];
                } else {
                    gq[2 * 4 + k] = PB[LPB ? 0 : st][k];
                    gq[3 * 4 + k] = PB[LPB ? 0 : st][4 + k];
                    PB[LPB ? 0 : st][k] = b23[k];
                    PB[LPB ? 0 : st][4 + k] = b23[4 + k];
                }
                PA[st][k] = u2[k];
                PA[st][4 + k] = u3[k];
            }
            if (wtop || wbot || xwall) wall_images(gq, wtop, wbot, wxlo, wxhi);
            if (st < K - 1 && xfix) {
                // a clamped side: beyond it, the next step pulls the edge column's values
#pragma unroll
                for (int p = 0; p < 16; ++p) {
                    const double fr = lane_from_right(gq[p]);
                    const double fl = lane_from_left(gq[p]);
                    gq[p] = x == -1 ? fr : (x == nx ? fl : gq[p]);
                }
            }
            double U1[4], l1;
            moments_d2q4(gq, U1);
            const bool own = out_lane && o >= y0 && o < y1;
            // the bounds are needed with per-step speeds only, which always
            // run the form that lists candidates; the others test
            // admissibility alone (no square root, one division fewer)
            bool ok;
            if constexpr (CAND) {
                ok = bound_d2q4(U1, g.gamma, &l1);
            } else {
                ok = admissible_d2q4(U1, euler2(U1, gm1));
                l1 = 0.0;
            }
            bad[st] |= own && !ok;
            lm[st] = fmax(lm[st], own ? l1 : 0.0);
            if (st == K - 1) {
                // an output row of the tile; the store is unconditional (an
                // out-of-range offset is dropped by the buffer range check),
                // so the wait for the next row's loads never has to cover it
                const bool row_out = store && o >= y0 && o < y1;
                store_full_row(g.fout + (long long)(row_out ? o : y0) * g.rs, g.ps, row_bytes,
                               row_out ? voff : 0x7fffffff, gq);
                if (CAND) candidates(own && ok ? l1 : -1.0, o);
            } else {
                if (TAPE) tape_row(g.tape[st + 1], g.tape_ps, nx, o, y0, y1, voff, U1);
#pragma unroll
                for (int p = 0; p < 16; ++p) cur[p] = gq[p];
#pragma unroll
                for (int k = 0; k < 4; ++k) Uc[k] = U1[k];
            }
        }
    }
    if (CAND) {
        // the tile's last row is decided without the row after it
        candidates(-1.0, y1);
        list_candidates();
    }
}

__device__ inline double from_bits(unsigned long long b) { return __longlong_as_double((long long)b); }


// dt and the lattice speed of one step, in the order of operations of the
// single-step control (so that both produce the same bits).
__device__ __forceinline__ void step_size(int lam_mode, double lam_star, double lam_fixed, double dx,
                                 double cfl, double t, double t_end, double& lam, double& t_new) {
    if (lam_mode == LAM_PER_STEP) {
        double dt = cfl * dx / lam_star;
        const double rem = t_end - t;
        bool last = false;
        if (dt >= rem) {
            dt = rem;
            last = true;
        }
        lam = dx / dt;
        t_new = last ? t_end : t + dt;
    } else {
        lam = lam_fixed;
        t_new = t + dx / lam;
    }
}

// Time control of one fused launch (identical in every thread).  Written
// out for up to four steps, in scalars: a local array indexed by a run-time
// step count would live in scratch memory.
static_assert(KMAX_STEPS == 4, "the launch control is written out for four steps");

struct PairCtl {
    bool active;        // at least one step, or a bound-only pass
    int k;              // steps of this launch (0: none; a bound-only launch has k = 0)
    bool tentative;     // the result waits for the next launch's check
    bool bound;         // this launch only reduces the bound of f^{n+1}
    bool accepted_bad;  // the previous launch's result stands, with a non-physical last state
    bool predicted;     // this launch's guesses are predictions
    bool cand;          // this launch lists candidates for the next launch's predictions
    int trust;          // saturating count of repeated bounds at the last checks (0..3)
    int check;          // outcome of the check of the previous launch (for the counters):
                        // 0 none, 1 accepted, 2 predicted and accepted, 3 rejected,
                        // 4 predicted and rejected
    int checked_k;      // steps of the checked result
    int cur;
    long long n;
    double t, lam_used;
    unsigned long long lstar;         // bits of lambda*_n (the current state's bound)
    unsigned long long g1, g2, g3;    // bits of lambda*_{n+1..n+3} taken (guessed or known)
                                      // for steps 2..4
    unsigned bad;
    double lam1, lam2, lam3, lam4;    // lattice speed of steps 1..4
    double t1, t2, t3, t4;            // time after them
    double t_out, lam_out;            // time after the last step, its speed
    double t0;                        // floor of the candidates' bounds
    int pred_n;                       // predictions the record read holds for the state
    unsigned long long p1, p2, p3;
};

__device__ __forceinline__ PairCtl pair_control(const Pair2DArgs& a, LaunchSlots ls) {
    const DevState* st = a.st;
    const PairState* ps = a.pst;
    const bool per_step = a.lam_mode == LAM_PER_STEP;
    PairCtl c;
    Slot s = st->s[ls.sr];
    // the record read field by field (a copy of the struct would go through
    // scratch memory)
    const PairSlot& q = ps->q[ls.sr];
    unsigned long long lstar = st->lam[ls.lr];
    unsigned bad = st->bad[ls.lr];
    // exact bounds of the states after steps 1 .. known of this launch
    int known = 0;
    unsigned long long next1 = 0ull, next2 = 0ull, next3 = 0ull;
    int force_k = 0;  // > 0: take exactly these steps (a non-physical state at the last)
    int trust = q.trust;
    // the previous launch left predictions for the state it produced
    int pred_n = q.pred_valid;
    const unsigned long long qp1 = q.pred[1], qp2 = q.pred[2], qp3 = q.pred[3];
    if (pred_n > 0 && qp1 == 0ull) pred_n = 0;
    if (pred_n > 1 && qp2 == 0ull) pred_n = 1;
    if (pred_n > 2 && qp3 == 0ull) pred_n = 2;
    c.accepted_bad = false;
    c.check = 0;
    c.checked_k = q.tentative;
    if (q.tentative > 0) {
        // the first intermediate state that was non-physical or whose bound
        // differs from the guess (0: none)
        const int kt = q.tentative;
        const unsigned long long m1 = ps->lamk[0][ls.lr], m2 = ps->lamk[1][ls.lr],
                                 m3 = ps->lamk[2][ls.lr];
        const bool b1 = ps->badk[0][ls.lr] != 0u, b2 = kt >= 3 && ps->badk[1][ls.lr] != 0u,
                   b3 = kt >= 4 && ps->badk[2][ls.lr] != 0u;
        int fail = 0;
        bool fail_bad = false;
        next1 = m1;
        if (b1) {
            fail = 1;
            fail_bad = true;
        } else if (per_step && m1 != q.guess[1]) {
            fail = 1;
        } else if (kt >= 3) {
            next2 = m2;
            if (b2) {
                fail = 2;
                fail_bad = true;
            } else if (per_step && m2 != q.guess[2]) {
                fail = 2;
            } else if (kt >= 4) {
                next3 = m3;
                if (b3) {
                    fail = 3;
                    fail_bad = true;
                } else if (per_step && m3 != q.guess[3]) {
                    fail = 3;
                }
            }
        }
        const bool ok = fail == 0;
        if (!q.predicted && !b1) trust = ok ? min(trust + 1, 3) : max(trust - 1, 0);
        c.check = ok ? (q.predicted ? 2 : 1) : (q.predicted ? 4 : 3);
        if (ok) {
            c.accepted_bad = bad != 0u;
        } else {
            // back to f^n, knowing the bounds up to the failing state
            s.t = q.t_base;
            s.n = q.n_base;
            s.cur = q.cur_base;
            lstar = q.guess_base;
            bad = 0u;
            if (fail_bad) {
                force_k = fail;
                known = fail - 1;
            } else {
                known = fail;
            }
            pred_n = 0;
        }
    } else if (q.known) {
        // the previous launch reduced the bound of f^{n+1} of this state
        const unsigned long long m1 = ps->lamk[0][ls.lr];
        const bool b1 = ps->badk[0][ls.lr] != 0u;
        if (b1) {
            force_k = 1;
        } else {
            known = 1;
            next1 = m1;
            trust = m1 == lstar ? min(trust + 1, 3) : max(trust - 1, 0);
        }
        pred_n = 0;
    }
    c.cur = s.cur;
    c.n = s.n;
    c.t = s.t;
    c.lam_used = s.lam_used;
    c.lstar = lstar;
    c.bad = bad;
    const long long n_limit = ps->n_limit;
    c.active = bad == 0u && s.t < a.t_end && s.n < n_limit;
    const unsigned long long lbc = st->lam_bc;
    // the most steps the time, the step limit and a forced count allow
    int kcap = a.kmax;
    if (force_k > 0 && force_k < kcap) kcap = force_k;
    if (s.n + kcap > n_limit) kcap = (int)(n_limit - s.n);
    // where the speeds of steps 2.. come from: known bounds, else
    // predictions, else the current bound while it has been repeating (a
    // guess), else a bound-only pass first
    const bool use_pred = per_step && known == 0 && pred_n > 0;
    int kguess;  // steps reachable with known or guessed speeds
    if (!per_step) kguess = KMAX_STEPS;
    else if (known > 0) kguess = known + 1;
    else if (use_pred) kguess = pred_n + 1;
    else kguess = trust > 0 ? KMAX_STEPS : 1;
    if (kcap > kguess) kcap = kguess;
    c.g1 = known >= 1 ? next1 : (use_pred ? qp1 : lstar);
    c.g2 = known >= 2 ? next2 : (use_pred ? qp2 : lstar);
    c.g3 = known >= 3 ? next3 : (use_pred ? qp3 : lstar);
    const double fix = st->lam_fixed;
    step_size(a.lam_mode, from_bits(lstar > lbc ? lstar : lbc), fix, a.dx, a.cfl, s.t, a.t_end,
              c.lam1, c.t1);
    step_size(a.lam_mode, from_bits(c.g1 > lbc ? c.g1 : lbc), fix, a.dx, a.cfl, c.t1, a.t_end,
              c.lam2, c.t2);
    step_size(a.lam_mode, from_bits(c.g2 > lbc ? c.g2 : lbc), fix, a.dx, a.cfl, c.t2, a.t_end,
              c.lam3, c.t3);
    step_size(a.lam_mode, from_bits(c.g3 > lbc ? c.g3 : lbc), fix, a.dx, a.cfl, c.t3, a.t_end,
              c.lam4, c.t4);
    // each step runs when the one before did, it is within the caps and the
    // time before it is short of t_end
    c.k = 0;
    if (c.active && kcap >= 1) c.k = 1;
    if (c.k == 1 && kcap >= 2 && c.t1 < a.t_end) c.k = 2;
    if (c.k == 2 && kcap >= 3 && c.t2 < a.t_end) c.k = 3;
    if (c.k == 3 && kcap >= 4 && c.t3 < a.t_end) c.k = 4;
    // an intermediate state whose bound is not yet known: the speed after it
    // is a guess (per-step speeds), or its positivity is unchecked
    c.tentative = c.k >= 2 && c.k - 1 > known;
    c.predicted = c.tentative && use_pred;
    // per-step speeds with nothing to guess from: reduce the bound first
    c.bound = per_step && c.active && known == 0 && !use_pred && trust == 0 && force_k == 0 &&
              a.kmax >= 2 && s.n + 2 <= n_limit && c.t1 < a.t_end;
    if (c.bound) c.k = 0;
    // the last launch of a call leaves an ordinary time state
    if (a.last && (c.tentative || c.bound)) {
        c.k = c.bound ? 1 : (per_step ? min(c.k, known + 1) : 1);
        c.tentative = c.bound = c.predicted = false;
    }
    c.trust = trust;
    c.t_out = c.k == 4 ? c.t4 : (c.k == 3 ? c.t3 : (c.k == 2 ? c.t2 : c.t1));
    c.lam_out = c.k == 4 ? c.lam4 : (c.k == 3 ? c.lam3 : (c.k == 2 ? c.lam2 : c.lam1));
    // candidates for the predictions of the next launch's bounds: bounds of
    // the state this launch leaves from CAND_REL below the last known or
    // guessed one up
    c.cand = c.active && c.k > 0 && per_step && a.cand != nullptr && c.t_out < a.t_end;
    const unsigned long long lref =
        c.k == 4 ? c.g3 : (c.k == 3 ? c.g2 : (c.k == 2 ? c.g1 : lstar));
    c.t0 = c.cand ? from_bits(lref) * (1.0 - CAND_REL) : 0.0;
    c.pred_n = pred_n;
    c.p1 = qp1;
    c.p2 = qp2;
    c.p3 = qp3;
    return c;
}

// Block 0, thread 0: the time state after this launch and its record;
// clears the accumulators of launch p+2; arms the prediction kernels.
__device__ __forceinline__ void publish_pair(const Pair2DArgs& a, LaunchSlots ls, const PairCtl& c) {
    DevState* st = a.st;
    PairState* ps = a.pst;
    Slot s;
    s.pad = 0;
    // written field by field into the slot (see pair_control)
    PairSlot& q = ps->q[ls.sw];
    q.t_base = c.t;
    q.n_base = c.n;
    q.cur_base = c.cur;
    q.guess[0] = 0ull;
    q.guess[1] = c.k >= 2 ? c.g1 : 0ull;
    q.guess[2] = c.k >= 3 ? c.g2 : 0ull;
    q.guess[3] = c.k >= 4 ? c.g3 : 0ull;
    q.pred[0] = q.pred[1] = q.pred[2] = q.pred[3] = 0ull;
    q.guess_base = c.lstar;
    q.tentative = 0;
    q.known = 0;
    q.trust = c.trust;
    q.pred_valid = 0;
    q.predicted = c.predicted ? 1 : 0;
    if (!c.active) {
        s.t = c.t;
        s.n = c.n;
        s.lam_used = c.lam_used;
        s.cur = c.cur;
        st->lam[ls.la] = c.lstar;
        st->bad[ls.la] = c.bad;
        // the state stays: so do predictions for it (also into the next call)
        q.pred_valid = c.pred_n;
        q.pred[1] = c.p1;
        q.pred[2] = c.p2;
        q.pred[3] = c.p3;
    } else if (c.bound) {
        // no step: the state and its bound carry over; the first intermediate
        // accumulators receive the bound of f^{n+1}
        s.t = c.t;
        s.n = c.n;
        s.lam_used = c.lam_used;
        s.cur = c.cur;
        st->lam[ls.la] = c.lstar;
        st->bad[ls.la] = 0u;
        q.known = 1;
    } else {
        s.t = c.t_out;
        s.n = c.n + c.k;
        s.lam_used = c.lam_out;
        s.cur = c.cur ^ 1;
        q.tentative = c.tentative ? c.k : 0;
    }
    st->s[ls.sw] = s;
    st->lam[ls.lz] = 0ull;
    st->bad[ls.lz] = 0u;
#pragma unroll
    for (int i = 0; i < KMAX_STEPS - 1; ++i) {
        ps->lamk[i][ls.lz] = 0ull;
        ps->badk[i][ls.lz] = 0u;
    }
    // this launch's candidate header (its candidate count was cleared by the
    // launch before) and the next launch's, whose last user, the prediction
    // after the launch before, has finished
    PredHeader& h = ps->pred[a.launch & 1];
    h.armed = c.cand ? 1 : 0;
    h.cur_out = c.cur ^ 1;
    h.t_out = c.t_out;
    PredHeader& hn = ps->pred[(a.launch + 1) & 1];
    hn.armed = 0;
    hn.ncand = 0u;
    // counters
    if (c.check >= 3) ps->stat[PST_REJECTED] += 1;
    else if (c.check > 0) ps->stat[PST_PAIRS] += 1;
    if (c.check > 0 && c.check < 3 && c.checked_k == 3) ps->stat[PST_STEPS3] += 1;
    if (c.check > 0 && c.check < 3 && c.checked_k == 4) ps->stat[PST_STEPS4] += 1;
    if (c.check == 2) ps->stat[PST_PRED_HIT] += 1;
    if (c.check == 4) ps->stat[PST_PRED_MISS] += 1;
    if (c.active) {
        if (c.bound) ps->stat[PST_BOUND_ONLY] += 1;
        else if (c.k == 1) ps->stat[PST_SINGLE] += 1;
        else if (!c.tentative) {
            ps->stat[PST_PAIRS] += 1;
            if (c.k == 3) ps->stat[PST_STEPS3] += 1;
            if (c.k == 4) ps->stat[PST_STEPS4] += 1;
        }
    }
    if (c.accepted_bad) {
        atomicOr(&st->status, 1u);
        atomicMin(&st->fail_step, (unsigned long long)c.n);
    }
}

// One strip and row segment of a launch in its number of steps.  (The form
// that lists candidates runs its own march also where it lists none: its
// floor is then infinite.)
template <int WPB, int KM, bool TAPE, bool CAND, bool LPB>
__device__ __forceinline__ void march_launch(const PairGeom& g, int k, bool store, int strip,
                                             int y0, int y1, int lane, double (&lm)[KMAX_STEPS],
                                             bool (&bad)[KMAX_STEPS], double* pbl) {
    if (KM >= 4 && k == 4)
        march_k<WPB, (KM >= 4 ? 4 : 1), TAPE, CAND, LPB>(g, strip, y0, y1, lane, lm, bad, true,
                                                         pbl);
    else if (KM >= 3 && k == 3)
        march_k<WPB, (KM >= 3 ? 3 : 1), TAPE, CAND, LPB>(g, strip, y0, y1, lane, lm, bad, true,
                                                         pbl);
    else if (k == 2)
        march_k<WPB, 2, TAPE, CAND, LPB>(g, strip, y0, y1, lane, lm, bad, true, pbl);
    else
        march_k<WPB, 1, TAPE, CAND, LPB>(g, strip, y0, y1, lane, lm, bad, store, pbl);
}

// Kernels of three or more steps keep the second row of their pipelines in
// LDS (the registers of the first, the prefetched row and the step's own
// values fill the budget of two waves per SIMD), and so do 12-wave
// workgroups (three waves per SIMD).
template <int WPB, int KM>
struct PipelineInLds {
    static constexpr bool value = KM >= 3 || WPB >= 12;
};

}  // namespace

template <int WPB, bool TAPE, bool CAND, int KM>
__global__ __launch_bounds__(64 * WPB) void step2d_pair(Pair2DArgs a) {
    const LaunchSlots ls = slots_for(a.launch);
    const PairCtl c = pair_control(a, ls);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_pair(a, ls, c);
    if (!c.active) return;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    PairGeom g;
    // the result goes to the other buffer; f^n stays intact
    g.fin = c.cur ? a.f1 : a.f0;
    g.fout = c.cur ? a.f0 : a.f1;
    g.ps = a.ps;
    g.rs = a.rs;
    g.nx = a.nx;
    g.ny = a.ny;
    g.strip = a.strip;
    g.c4lam[0] = 1.0 / (4.0 * c.lam1);
    g.c4lam[1] = 1.0 / (4.0 * (c.k >= 2 ? c.lam2 : c.lam1));
    g.c4lam[2] = 1.0 / (4.0 * (c.k >= 3 ? c.lam3 : c.lam1));
    g.c4lam[3] = 1.0 / (4.0 * (c.k >= 4 ? c.lam4 : c.lam1));
    g.omega = a.omega;
    g.gamma = a.gamma;
    for (int s = 0; s < 4; ++s) g.bc[s] = a.bc[s];
#pragma unroll
    for (int i = 0; i < KMAX_STEPS; ++i) g.tape[i] = a.tape[i];
    g.tape_ps = a.plane;
    g.t0 = c.cand ? c.t0 : INFINITY;
    g.ph = &a.pst->pred[a.launch & 1];
    g.cand = a.cand;
    const int total_waves = gridDim.x * WPB;
    const int ny = a.ny;
    // a bound-only pass marches one step and stores nothing
    const int km = c.bound ? 1 : c.k;

    double lm[KMAX_STEPS];
    bool bad[KMAX_STEPS];
#pragma unroll
    for (int i = 0; i < KMAX_STEPS; ++i) {
        lm[i] = 0.0;
        bad[i] = false;
    }
    constexpr bool LPB = PipelineInLds<WPB, KM>::value;
    __shared__ double pb_lds[LPB ? WPB * KM * 8 * 64 : 1];
    double* pbl = pb_lds + (LPB ? wave * KM * 8 * 64 : 0);
    for (int tile = xcd_remap(blockIdx.x, gridDim.x) * WPB + wave; tile < a.ntiles;
         tile += total_waves) {
        const int strip = tile % a.nstrips;
        const int seg = tile / a.nstrips;
        const int y0 = (int)(((long long)seg * ny) / a.nseg);
        const int y1 = (int)(((long long)(seg + 1) * ny) / a.nseg);
        march_launch<WPB, KM, TAPE, CAND, LPB>(g, km, !c.bound, strip, y0, y1, lane, lm, bad,
                                               pbl);
    }

    const bool per_step = a.lam_mode == LAM_PER_STEP;
    // the intermediate states (checked by the next launch)
#pragma unroll
    for (int i = 0; i < KMAX_STEPS - 1; ++i) {
        if (i < km - 1 || (c.bound && i == 0)) {
            if (per_step) {
                const double w = wave_max(lm[i]);
                if (lane == 0) publish_max(&a.pst->lamk[i][ls.la], w);
            }
            if (__any(bad[i]) && lane == 0) atomicOr(&a.pst->badk[i][ls.la], 1u);
        }
    }
    if (!c.bound) {
        // the state this launch leaves
        double wl = 0.0;
        bool wb = false;
#pragma unroll
        for (int i = 0; i < KMAX_STEPS; ++i) {
            if (i == km - 1) {
                wl = lm[i];
                wb = bad[i];
            }
        }
        if (per_step) {
            const double w = wave_max(wl);
            if (lane == 0) publish_max(&a.st->lam[ls.la], w);
        }
        if (__any(wb) && lane == 0) {
            // a tentative result is reported by the launch that accepts it
            if (c.tentative) atomicOr(&a.st->bad[ls.la], 1u);
            else publish_bad(a.st, ls, c.n + km);
        }
    }
}

// The predictions after fused launch a.launch, for the state S it leaves:
// level L (1 .. kmax-1, one launch each) evaluates the exact bound of the
// state after L steps from S on the 3 x 3 cells around every listed
// candidate whose bound is within CAND_REL of lambda*(S), and maxes it into
// pred[L] of the record the next launch reads.  Step 1 runs at the speed from
// lambda*(S) (known now), step L > 1 at the speed from the level L-1
// prediction (so each level is a launch of its own).  None when the launch
// listed no candidates or more than the list holds, or met a non-physical
// state.
//
// A one-wave workgroup takes a candidate at a time and marches its patch: the
// post-collision populations of S on the cells within L+1 of the centre,
// then of the states after 1 .. L-1 steps on shrinking patches (LDS, two
// buffers, population-major), and the bound after step L on the 3 x 3 cells.
// Every cell stands for its domain cell under the side conditions (a cell
// beyond a clamped side is the edge cell, a periodic side wraps), and its
// next state pulls from the domain cells its populations come from, as the
// step kernels do, with the step kernels' own device functions: the same
// bits.  Enough workgroups that every candidate of a usual list has its own
// wave; workgroup 0 also sets the record's count of valid levels and the
// counters.
static constexpr int PRED_BLOCKS = 2048;
static constexpr int PRED_R = KMAX_STEPS;              // patch radius of the deepest level
static constexpr int PRED_C0 = (2 * PRED_R + 1) * (2 * PRED_R + 1);  // cells, even stages
static constexpr int PRED_C1 = (2 * PRED_R - 1) * (2 * PRED_R - 1);  // cells, odd stages

namespace {

// Offset from the centre c (along one axis) of the domain cell that patch
// offset o stands for, shifted by -d: where a population of that cell comes
// from.  Periodic: offsets wrap with the domain, so they simply add.
__device__ inline int source_offset(int c, int o, int d, int n, bool periodic) {
    if (periodic) return o - d;
    return map_index(map_index(c + o, n, false) - d, n, false) - c;
}

// The state after one step at patch offset (ox, oy) of centre (cx, cy): the
// pulls from the post-collision patch `post` (radius rp, population-major
// with `stride` cells per plane), then the walls.
__device__ inline void gather_patch(const Pair2DArgs& a, int cx, int cy, int ox, int oy,
                                    const double* post, int rp, int stride, double g[16]) {
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    const int sxs[4] = {-1, 1, 1, -1}, sys[4] = {-1, -1, 1, 1};
    const int sp = 2 * rp + 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int fx = source_offset(cx, ox, sxs[j], a.nx, px);
        const int fy = source_offset(cy, oy, sys[j], a.ny, py);
        const int idx = (fy + rp) * sp + (fx + rp);
#pragma unroll
        for (int k = 0; k < 4; ++k) g[j * 4 + k] = post[(j * 4 + k) * stride + idx];
    }
    const int x = map_index(cx + ox, a.nx, px), y = map_index(cy + oy, a.ny, py);
    wall_images(g, a.bc[3] == BC_WALL && y == a.ny - 1, a.bc[2] == BC_WALL && y == 0,
                a.bc[0] == BC_WALL && x == 0, a.bc[1] == BC_WALL && x == a.nx - 1);
}

__device__ inline void collide_into(const double f[16], double gm1, double c4, double omega,
                                    double* post, int stride, int idx) {
    double U[4], fs[16];
    moments_d2q4(f, U);
    const Euler2 eu = euler2(U, gm1);
    collide_d2q4(f, U, eu, c4, omega, fs);
#pragma unroll
    for (int p = 0; p < 16; ++p) post[p * stride + idx] = fs[p];
}

}  // namespace

__global__ __launch_bounds__(64) void pair_predict_kernel(Pair2DArgs a, int level) {
    __shared__ double post0[16 * PRED_C0];
    __shared__ double post1[16 * PRED_C1];
    const LaunchSlots ls = slots_for(a.launch);
    PairState* ps = a.pst;
    const PredHeader* h = &ps->pred[a.launch & 1];
    PairSlot* q = &ps->q[ls.sw];
    const int lane = threadIdx.x;
    const unsigned ncand = h->ncand;
    const bool armed = h->armed != 0;
    bool ok = armed && ncand > 0u && ncand <= (unsigned)PRED_CAP && a.st->bad[ls.la] == 0u;
    if (level == 1 && blockIdx.x == 0 && lane == 0 && armed) {
        // (a launch that listed nothing keeps what its record carries)
        q->pred_valid = ok ? 1 : 0;
        ps->stat[ok ? PST_PREDICTED : PST_PRED_NONE] += 1;
        ps->stat[PST_LISTED] += ncand;
        if (ncand > (unsigned)PRED_CAP) ps->stat[PST_OVERFLOW] += 1;
    }
    if (level > 1) ok = ok && q->pred_valid >= level - 1;
    if (!ok) return;
    const unsigned long long lb = a.st->lam[ls.la];
    const unsigned long long lbc = a.st->lam_bc;
    // 1/(4 lambda) of the next launch's steps 1 .. level (scalars: an array
    // indexed by the run-time level would live in scratch memory); step s
    // runs only while the time before it is short of t_end
    static_assert(KMAX_STEPS <= 4, "three predicted steps at most");
    double c4a = 0.0, c4b = 0.0, c4c = 0.0;
    {
        double t = h->t_out;
        unsigned long long lstep = lb;
        for (int st = 1; st <= level; ++st) {
            if (lstep == 0ull || !(t < a.t_end)) return;
            double lam, t_next;
            step_size(LAM_PER_STEP, from_bits(lstep > lbc ? lstep : lbc), 0.0, a.dx, a.cfl, t,
                      a.t_end, lam, t_next);
            const double c4 = 1.0 / (4.0 * lam);
            if (st == 1) c4a = c4;
            else if (st == 2) c4b = c4;
            else c4c = c4;
            if (st < level) lstep = q->pred[st];
            t = t_next;
        }
    }
    auto c4_of = [&](int i) { return i == 0 ? c4a : (i == 1 ? c4b : c4c); };
    if (level > 1 && blockIdx.x == 0 && lane == 0) q->pred_valid = level;
    const double floor_l = from_bits(lb) * (1.0 - CAND_REL);
    const double gm1 = a.gamma - 1.0;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    const double* fin = h->cur_out ? a.f1 : a.f0;
    const int nx = a.nx, ny = a.ny;
    unsigned evaluated = 0;
    {
        double best = 0.0;
        for (unsigned i = blockIdx.x; i < ncand; i += gridDim.x) {
            const PredCand e = a.cand[i];
            if (!(e.l >= floor_l)) continue;
            const int cy = (int)(e.cell / nx), cx = (int)(e.cell % nx);
            // post-collision populations of S within level+1 of the centre
            {
                const int r = level + 1, sd = 2 * r + 1;
                for (int cell = lane; cell < sd * sd; cell += 64) {
                    const int ox = cell % sd - r, oy = cell / sd - r;
                    const int x = map_index(cx + ox, nx, px), y = map_index(cy + oy, ny, py);
                    const double* row = fin + (long long)y * a.rs;
                    double f[16];
#pragma unroll
                    for (int p = 0; p < 16; ++p) f[p] = row[p * a.ps + x];
                    collide_into(f, gm1, c4a, a.omega, post0, PRED_C0, cell);
                }
                __syncthreads();
            }
            // the states after steps 1 .. level-1, collided for the next step
            for (int st = 1; st < level; ++st) {
                const int r = level + 1 - st, sd = 2 * r + 1;
                const double* src = (st & 1) ? post0 : post1;
                double* dst = (st & 1) ? post1 : post0;
                const int sstride = (st & 1) ? PRED_C0 : PRED_C1;
                const int dstride = (st & 1) ? PRED_C1 : PRED_C0;
                for (int cell = lane; cell < sd * sd; cell += 64) {
                    const int ox = cell % sd - r, oy = cell / sd - r;
                    double g[16];
                    gather_patch(a, cx, cy, ox, oy, src, r + 1, sstride, g);
                    collide_into(g, gm1, c4_of(st), a.omega, dst, dstride, cell);
                }
                __syncthreads();
            }
            // the bound after step `level` on the 3 x 3 cells
            if (lane < 9) {
                const int ox = lane % 3 - 1, oy = lane / 3 - 1;
                const int x = cx + ox, y = cy + oy;
                const bool inside = (px || (x >= 0 && x < nx)) && (py || (y >= 0 && y < ny));
                if (inside) {
                    const bool odd = ((level - 1) & 1) != 0;
                    double g[16], U1[4], l1;
                    gather_patch(a, cx, cy, ox, oy, odd ? post1 : post0, 2,
                                 odd ? PRED_C1 : PRED_C0, g);
                    moments_d2q4(g, U1);
                    if (bound_d2q4(U1, a.gamma, &l1)) best = fmax(best, l1);
                    ++evaluated;
                }
            }
            __syncthreads();  // the patches are free for the next candidate
        }
        best = wave_max(best);
        if (lane == 0 && best > 0.0) publish_max(&q->pred[level], best);
    }
    unsigned cnt = evaluated;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane == 0 && cnt) atomicAdd(&ps->stat[PST_EVALUATED], (unsigned long long)cnt);
}

// K fused steps of every domain of a 2D batch (fixed lattice speeds, so
// nothing is guessed): the single-domain march over the fused launches'
// tile list, numbered domain by domain (each domain's strip count a multiple
// of the waves per workgroup, so a workgroup's waves share a domain and a
// row segment; strips of at most 64 - 2K columns); a non-physical state
// after any of the K steps sets the domain's status.  TAPE: U of every
// step's input to a.ktape[s].
template <int WPB, bool TAPE, int K>
__global__ __launch_bounds__(64 * WPB) void step2d_batch_pair(Batch2DArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long total_waves = (long long)gridDim.x * WPB;
    constexpr bool LPB = PipelineInLds<WPB, K>::value;
    __shared__ double pb_lds[LPB ? WPB * K * 8 * 64 : 1];
    double* pbl = pb_lds + (LPB ? wave * K * 8 * 64 : 0);
    for (long long tile = (long long)xcd_remap(blockIdx.x, gridDim.x) * WPB + wave;
         tile < a.pntiles; tile += total_waves) {
        int lo = 0, hi = a.ndom - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.doms[mid].ptile0 <= tile) lo = mid;
            else hi = mid - 1;
        }
        const Domain2D& d = a.doms[lo];
        PairGeom g;
        const long long fo = 16 * d.coff;
        g.fin = (a.cur ? a.f1 : a.f0) + fo;
        g.fout = (a.cur ? a.f0 : a.f1) + fo;
        g.ps = d.nx;
        g.rs = 16LL * d.nx;
        g.nx = d.nx;
        g.ny = d.ny;
        g.strip = d.pstrip;
#pragma unroll
        for (int i = 0; i < KMAX_STEPS; ++i) g.c4lam[i] = 1.0 / (4.0 * d.lam);
        g.omega = d.omega;
        g.gamma = d.gamma;
        for (int s = 0; s < 4; ++s) g.bc[s] = d.bc[s];
#pragma unroll
        for (int i = 0; i < KMAX_STEPS; ++i)
            g.tape[i] = TAPE && i < K ? a.ktape[i] + d.coff : nullptr;
        g.tape_ps = a.total;
        const int local = (int)(tile - d.ptile0);
        const int strip = local % d.pnstrips;
        const int seg = local / d.pnstrips;
        const int y0 = (int)(((long long)seg * d.ny) / d.nseg);
        const int y1 = (int)(((long long)(seg + 1) * d.ny) / d.nseg);
        double lm[KMAX_STEPS];
        bool bad[KMAX_STEPS];
#pragma unroll
        for (int i = 0; i < KMAX_STEPS; ++i) {
            lm[i] = 0.0;
            bad[i] = false;
        }
        march_k<WPB, K, TAPE, false, LPB, K != 3>(g, strip, y0, y1, lane, lm, bad, true, pbl);
        bool any_bad = false;
#pragma unroll
        for (int i = 0; i < K; ++i) any_bad = any_bad || bad[i];
        if (__any(any_bad) && lane == 0) atomicOr(&a.status[lo], 1u);
    }
}

__global__ void pair_prepare_kernel(PairState* ps, const DevState* st, int slot,
                                    long long max_steps) {
    if (threadIdx.x != 0) return;
    for (int i = 0; i < 2; ++i) {
        ps->q[i].t_base = 0.0;
        ps->q[i].n_base = 0;
        ps->q[i].cur_base = 0;
        ps->q[i].tentative = 0;
        for (int j = 0; j < KMAX_STEPS; ++j) ps->q[i].guess[j] = 0ull;
        ps->q[i].guess_base = 0ull;
        ps->q[i].known = 0;
        ps->q[i].trust = 3;  // start a call by guessing
        ps->q[i].predicted = 0;
        // a prediction the last call left stays (it is only a guess: checked)
    }
    for (int i = 0; i < KMAX_STEPS - 1; ++i)
        for (int j = 0; j < 3; ++j) {
            ps->lamk[i][j] = 0ull;
            ps->badk[i][j] = 0u;
        }
    for (int i = 0; i < 2; ++i) {
        ps->pred[i].armed = 0;
        ps->pred[i].ncand = 0u;
    }
    ps->n_limit = st->s[slot].n + max_steps;
}

__global__ void pair_reset_kernel(PairState* ps, bool counters) {
    if (threadIdx.x != 0) return;
    if (counters)
        for (int i = 0; i < PST_COUNT; ++i) ps->stat[i] = 0ull;
    for (int i = 0; i < 2; ++i) {
        ps->pred[i].armed = 0;
        ps->pred[i].ncand = 0u;
        ps->q[i].tentative = 0;
        ps->q[i].known = 0;
        ps->q[i].pred_valid = 0;
        ps->q[i].predicted = 0;
    }
}

hipError_t launch_pair_prepare(PairState* ps, const DevState* st, int slot, long long max_steps,
                               hipStream_t s) {
    hipLaunchKernelGGL(pair_prepare_kernel, dim3(1), dim3(64), 0, s, ps, st, slot, max_steps);
    return hipGetLastError();
}

hipError_t launch_pair_reset(PairState* ps, bool counters, hipStream_t s) {
    hipLaunchKernelGGL(pair_reset_kernel, dim3(1), dim3(64), 0, s, ps, counters);
    return hipGetLastError();
}

hipError_t launch_pair_predict(const Pair2DArgs& a, hipStream_t s) {
    for (int level = 1; level < a.kmax; ++level)
        hipLaunchKernelGGL(pair_predict_kernel, dim3(PRED_BLOCKS), dim3(64), 0, s, a, level);
    return hipGetLastError();
}

template <int WPB, int KM>
static hipError_t launch_pair_wk(const Pair2DArgs& a, bool tape, int max_blocks, hipStream_t s) {
    int nblocks = (a.ntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    // per-step speeds with a candidate list: the form that lists candidates
    // (the only form that reduces the bounds per-step speeds need)
    const bool cand = a.cand != nullptr && a.lam_mode == LAM_PER_STEP && !tape;
    if (a.lam_mode == LAM_PER_STEP && !cand) return hipErrorInvalidValue;
    if (cand)
        hipLaunchKernelGGL((step2d_pair<WPB, false, true, KM>), dim3(nblocks), dim3(64 * WPB), 0, s,
                           a);
    else if (tape)
        hipLaunchKernelGGL((step2d_pair<WPB, true, false, KM>), dim3(nblocks), dim3(64 * WPB), 0,
                           s, a);
    else
        hipLaunchKernelGGL((step2d_pair<WPB, false, false, KM>), dim3(nblocks), dim3(64 * WPB), 0,
                           s, a);
    return hipGetLastError();
}

// Launches of three or more steps run in workgroups of 8 waves at most.
template <int WPB>
static hipError_t launch_pair_w(const Pair2DArgs& a, bool tape, int max_blocks, hipStream_t s) {
    if (a.kmax <= 2) return launch_pair_wk<WPB, 2>(a, tape, max_blocks, s);
    if constexpr (WPB <= 8) {
        if (a.kmax == 3) return launch_pair_wk<WPB, 3>(a, tape, max_blocks, s);
        if (a.kmax == 4) return launch_pair_wk<WPB, 4>(a, tape, max_blocks, s);
    }
    return hipErrorInvalidValue;
}

template <int WPB, int KM>
static int occupancy(bool cand, bool tape) {
    int n = 0;
    hipError_t e;
    if (tape)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2d_pair<WPB, true, false, KM>,
                                                         64 * WPB, 0);
    else if (cand)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2d_pair<WPB, false, true, KM>,
                                                         64 * WPB, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2d_pair<WPB, false, false, KM>,
                                                         64 * WPB, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

template <int WPB>
static int pair_blocks_w(bool cand, int kmax, bool tape) {
    if (kmax <= 2) return occupancy<WPB, 2>(cand && !tape, tape);
    if constexpr (WPB <= 8) {
        if (kmax == 3) return occupancy<WPB, 3>(cand && !tape, tape);
        return occupancy<WPB, 4>(cand && !tape, tape);
    }
    return 1;
}

#define LBRS_PAIR_WPB_CASES(X) X(1) X(2) X(4) X(6) X(8) X(12)

hipError_t launch_step2d_pair(const Pair2DArgs& a, int wpb, bool tape, int max_blocks,
                              hipStream_t s) {
#define LBRS_CASE(W) \
    if (wpb == W) return launch_pair_w<W>(a, tape, max_blocks, s);
    LBRS_PAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

int step2d_pair_blocks_per_cu(int wpb, bool cand, int kmax, bool tape) {
#define LBRS_CASE(W) \
    if (wpb == W) return pair_blocks_w<W>(cand, kmax, tape);
    LBRS_PAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

template <int WPB, int K>
static hipError_t launch_batch_pair_wk(const Batch2DArgs& a, bool tape, int max_blocks,
                                       hipStream_t s) {
    long long nblocks = (a.pntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    if (tape)
        hipLaunchKernelGGL((step2d_batch_pair<WPB, true, K>), dim3((unsigned)nblocks),
                           dim3(64 * WPB), 0, s, a);
    else
        hipLaunchKernelGGL((step2d_batch_pair<WPB, false, K>), dim3((unsigned)nblocks),
                           dim3(64 * WPB), 0, s, a);
    return hipGetLastError();
}

// Launches of three or more steps run in workgroups of 8 waves at most.
template <int WPB>
static hipError_t launch_batch_pair_w(const Batch2DArgs& a, bool tape, int k, int max_blocks,
                                      hipStream_t s) {
    if (k == 2) return launch_batch_pair_wk<WPB, 2>(a, tape, max_blocks, s);
    if constexpr (WPB <= 8) {
        if (k == 3) return launch_batch_pair_wk<WPB, 3>(a, tape, max_blocks, s);
        if (k == 4) return launch_batch_pair_wk<WPB, 4>(a, tape, max_blocks, s);
    }
    return hipErrorInvalidValue;
}

template <int WPB, bool TAPE, int K>
static int batch_occupancy() {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, step2d_batch_pair<WPB, TAPE, K>, 64 * WPB, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

// Resident workgroups per CU of the k-step forms (the plain and the taped
// one, whichever fits fewer).
template <int WPB, int K>
static int batch_pair_blocks_k() {
    const int n = batch_occupancy<WPB, false, K>(), m = batch_occupancy<WPB, true, K>();
    return n < m ? n : m;
}

template <int WPB>
static int batch_pair_blocks_w(int k) {
    if (k == 2) return batch_pair_blocks_k<WPB, 2>();
    if constexpr (WPB <= 8) {
        if (k == 3) return batch_pair_blocks_k<WPB, 3>();
        if (k == 4) return batch_pair_blocks_k<WPB, 4>();
    }
    return 1;
}

hipError_t launch_step2d_batch_pair(const Batch2DArgs& a, int wpb, bool tape, int k,
                                    int max_blocks, hipStream_t s) {
#define LBRS_CASE(W) \
    if (wpb == W) return launch_batch_pair_w<W>(a, tape, k, max_blocks, s);
    LBRS_PAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

int step2d_batch_pair_blocks_per_cu(int wpb, int k) {
#define LBRS_CASE(W) \
    if (wpb == W) return batch_pair_blocks_w<W>(k);
    LBRS_PAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

}  // namespace lbrs
