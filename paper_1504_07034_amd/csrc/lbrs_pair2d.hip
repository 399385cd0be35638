// Two fused LBRS steps per launch for the 2D Euler equations (D2Q4, gfx950).
//
// The single-step kernel reads f^n and writes f^{n+1} once per step: 256 B of
// HBM traffic per cell and step, which bounds it.  Here a wavefront feeds
// every row of f^{n+1} it has just streamed straight into a second collision
// and streaming, so f^n is read once and f^{n+2} written once: 128 B per cell
// and step.  Both steps are the scheme of Sec. II.D unchanged (moments, the
// folded equilibria, relaxation, exact diagonal hops, Sec. II.E walls,
// transmissive and periodic sides); nothing but the order of the work differs.
//
// Lanes and rows.  Lane l holds column x0 - 2 + l.  The first step is valid
// on lanes 1..62, the second on lanes 2..61, so a strip has <= 60 output
// columns.  A tile's first step computes rows y0-1 .. y1 of f^{n+1} (one halo
// row on each side, from f^n rows y0-2 .. y1+1), the second rows y0 .. y1-1 of
// f^{n+2}.  Register pipelines: the upward hops of the last two rows of each
// step, and the next row of f^n in flight.  At a clamped (transmissive or
// wall) side the second step must pull from the edge cell of f^{n+1} itself,
// not from a ghost row or column that the first step would make up: there
// the edge column's values are copied into the halo lane, and at a clamped
// bottom or top the edge row's hops are reused (selects, no extra rows).
//
// Lattice speed of the second step.  With a fixed speed it is known.  With
// the per-step speed it is the global bound over f^{n+1}, which no workgroup
// has before the launch ends.  The launch then takes lambda*_{n+1} equal to
// lambda*_n, reduces the true bound of its f^{n+1} on the side, and leaves
// its result tentative.  The next launch checks the guess: equal bit for bit
// (and the first step admissible) means the two steps are exactly those of
// two single steps, and it continues from f^{n+2}; otherwise f^n, still
// intact in the other buffer, is current again, and that launch repeats the
// pair with the now known lambda*_{n+1} (or one step when the first step was
// non-physical).  Where the bound keeps changing, guessing wastes a pass per
// two steps; a saturating count of how often the checked bound repeated
// (0..3, one up for a repeat, one down for a change) decides: at 0 a launch
// first reduces the bound of f^{n+1} alone (reading f^n, storing nothing) and
// the next launch takes the two steps with it; above 0 it guesses.  Every
// workgroup of a launch takes the same decisions from the same slots, so no
// grid barrier is needed.  The last launch of a call never leaves a
// tentative result, so every other call sees an ordinary time state.
//
// Also here: the taped form (U^n and U^{n+1} stored for the gradients'
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
    double c4lam1, c4lam2, omega, gamma;
    int bc[4];
    double* tape0;   // TAPE: U^n and U^{n+1}, element (k, y, x) at k*tape_ps + y*nx + x
    double* tape1;
    long long tape_ps;
    // CAND: the floor of the candidates' bounds, this launch's header and
    // where candidates go
    double t0;
    PredHeader* ph;
    PredCand* cand;
};

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

// Rows y0..y1-1 of one strip, one step (TWO = false: f^{n+1} is the output)
// or two.  lm1/bad1 gather the bound and admissibility of this tile's cells
// of f^{n+1}, lm2/bad2 those of f^{n+2}.
// Moments of row j of a tape (rows [y0, y1) of the tile only: other rows
// and lanes carry an out-of-range offset, so the store is unconditional).
__device__ inline void tape_row(double* tape, long long tape_ps, int nx, int j, int y0, int y1,
                                int voff, const double U[4]) {
    const bool own = j >= y0 && j < y1;
    double* row = tape + (long long)(own ? j : y0) * nx;
#pragma unroll
    for (int k = 0; k < 4; ++k) store_row(row + k * tape_ps, nx * 8, own ? voff : 0x7fffffff, U[k]);
}

template <int WPB, bool TWO, bool TAPE, bool CAND = false>
__device__ __forceinline__ void march_pair(const PairGeom& g, int strip, int y0, int y1, int lane,
                                           double& lm1, bool& bad1, double& lm2, bool& bad2,
                                           bool store = true) {
    static_assert(!CAND || !TAPE, "candidates ride on plain launches");
    const int nx = g.nx, ny = g.ny;
    const bool px = g.bc[0] == BC_PERIODIC, py = g.bc[2] == BC_PERIODIC;
    const double gm1 = g.gamma - 1.0;
    const int row_bytes = nx * 8;
    const int x0 = strip * g.strip;
    const int x = x0 - 2 + lane;
    const int xl = map_index(x, nx, px);
    const bool out_lane = lane >= 2 && lane <= g.strip + 1 && x < nx;
    const int voff = out_lane ? x * 8 : 0x7fffffff;
    const bool wxlo = g.bc[0] == BC_WALL && x == 0;
    const bool wxhi = g.bc[1] == BC_WALL && x == nx - 1;
    const bool wlo = g.bc[2] == BC_WALL, whi = g.bc[3] == BC_WALL;
    // rows [a0, b0) of f^{n+1}; f^n rows a0-1 .. b0 are read
    const int a0 = TWO ? y0 - 1 : y0, b0 = TWO ? y1 + 1 : y1;
    // strips that may hold the ghost lanes x = -1 or x = nx of a clamped x side
    const bool xfix = TWO && !px && (x0 == 0 || x0 + 61 >= nx);
    const bool clamp_lo = TWO && !py && y0 == 0;
    const bool clamp_hi = TWO && !py && y1 == ny;

    double A3[4], A4[4], B3[4], B4[4];  // first step: upward hops of rows r-1, r-2
    double P3[4], P4[4], Q3[4], Q4[4];  // second step: upward hops of rows q-1, q-2
    double U[4];
    Hops h;

    // CAND: candidates for the prediction of lambda*_{n+3} (see PredCand).
    // A row's cells are decided when the row after it is known: l of rows
    // o2-1 (lp, pending) and o2-2 (lpp) in this lane, -1 outside the tile;
    // the wave's largest bound so far, the threshold CAND_REL below it (at
    // least the launch's floor), and the first lane of the pending row that
    // raised the largest bound (-1: none).
    double thr = CAND ? g.t0 : 0.0, wmax = 0.0, lp = -1.0, lpp = -1.0;
    int rec_prev = -1;
    auto candidates = [&](double lc, int o2) {
        int rec_cur = -1;
        if (__any(lc > thr)) {
            const double rowmax = wave_max(lc);
            if (rowmax > wmax) {
                rec_cur = __ffsll((long long)__ballot(lc == rowmax)) - 1;
                wmax = rowmax;
                thr = fmax(g.t0, wmax * (1.0 - CAND_REL));
            }
        }
        // row o2-1: a cell goes in when its bound is above the threshold and
        // no neighbour's exceeds it (a neighbour outside the tile is
        // ignored), except inside a flat region, which leaves only the cell
        // that first reached its value
        if (__any(lp > thr)) {
            const double ll = lane_from_left(lp), lr = lane_from_right(lp);
            const bool top = (ll < 0.0 || lp >= ll) && (lr < 0.0 || lp >= lr) &&
                             (lpp < 0.0 || lp >= lpp) && (lc < 0.0 || lp >= lc);
            const bool flat = (ll < 0.0 || lp == ll) && (lr < 0.0 || lp == lr) &&
                              (lpp < 0.0 || lp == lpp) && (lc < 0.0 || lp == lc);
            const bool emit = lp > thr && top && (!flat || lane == rec_prev);
            const unsigned long long m = __ballot(emit);
            if (m) {
                unsigned base = 0;
                if (lane == 0) base = atomicAdd(&g.ph->ncand, (unsigned)__popcll(m));
                base = __shfl(base, 0, 64);
                if (emit) {
                    const unsigned idx = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
                    if (idx < (unsigned)PRED_CAP) {
                        g.cand[idx].cell = (long long)(o2 - 1) * nx + x;
                        g.cand[idx].l = lp;
                    }
                }
            }
        }
        rec_prev = rec_cur;
        lpp = lp;
        lp = lc;
    };

    // Row r of f^n (in cur) completes row r-1 of f^{n+1} and, with TWO, row
    // r-2 of f^{n+2}; row r+1 is loaded into nxt first, so that it is in
    // flight while row r is computed.  One copy of this code serves every
    // row: two inlined copies may be contracted into different multiply-adds
    // by the compiler, and rows would then round differently.
    auto row = [&](double (&cur)[16], double (&nxt)[16], int r) {
        // lockstep with the workgroup's neighbouring strips (equal trip counts)
        if (WPB > 1) __builtin_amdgcn_s_barrier();
        load_row(nxt, g.fin, g.ps, g.rs, map_index(r + 1, ny, py), xl);
        moments_d2q4(cur, U);
        if (TAPE) tape_row(g.tape0, g.tape_ps, nx, r, y0, y1, voff, U);  // U^n of row r
        collide_hops(cur, U, gm1, g.c4lam1, g.omega, h);
        const int o1 = r - 1;
        double g1[16];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            g1[0 * 4 + k] = h.d0[k];
            g1[1 * 4 + k] = h.d1[k];
            g1[2 * 4 + k] = B3[k];
            g1[3 * 4 + k] = B4[k];
            B3[k] = A3[k];
            B4[k] = A4[k];
            A3[k] = h.u2[k];
            A4[k] = h.u3[k];
        }
        wall_images(g1, whi && o1 == ny - 1, wlo && o1 == 0, wxlo, wxhi);
        if (xfix) {
            // a clamped side: beyond it, f^{n+1} is the edge column's
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const double fr = lane_from_right(g1[p]);
                const double fl = lane_from_left(g1[p]);
                g1[p] = x == -1 ? fr : (x == nx ? fl : g1[p]);
            }
        }
        double U1[4], l1;
        moments_d2q4(g1, U1);
        const bool own1 = out_lane && o1 >= y0 && o1 < y1;
        if (TAPE && TWO) tape_row(g.tape1, g.tape_ps, nx, o1, y0, y1, voff, U1);  // U^{n+1}
        const bool ok1 = bound_d2q4(U1, g.gamma, &l1);
        bad1 |= own1 && !ok1;
        lm1 = fmax(lm1, own1 ? l1 : 0.0);
        if (!TWO) {
            // (a bound-only launch drops the row: out-of-range offset)
            store_full_row(g.fout + (long long)o1 * g.rs, g.ps, row_bytes,
                           store ? voff : 0x7fffffff, g1);
            if (CAND) candidates(own1 && ok1 ? l1 : -1.0, o1);
            return;
        }
        // second step: row q = o1 of f^{n+1} completes row q - 1 of f^{n+2}
        const int q = o1;
        Hops h2;
        collide_hops(g1, U1, gm1, g.c4lam2, g.omega, h2);
        {
            // row q - 1 of f^{n+2}, an output row once q > y0.  The store is
            // unconditional (an out-of-range offset is dropped by the buffer
            // range check), so the wait for the next row's loads never has
            // to cover this row's stores.
            const bool row_out = q > y0 && q - 1 < y1;
            const int o2 = row_out ? q - 1 : y0;
            // at a clamped top, row ny of f^{n+1} is row ny-1 again: its
            // downward hops were kept in P at q = ny-1
            const bool top_virtual = clamp_hi && q == ny;
            double g2[16];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                g2[0 * 4 + k] = top_virtual ? P3[k] : h2.d0[k];
                g2[1 * 4 + k] = top_virtual ? P4[k] : h2.d1[k];
                g2[2 * 4 + k] = Q3[k];
                g2[3 * 4 + k] = Q4[k];
            }
            // (the wall rows by the row's own index: the filter also reads the
            // halo rows y0-1 and y1, which are not stored)
            wall_images(g2, whi && q - 1 == ny - 1, wlo && q - 1 == 0, wxlo, wxhi);
            store_full_row(g.fout + (long long)o2 * g.rs, g.ps, row_bytes,
                           row_out ? voff : 0x7fffffff, g2);
            double U2[4], l2;
            moments_d2q4(g2, U2);
            const bool ok2 = bound_d2q4(U2, g.gamma, &l2);
            const bool own2 = out_lane && row_out;
            bad2 |= own2 && !ok2;
            lm2 = fmax(lm2, own2 ? l2 : 0.0);
            // at a clamped bottom, row -1 of f^{n+1} is row 0 again; at a
            // clamped top, keep row ny-1's downward hops for the virtual row
            // ny (the hops are dead after this, before the filter's work)
            const bool lo_edge = clamp_lo && q == 0;
            const bool hi_edge = clamp_hi && q == ny - 1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                Q3[k] = lo_edge ? h2.u2[k] : P3[k];
                Q4[k] = lo_edge ? h2.u3[k] : P4[k];
                P3[k] = hi_edge ? h2.d0[k] : h2.u2[k];
                P4[k] = hi_edge ? h2.d1[k] : h2.u3[k];
            }
            if (CAND) candidates(own2 && ok2 ? l2 : -1.0, q - 1);
        }
    };

    // prologue: rows a0-1 and a0 of f^n fill the first step's pipeline
    double f[16], nxt[16];
    load_row(f, g.fin, g.ps, g.rs, map_index(a0 - 1, ny, py), xl);
    load_row(nxt, g.fin, g.ps, g.rs, map_index(a0, ny, py), xl);
    moments_d2q4(f, U);
    collide_hops(f, U, gm1, g.c4lam1, g.omega, h);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        A3[k] = h.u2[k];
        A4[k] = h.u3[k];
    }
#pragma unroll
    for (int p = 0; p < 16; ++p) f[p] = nxt[p];
    load_row(nxt, g.fin, g.ps, g.rs, map_index(a0 + 1, ny, py), xl);
    moments_d2q4(f, U);
    if (TAPE && !TWO) tape_row(g.tape0, g.tape_ps, nx, a0, y0, y1, voff, U);  // U^n of row y0
    collide_hops(f, U, gm1, g.c4lam1, g.omega, h);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        B3[k] = A3[k];
        B4[k] = A4[k];
        A3[k] = h.u2[k];
        A4[k] = h.u3[k];
        P3[k] = P4[k] = Q3[k] = Q4[k] = 0.0;
    }
    for (int r = a0 + 1; r <= b0; ++r) {
#pragma unroll
        for (int p = 0; p < 16; ++p) f[p] = nxt[p];
        row(f, nxt, r);
    }
    // the tile's last row is decided without the row after it
    if (CAND) candidates(-1.0, y1);
}

__device__ inline double from_bits(unsigned long long b) { return __longlong_as_double((long long)b); }

// dt and the lattice speed of one step, in the order of operations of the
// single-step control (so that both produce the same bits).
__device__ inline void step_size(int lam_mode, double lam_star, double lam_fixed, double dx,
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

// Time control of one fused launch (identical in every thread).
struct PairCtl {
    bool active;        // at least one step
    bool two;           // two steps
    bool tentative;     // the result waits for the next launch's check
    bool bound;         // this launch only reduces the bound of f^{n+1}
    bool accepted_bad;  // the previous launch's pair stands, with a non-physical f^{n+2}
    bool predicted;     // this launch's guess is the predicted bound
    bool cand;          // this launch lists candidates for the prediction of lambda*_{n+3}
    int trust;          // saturating count of repeated bounds at the last checks (0..3)
    int check;          // outcome of the check of the previous launch (for the counters):
                        // 0 none, 1 accepted, 2 predicted and accepted, 3 rejected,
                        // 4 predicted and rejected
    int cur;
    long long n;
    double t, lam_used;
    unsigned long long lstar;  // bits of lambda*_n (the bound of the current state)
    unsigned long long guess;  // bits of the lambda*_{n+1} a tentative pair takes
    unsigned bad;
    double lam1, t1, lam2, t2;
    double t0;          // floor of the candidates' bounds
    bool pred_ok;       // the record read holds a prediction for the current state
    unsigned long long pred;  // its bits
};

__device__ inline PairCtl pair_control(const Pair2DArgs& a, LaunchSlots ls) {
    const DevState* st = a.st;
    const PairState* ps = a.pst;
    PairCtl c;
    Slot s = st->s[ls.sr];
    const PairSlot q = ps->q[ls.sr];
    unsigned long long lstar = st->lam[ls.lr];
    unsigned bad = st->bad[ls.lr];
    bool know_next = false, force_single = false;
    unsigned long long next = 0ull;
    int trust = q.trust;
    // the previous launch left a prediction for the state it produced
    bool pred_ok = q.pred_valid != 0 && q.pred != 0ull;
    c.accepted_bad = false;
    c.check = 0;
    if (q.tentative) {
        const unsigned long long m1 = ps->lam1[ls.lr];
        const bool b1 = ps->bad1[ls.lr] != 0u;
        const bool exact = m1 == q.guess;
        const bool ok = !b1 && (a.lam_mode != LAM_PER_STEP || exact);
        if (!b1 && !q.predicted) trust = exact ? min(trust + 1, 3) : max(trust - 1, 0);
        c.check = ok ? (q.predicted ? 2 : 1) : (q.predicted ? 4 : 3);
        if (ok) {
            c.accepted_bad = bad != 0u;
        } else {
            // back to f^n; the bound of f^{n+1} is known now
            s.t = q.t_base;
            s.n = q.n_base;
            s.cur = q.cur_base;
            lstar = q.guess_base;
            bad = 0u;
            force_single = b1;
            know_next = !b1;
            next = m1;
            pred_ok = false;
        }
    } else if (q.known) {
        // the previous launch reduced the bound of f^{n+1} of this state
        const unsigned long long m1 = ps->lam1[ls.lr];
        const bool b1 = ps->bad1[ls.lr] != 0u;
        force_single = b1;
        know_next = !b1;
        next = m1;
        if (!b1) trust = m1 == lstar ? min(trust + 1, 3) : max(trust - 1, 0);
        pred_ok = false;
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
    step_size(a.lam_mode, from_bits(lstar > lbc ? lstar : lbc), st->lam_fixed, a.dx, a.cfl, s.t,
              a.t_end, c.lam1, c.t1);
    c.two = c.active && !force_single && c.t1 < a.t_end && s.n + 2 <= n_limit;
    // a new pair with per-step speeds: take the predicted bound, else guess
    // the current one while it has been repeating, else reduce it first
    const bool per_step = a.lam_mode == LAM_PER_STEP;
    c.predicted = c.two && !know_next && per_step && pred_ok;
    c.bound = c.two && !know_next && per_step && !c.predicted && trust == 0;
    if (c.bound) c.two = false;
    c.tentative = c.two && !know_next;
    if (a.last && (c.tentative || c.bound)) c.two = c.tentative = c.bound = c.predicted = false;
    c.trust = trust;
    c.lam2 = c.lam1;
    c.t2 = c.t1;
    c.guess = c.predicted ? q.pred : lstar;
    const unsigned long long l2 = know_next ? next : c.guess;
    if (c.two)
        step_size(a.lam_mode, from_bits(l2 > lbc ? l2 : lbc), st->lam_fixed, a.dx, a.cfl, c.t1,
                  a.t_end, c.lam2, c.t2);
    // candidates for the prediction of the bound after the next launch's
    // first step: bounds of the state this launch leaves (U^{n+2}, or U^{n+1}
    // of a one-step launch) from CAND_REL below the last known one up
    c.cand = c.active && !c.bound && per_step && a.cand != nullptr &&
             (c.two ? c.t2 : c.t1) < a.t_end;
    c.t0 = c.cand ? from_bits(c.two ? l2 : lstar) * (1.0 - CAND_REL) : 0.0;
    c.pred_ok = pred_ok;
    c.pred = q.pred;
    return c;
}

// Block 0, thread 0: the time state after this launch and its pair record;
// clears the accumulators of launch p+2; arms the prediction kernel.
__device__ inline void publish_pair(const Pair2DArgs& a, LaunchSlots ls, const PairCtl& c) {
    DevState* st = a.st;
    PairState* ps = a.pst;
    Slot s;
    s.pad = 0;
    PairSlot q;
    q.t_base = c.t;
    q.n_base = c.n;
    q.cur_base = c.cur;
    q.guess = c.guess;
    q.guess_base = c.lstar;
    q.tentative = 0;
    q.known = 0;
    q.trust = c.trust;
    q.pred_valid = 0;
    q.predicted = c.predicted ? 1 : 0;
    q.pred = 0ull;
    if (!c.active) {
        s.t = c.t;
        s.n = c.n;
        s.lam_used = c.lam_used;
        s.cur = c.cur;
        st->lam[ls.la] = c.lstar;
        st->bad[ls.la] = c.bad;
        // the state stays: so does a prediction for it (also into the next call)
        q.pred_valid = c.pred_ok ? 1 : 0;
        q.pred = c.pred;
    } else if (c.bound) {
        // no step: the state and its bound carry over; the first-step
        // accumulators receive the bound of f^{n+1}
        s.t = c.t;
        s.n = c.n;
        s.lam_used = c.lam_used;
        s.cur = c.cur;
        st->lam[ls.la] = c.lstar;
        st->bad[ls.la] = 0u;
        q.known = 1;
    } else if (!c.two) {
        s.t = c.t1;
        s.n = c.n + 1;
        s.lam_used = c.lam1;
        s.cur = c.cur ^ 1;
    } else {
        s.t = c.t2;
        s.n = c.n + 2;
        s.lam_used = c.lam2;
        s.cur = c.cur ^ 1;
        q.tentative = c.tentative ? 1 : 0;
    }
    st->s[ls.sw] = s;
    ps->q[ls.sw] = q;
    st->lam[ls.lz] = 0ull;
    st->bad[ls.lz] = 0u;
    ps->lam1[ls.lz] = 0ull;
    ps->bad1[ls.lz] = 0u;
    // this launch's candidate header (its candidate count was cleared by the
    // launch before) and the next launch's, whose last user, the prediction
    // after the launch before, has finished
    PredHeader& h = ps->pred[a.launch & 1];
    h.armed = c.cand ? 1 : 0;
    h.cur_out = c.cur ^ 1;
    h.t2 = c.two ? c.t2 : c.t1;
    PredHeader& hn = ps->pred[(a.launch + 1) & 1];
    hn.armed = 0;
    hn.ncand = 0u;
    // counters
    if (c.check >= 3) ps->stat[PST_REJECTED] += 1;
    else if (c.check > 0) ps->stat[PST_PAIRS] += 1;
    if (c.check == 2) ps->stat[PST_PRED_HIT] += 1;
    if (c.check == 4) ps->stat[PST_PRED_MISS] += 1;
    if (c.active) {
        if (c.bound) ps->stat[PST_BOUND_ONLY] += 1;
        else if (!c.two) ps->stat[PST_SINGLE] += 1;
        else if (!c.tentative) ps->stat[PST_PAIRS] += 1;
    }
    if (c.accepted_bad) {
        atomicOr(&st->status, 1u);
        atomicMin(&st->fail_step, (unsigned long long)c.n);
    }
}

}  // namespace

template <int WPB, bool TAPE, bool CAND>
__global__ __launch_bounds__(64 * WPB) void step2d_pair(Pair2DArgs a) {
    const LaunchSlots ls = slots_for(a.launch);
    const PairCtl c = pair_control(a, ls);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_pair(a, ls, c);
    if (!c.active) return;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    PairGeom g;
    // f^{n+2} (or f^{n+1}) goes to the other buffer; f^n stays intact
    g.fin = c.cur ? a.f1 : a.f0;
    g.fout = c.cur ? a.f0 : a.f1;
    g.ps = a.ps;
    g.rs = a.rs;
    g.nx = a.nx;
    g.ny = a.ny;
    g.strip = a.strip;
    g.c4lam1 = 1.0 / (4.0 * c.lam1);
    g.c4lam2 = 1.0 / (4.0 * c.lam2);
    g.omega = a.omega;
    g.gamma = a.gamma;
    for (int s = 0; s < 4; ++s) g.bc[s] = a.bc[s];
    g.tape0 = a.tape0;
    g.tape1 = a.tape1;
    g.tape_ps = a.plane;
    g.t0 = c.t0;
    g.ph = &a.pst->pred[a.launch & 1];
    g.cand = a.cand;
    const int total_waves = gridDim.x * WPB;
    const int ny = a.ny;

    double lm1 = 0.0, lm2 = 0.0;
    bool bad1 = false, bad2 = false;
    for (int tile = xcd_remap(blockIdx.x, gridDim.x) * WPB + wave; tile < a.ntiles;
         tile += total_waves) {
        const int strip = tile % a.nstrips;
        const int seg = tile / a.nstrips;
        const int y0 = (int)(((long long)seg * ny) / a.nseg);
        const int y1 = (int)(((long long)(seg + 1) * ny) / a.nseg);
        if (c.two) {
            if (CAND && c.cand)
                march_pair<WPB, true, false, true>(g, strip, y0, y1, lane, lm1, bad1, lm2, bad2);
            else
                march_pair<WPB, true, TAPE>(g, strip, y0, y1, lane, lm1, bad1, lm2, bad2);
        } else {
            if (CAND && c.cand)
                march_pair<WPB, false, false, true>(g, strip, y0, y1, lane, lm1, bad1, lm2, bad2);
            else
                march_pair<WPB, false, TAPE>(g, strip, y0, y1, lane, lm1, bad1, lm2, bad2,
                                             !c.bound);
        }
    }

    const bool per_step = a.lam_mode == LAM_PER_STEP;
    if (c.two) {
        if (per_step) {
            const double w1 = wave_max(lm1), w2 = wave_max(lm2);
            if (lane == 0) {
                publish_max(&a.pst->lam1[ls.la], w1);
                publish_max(&a.st->lam[ls.la], w2);
            }
        }
        if (__any(bad1) && lane == 0) atomicOr(&a.pst->bad1[ls.la], 1u);
        if (__any(bad2) && lane == 0) {
            // a tentative f^{n+2} is reported by the launch that accepts it
            if (c.tentative) atomicOr(&a.st->bad[ls.la], 1u);
            else publish_bad(a.st, ls, c.n + 2);
        }
    } else if (c.bound) {
        const double w1 = wave_max(lm1);
        if (lane == 0) publish_max(&a.pst->lam1[ls.la], w1);
        if (__any(bad1) && lane == 0) atomicOr(&a.pst->bad1[ls.la], 1u);
    } else {
        if (per_step) {
            const double w1 = wave_max(lm1);
            if (lane == 0) publish_max(&a.st->lam[ls.la], w1);
        }
        if (__any(bad1) && lane == 0) publish_bad(a.st, ls, c.n + 1);
    }
}

// The prediction after fused launch a.launch: the exact bound of the state
// after the next launch's first step on the 3 x 3 cells around every
// candidate the launch listed whose bound of U^{n+2} is within CAND_REL of
// lambda*_{n+2}, by the first step's own arithmetic (f^{n+2} of the cell's
// four pull sources, their collision at the now known speed of step n+2,
// the pulls, walls, moments, bound: the same device functions, so the same
// bits), maxed into the pair record the next launch reads.  None when the
// launch listed no candidates or more than the list holds, or met a
// non-physical state.  PRED_BLOCKS workgroups stride over (candidate,
// neighbour) pairs; workgroup 0 also sets the record's validity and counters.
static constexpr int PRED_BLOCKS = 64;

__global__ __launch_bounds__(256) void pair_predict_kernel(Pair2DArgs a) {
    const LaunchSlots ls = slots_for(a.launch);
    PairState* ps = a.pst;
    const PredHeader* h = &ps->pred[a.launch & 1];
    const int tid = threadIdx.x;
    const unsigned ncand = h->ncand;
    const bool ok = h->armed != 0 && ncand > 0u && ncand <= (unsigned)PRED_CAP &&
                    a.st->bad[ls.la] == 0u;
    if (blockIdx.x == 0 && tid == 0 && h->armed) {
        // (a launch that listed nothing keeps what its record carries)
        ps->q[ls.sw].pred_valid = ok ? 1 : 0;
        ps->stat[ok ? PST_PREDICTED : PST_PRED_NONE] += 1;
        ps->stat[PST_LISTED] += ncand;
        if (ncand > (unsigned)PRED_CAP) ps->stat[PST_OVERFLOW] += 1;
    }
    if (!ok) return;
    const unsigned long long lb = a.st->lam[ls.la];
    const unsigned long long lbc = a.st->lam_bc;
    const double lstar = from_bits(lb > lbc ? lb : lbc);
    const double floor_l = from_bits(lb) * (1.0 - CAND_REL);
    double lam, tn;
    step_size(LAM_PER_STEP, lstar, 0.0, a.dx, a.cfl, h->t2, a.t_end, lam, tn);
    const double c4lam = 1.0 / (4.0 * lam);
    const double gm1 = a.gamma - 1.0;
    const double* fin = h->cur_out ? a.f1 : a.f0;
    const int nx = a.nx, ny = a.ny;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    const int sxs[4] = {-1, 1, 1, -1}, sys[4] = {-1, -1, 1, 1};
    double best = 0.0;
    unsigned evaluated = 0;
    const unsigned work = ncand * 9u;
    for (unsigned i = blockIdx.x * blockDim.x + tid; i < work; i += gridDim.x * blockDim.x) {
        const PredCand e = a.cand[i / 9u];
        if (!(e.l >= floor_l)) continue;
        const int cy = (int)(e.cell / nx), cx = (int)(e.cell % nx);
        int x = cx + (int)(i % 3u) - 1, y = cy + (int)((i / 3u) % 3u) - 1;
        if (px) x = map_index(x, nx, true);
        if (py) y = map_index(y, ny, true);
        if (x < 0 || x >= nx || y < 0 || y >= ny) continue;
        ++evaluated;
        double g1[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int xs = map_index(x - sxs[j], nx, px), ys = map_index(y - sys[j], ny, py);
            double f[16], U[4], fs[16];
            const double* row = fin + (long long)ys * a.rs;
#pragma unroll
            for (int p = 0; p < 16; ++p) f[p] = row[p * a.ps + xs];
            moments_d2q4(f, U);
            const Euler2 eu = euler2(U, gm1);
            collide_d2q4(f, U, eu, c4lam, a.omega, fs);
#pragma unroll
            for (int k = 0; k < 4; ++k) g1[j * 4 + k] = fs[j * 4 + k];
        }
        wall_images(g1, a.bc[3] == BC_WALL && y == ny - 1, a.bc[2] == BC_WALL && y == 0,
                    a.bc[0] == BC_WALL && x == 0, a.bc[1] == BC_WALL && x == nx - 1);
        double U1[4], l1;
        moments_d2q4(g1, U1);
        if (bound_d2q4(U1, a.gamma, &l1)) best = fmax(best, l1);
    }
    best = wave_max(best);
    unsigned cnt = evaluated;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((tid & 63) == 0) {
        if (best > 0.0) publish_max(&ps->q[ls.sw].pred, best);
        if (cnt) atomicAdd(&ps->stat[PST_EVALUATED], (unsigned long long)cnt);
    }
}

// Two fused steps of every domain of a 2D batch (fixed lattice speeds, so
// nothing is guessed): the single-domain march over the fused launches' tile
// list, numbered domain by domain (each domain's strip count a multiple of
// the waves per workgroup, so a workgroup's waves share a domain and a row
// segment); a non-physical f^{n+1} or f^{n+2} sets the domain's status.
template <int WPB, bool TAPE>
__global__ __launch_bounds__(64 * WPB) void step2d_batch_pair(Batch2DArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long total_waves = (long long)gridDim.x * WPB;
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
        g.c4lam1 = g.c4lam2 = 1.0 / (4.0 * d.lam);
        g.omega = d.omega;
        g.gamma = d.gamma;
        for (int s = 0; s < 4; ++s) g.bc[s] = d.bc[s];
        g.tape0 = TAPE ? a.tape + d.coff : nullptr;
        g.tape1 = TAPE ? a.tape2 + d.coff : nullptr;
        g.tape_ps = a.total;
        const int local = (int)(tile - d.ptile0);
        const int strip = local % d.pnstrips;
        const int seg = local / d.pnstrips;
        const int y0 = (int)(((long long)seg * d.ny) / d.nseg);
        const int y1 = (int)(((long long)(seg + 1) * d.ny) / d.nseg);
        double lm1 = 0.0, lm2 = 0.0;
        bool bad1 = false, bad2 = false;
        march_pair<WPB, true, TAPE>(g, strip, y0, y1, lane, lm1, bad1, lm2, bad2);
        if (__any(bad1 || bad2) && lane == 0) atomicOr(&a.status[lo], 1u);
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
        ps->q[i].guess = 0ull;
        ps->q[i].guess_base = 0ull;
        ps->q[i].known = 0;
        ps->q[i].trust = 3;  // start a call by guessing
        ps->q[i].predicted = 0;
        // a prediction the last call left stays (it is only a guess: checked)
    }
    for (int i = 0; i < 3; ++i) {
        ps->lam1[i] = 0ull;
        ps->bad1[i] = 0u;
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
    hipLaunchKernelGGL(pair_predict_kernel, dim3(PRED_BLOCKS), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int WPB>
static hipError_t launch_pair_w(const Pair2DArgs& a, bool tape, int max_blocks, hipStream_t s) {
    int nblocks = (a.ntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    // per-step speeds with a candidate list: the form that lists candidates
    const bool cand = a.cand != nullptr && a.lam_mode == LAM_PER_STEP && !tape;
    if (cand)
        hipLaunchKernelGGL((step2d_pair<WPB, false, true>), dim3(nblocks), dim3(64 * WPB), 0, s, a);
    else if (tape)
        hipLaunchKernelGGL((step2d_pair<WPB, true, false>), dim3(nblocks), dim3(64 * WPB), 0, s, a);
    else
        hipLaunchKernelGGL((step2d_pair<WPB, false, false>), dim3(nblocks), dim3(64 * WPB), 0, s,
                           a);
    return hipGetLastError();
}

template <int WPB>
static int pair_blocks_w(bool cand) {
    int n = 0, m = 0;
    hipError_t e, f;
    if (cand) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2d_pair<WPB, false, true>,
                                                         64 * WPB, 0);
        f = e;
        m = n;
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2d_pair<WPB, false, false>,
                                                         64 * WPB, 0);
        f = hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, step2d_pair<WPB, true, false>,
                                                         64 * WPB, 0);
    }
    if (e != hipSuccess || f != hipSuccess) return 1;
    n = n < m ? n : m;  // one persistent grid size serves both plain forms
    return n > 0 ? n : 1;
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

int step2d_pair_blocks_per_cu(int wpb, bool cand) {
#define LBRS_CASE(W) \
    if (wpb == W) return pair_blocks_w<W>(cand);
    LBRS_PAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

template <int WPB>
static hipError_t launch_batch_pair_w(const Batch2DArgs& a, bool tape, int max_blocks,
                                      hipStream_t s) {
    long long nblocks = (a.pntiles + WPB - 1) / WPB;
    if (max_blocks > 0 && nblocks > max_blocks) nblocks = max_blocks;
    if (tape)
        hipLaunchKernelGGL((step2d_batch_pair<WPB, true>), dim3((unsigned)nblocks), dim3(64 * WPB),
                           0, s, a);
    else
        hipLaunchKernelGGL((step2d_batch_pair<WPB, false>), dim3((unsigned)nblocks),
                           dim3(64 * WPB), 0, s, a);
    return hipGetLastError();
}

template <int WPB>
static int batch_pair_blocks_w() {
    int n = 0, m = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2d_batch_pair<WPB, false>,
                                                                64 * WPB, 0);
    hipError_t f = hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, step2d_batch_pair<WPB, true>,
                                                                64 * WPB, 0);
    if (e != hipSuccess || f != hipSuccess) return 1;
    n = n < m ? n : m;
    return n > 0 ? n : 1;
}

hipError_t launch_step2d_batch_pair(const Batch2DArgs& a, int wpb, bool tape, int max_blocks,
                                    hipStream_t s) {
#define LBRS_CASE(W) \
    if (wpb == W) return launch_batch_pair_w<W>(a, tape, max_blocks, s);
    LBRS_PAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return hipErrorInvalidValue;
}

int step2d_batch_pair_blocks_per_cu(int wpb) {
#define LBRS_CASE(W) \
    if (wpb == W) return batch_pair_blocks_w<W>();
    LBRS_PAIR_WPB_CASES(LBRS_CASE)
#undef LBRS_CASE
    return 1;
}

}  // namespace lbrs
