// Sanitizer driver of the oracle (CPU): every code path of lbrs_oracle.cpp on
// small problems -- all models and laws, every side condition, Dirichlet
// data, a solid body, the three lattice-speed modes, the tangent runs and the
// rejected inputs.  Built with -fsanitize=address,undefined by
// tests/test_sanitizers.py; any report ends the run with a non-zero status.
#include "../../oracle/lbrs_oracle.cpp"

#include <cstdio>

namespace {

Problem base(int model, int nx, int ny) {
    Problem P{};
    P.model = model;
    P.flux = FLUX_EULER;
    P.nx = nx;
    P.ny = ny;
    P.x0 = 0.0;
    P.x1 = 1.0;
    P.y0 = 0.0;
    P.y1 = double(ny) / nx;
    P.gamma = 1.4;
    P.omega = 1.3;
    P.cfl = model == D1Q3 ? 0.6 : 0.9;
    P.lam_mode = LAM_PER_STEP;
    P.lam_user = 0.0;
    return P;
}

// A smooth positive primitive state -> conserved U [K][ny][nx].
std::vector<double> state(const Problem& P, double phase) {
    const int K = ncomp(P);
    const long n = (long)P.nx * P.ny;
    std::vector<double> W((size_t)K * n), U((size_t)K * n);
    for (int y = 0; y < P.ny; ++y)
        for (int x = 0; x < P.nx; ++x) {
            const long c = (long)y * P.nx + x;
            const double s = std::sin(0.7 * x + 0.3 * y + phase), q = std::cos(0.4 * x - 0.9 * y);
            if (K == 1) {
                W[c] = 0.5 + 0.3 * s;
                continue;
            }
            W[c] = 1.0 + 0.3 * s;
            W[n + c] = 0.2 * q;
            if (K == 4) W[2 * n + c] = -0.1 * s;
            W[(size_t)(K - 1) * n + c] = 1.0 + 0.2 * q;
        }
    orc_prim_to_cons(&P, W.data(), U.data());
    return U;
}

int runs = 0;

int run(const Problem& P, double phase, long steps) {
    const int K = ncomp(P), Q = nq(P.model);
    const long n = (long)P.nx * P.ny;
    std::vector<double> U0 = state(P, phase), U((size_t)K * n), f((size_t)Q * K * n);
    std::vector<double> dt(steps), lam(steps);
    long ns = 0, fail = 0;
    double t = 0.0;
    int st = orc_run(&P, U0.data(), 1e9, steps, U.data(), f.data(), dt.data(), lam.data(), &ns, &t,
                     &fail);
    ++runs;
    return st;
}

void expect(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "unexpected result: %s\n", what);
        std::exit(2);
    }
}

}  // namespace

int main() {
    // 1D Euler, both models, transmissive and periodic, three speed modes
    for (int model : {D1Q2, D1Q3})
        for (int side : {SIDE_TRANSMISSIVE, SIDE_PERIODIC})
            for (int mode : {LAM_PER_STEP, LAM_FROZEN, LAM_USER}) {
                Problem P = base(model, 37, 1);
                P.side[0] = P.side[1] = side;
                P.lam_mode = mode;
                P.lam_user = 6.0;
                expect(run(P, 0.1, 20) == ST_OK, "1D Euler run");
            }
    // 2D Euler: every side combination on each axis (walls on one axis)
    const int sides[3] = {SIDE_TRANSMISSIVE, SIDE_PERIODIC, SIDE_WALL};
    for (int a : sides)
        for (int b : sides) {
            if (a == SIDE_WALL && b == SIDE_WALL) continue;
            Problem P = base(D2Q4, 19, 13);
            P.side[0] = P.side[1] = a;
            P.side[2] = P.side[3] = b;
            expect(run(P, 0.2, 12) == ST_OK, "2D Euler run");
        }
    // Dirichlet sides (prescribed states on x-low and y-high, and a periodic x)
    {
        Problem P = base(D2Q4, 17, 11);
        std::vector<double> dx = state(base(D2Q4, 11, 1), 0.5), dy = state(base(D2Q4, 17, 1), 0.9);
        // states along a side: [K][n]; reuse the first rows of two smooth fields
        std::vector<double> xs(4 * 11), ys(4 * 17);
        for (int k = 0; k < 4; ++k) {
            for (int j = 0; j < 11; ++j) xs[k * 11 + j] = dx[k * 11 + j];
            for (int j = 0; j < 17; ++j) ys[k * 17 + j] = dy[k * 17 + j];
        }
        P.side[0] = SIDE_DIRICHLET;
        P.side[3] = SIDE_DIRICHLET;
        P.dir[0] = xs.data();
        P.dir[3] = ys.data();
        expect(run(P, 0.3, 10) == ST_OK, "Dirichlet run");
        P.side[0] = P.side[1] = SIDE_PERIODIC;
        P.dir[0] = nullptr;
        expect(run(P, 0.3, 10) == ST_OK, "Dirichlet run, periodic x");
    }
    // a solid body with wall sides meeting at corners (faces, concave corners, tips)
    {
        Problem P = base(D2Q4, 24, 16);
        std::vector<unsigned char> m(24 * 16, 0);
        for (int y = 5; y < 9; ++y)
            for (int x = 6; x < 12; ++x) m[y * 24 + x] = 1;
        for (int y = 0; y < 3; ++y)
            for (int x = 16; x < 20; ++x) m[y * 24 + x] = 1;
        P.solid = m.data();
        P.side[0] = P.side[2] = SIDE_WALL;
        P.side[1] = P.side[3] = SIDE_TRANSMISSIVE;
        expect(run(P, 0.4, 15) == ST_OK, "body run");
        m[4 * 24 + 3] = 1;  // a one-cell gap to the wall: rejected
        m[4 * 24 + 1] = 1;
        expect(run(P, 0.4, 3) == ST_INVAL, "inadmissible mask rejected");
    }
    // scalar laws: linear advection and a quadratic flux, 1D and 2D, with a
    // Dirichlet side in 2D
    for (int model : {D1Q2, D1Q3, D2Q4})
        for (int fl : {FLUX_LINEAR, FLUX_QUADRATIC}) {
            Problem P = base(model, 21, model == D2Q4 ? 21 : 1);
            P.flux = fl;
            P.adv_x = 0.7;
            P.adv_y = -0.4;
            P.q[0] = 0.1;
            P.q[1] = 1.0;
            P.q[2] = 0.2;
            P.q[3] = 0.5;
            std::vector<double> ud(21, 0.6);
            if (model == D2Q4) {
                P.side[2] = SIDE_DIRICHLET;
                P.dir[2] = ud.data();
            }
            expect(run(P, 0.6, 10) == ST_OK, "scalar run");
        }
    // the tangent (dual-number) paths and single fixed steps
    {
        Problem P = base(D2Q4, 12, 12);
        P.side[0] = P.side[1] = P.side[2] = P.side[3] = SIDE_PERIODIC;
        P.lam_mode = LAM_USER;
        P.lam_user = 5.0;
        const long n = 144;
        std::vector<double> W(4 * n), dW(4 * n), U(4 * n), dU(4 * n);
        for (long c = 0; c < n; ++c) {
            W[c] = 1.0 + 0.01 * (c % 7);
            W[n + c] = W[2 * n + c] = 0.0;
            W[3 * n + c] = 1.0;
            dW[c] = 0.001 * (c % 3);
        }
        expect(orc_run_tangent(&P, W.data(), dW.data(), 1, 5.0, 6, U.data(), dU.data()) == ST_OK,
               "tangent run");
        std::vector<double> U0 = state(P, 0.7), f0(16 * n), df0(16 * n), f1(16 * n), df1(16 * n);
        expect(orc_init_tangent(&P, U0.data(), U0.data(), 5.0, f0.data(), df0.data()) == ST_OK,
               "init tangent");
        expect(orc_step_fixed(&P, f0.data(), df0.data(), 5.0, f1.data(), df1.data()) == ST_OK,
               "fixed step with tangent");
        expect(orc_step_fixed(&P, f0.data(), nullptr, 5.0, f1.data(), nullptr) == ST_OK,
               "fixed step");
        double l = orc_initial_lattice_speed(&P, U0.data());
        expect(l == 5.0, "user lattice speed");
    }
    // rejected inputs and a non-physical start
    {
        Problem P = base(D1Q3, 20, 1);
        P.cfl = 0.7;
        expect(run(P, 0.0, 2) == ST_INVAL, "cfl above 2/3 for D1Q3");
        P = base(D2Q4, 20, 10);
        P.y1 = 1.0;
        expect(run(P, 0.0, 2) == ST_INVAL, "dx != dy");
        P = base(D1Q3, 20, 1);
        const int K = 3;
        std::vector<double> U0 = state(P, 0.0), U(K * 20);
        U0[5] = -1.0;
        long ns = 0, fail = 0;
        double t = 0.0;
        expect(orc_run(&P, U0.data(), 1.0, 5, U.data(), nullptr, nullptr, nullptr, &ns, &t, &fail) ==
                   ST_NONPHYSICAL && fail == 0,
               "non-physical start");
    }
    std::printf("oracle sanitizer driver: %d runs clean\n", runs);
    return 0;
}
