// Sanitizer driver of the library's host-side checks (CPU, no HIP): parameter
// validation over random and edge-case parameter sets, and the node codes of
// random solid bodies on grids with every side combination.  Built from
// csrc/lbrs_host.cpp with -fsanitize=address,undefined by
// tests/test_sanitizers.py; any report ends the run with a non-zero status.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "lbrs_host.hpp"

using namespace lbrs;

int main() {
    std::mt19937_64 rng(7);
    auto pick = [&](int n) { return (int)(rng() % (unsigned)n); };
    auto real = [&](double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); };
    const double specials[] = {0.0, -1.0, 1.0, 0.5, 2.0, 1e300, -1e300, NAN, INFINITY, 2.0 / 3.0};
    long ok = 0, rejected = 0;
    for (int it = 0; it < 200000; ++it) {
        lbrs_params p{};
        p.model = pick(5) - 1;
        p.nx = pick(4) == 0 ? pick(6) - 1 : 3 + pick(100);
        p.ny = p.model == LBRS_D2Q4 ? (pick(4) == 0 ? pick(6) - 1 : 3 + pick(100)) : (pick(8) ? 1 : 2);
        p.x0 = pick(8) ? 0.0 : specials[pick(10)];
        p.x1 = pick(8) ? 1.0 : specials[pick(10)];
        p.y0 = 0.0;
        p.y1 = pick(6) ? (double)p.ny / (p.nx > 0 ? p.nx : 1) : real(0.1, 2.0);
        p.gamma = pick(8) ? 1.4 : specials[pick(10)];
        p.omega = pick(6) ? real(0.01, 1.99) : specials[pick(10)];
        p.cfl = pick(6) ? real(0.01, 1.0) : specials[pick(10)];
        for (int s = 0; s < 4; ++s) p.bc[s] = pick(10) ? pick(4) : pick(9) - 3;
        p.lambda_mode = pick(10) ? pick(3) : pick(7) - 2;
        p.lambda_user = pick(4) ? real(0.1, 10.0) : specials[pick(10)];
        p.layout = pick(10) ? pick(2) : 5;
        static double dummy[8];
        for (int s = 0; s < 4; ++s) p.dirichlet[s] = pick(3) ? nullptr : dummy;
        p.law = pick(10) ? pick(2) : 3;
        for (int k = 0; k < 4; ++k) p.scalar_flux[k] = pick(10) ? real(-1, 1) : specials[pick(10)];
        std::vector<unsigned char> mask;
        if (p.model == LBRS_D2Q4 && p.nx > 0 && p.ny > 0 && pick(4) == 0) {
            mask.assign((size_t)p.nx * p.ny, 0);
            for (int b = 0; b < 1 + pick(4); ++b) {
                int w = 1 + pick(6), h = 1 + pick(6), x0 = pick(p.nx), y0 = pick(p.ny);
                for (int y = y0; y < y0 + h && y < p.ny; ++y)
                    for (int x = x0; x < x0 + w && x < p.nx; ++x) mask[(size_t)y * p.nx + x] = 1;
            }
            p.solid = mask.data();
        }
        const int rc = check_params(&p);
        if (rc == LBRS_OK) {
            ++ok;
            volatile long long cells = fcells(&p) * nq(p.model) * nk(&p);
            (void)cells;
            if (p.solid) {
                std::vector<unsigned short> codes((size_t)p.nx * p.ny);
                (void)build_body_codes(&p, codes.data());
            }
        } else {
            ++rejected;
        }
    }
    // wide grids of random bodies with every side combination
    for (int it = 0; it < 400; ++it) {
        lbrs_params p{};
        p.model = LBRS_D2Q4;
        p.nx = 8 + pick(60);
        p.ny = 8 + pick(40);
        p.x1 = 1.0;
        p.y1 = (double)p.ny / p.nx;
        p.gamma = 1.4;
        p.omega = 1.0;
        p.cfl = 0.5;
        const int sx = pick(3), sy = pick(3);
        p.bc[0] = p.bc[1] = sx;
        p.bc[2] = p.bc[3] = sy;
        std::vector<unsigned char> mask((size_t)p.nx * p.ny, 0);
        for (int b = 0; b < 1 + pick(6); ++b) {
            int w = 2 + pick(8), h = 2 + pick(8), x0 = pick(p.nx), y0 = pick(p.ny);
            for (int y = y0; y < y0 + h && y < p.ny; ++y)
                for (int x = x0; x < x0 + w && x < p.nx; ++x) mask[(size_t)y * p.nx + x] = 1;
        }
        p.solid = mask.data();
        if (check_params(&p) != LBRS_OK) return 3;
        std::vector<unsigned short> codes((size_t)p.nx * p.ny);
        (void)build_body_codes(&p, codes.data());
    }
    if (ok == 0 || rejected == 0) return 4;
    std::printf("host-check sanitizer driver: %ld accepted, %ld rejected, clean\n", ok, rejected);
    return 0;
}
