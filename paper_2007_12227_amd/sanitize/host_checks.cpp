// host_checks.cpp -- the library's GPU-free host code under AddressSanitizer
// and UndefinedBehaviorSanitizer: argument validation, workspace sizing, the
// source-box planner over random geometries (each box checked to contain every
// node whose moved basis function reaches the tile, by brute force), status
// strings and refusals that return before any device call.  Built with the
// sanitizers on the host side only; runs without a GPU.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>

#include "vp.h"

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

int main() {
    std::mt19937_64 rng(12);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    // workspace sizing and invalid axes
    vp_axis x{-M_PI, M_PI, 64, 1}, p{-3.0, 3.0, 48, 0};
    CHECK(vp_workspace_bytes(&x, &p) > 0);
    vp_axis bad{1.0, 0.0, 64, 1};
    CHECK(vp_workspace_bytes(&bad, &p) == 0);
    CHECK(vp_workspace_bytes(nullptr, &p) == 0);
    vp_axis ax4[4] = {x, x, p, p};
    CHECK(vp4_workspace_bytes(ax4) > 0);
    ax4[3].n = 2;
    CHECK(vp4_workspace_bytes(ax4) == 0);
    // refusals that return before touching the device
    vp_grid* g = nullptr;
    vp_grid_desc d{};
    d.x = x;
    d.p = p;
    CHECK(vp_create_grid(&d, &g) == VP_ENOMEM && g == nullptr);
    d.p.periodic = 1;
    CHECK(vp_create_grid(&d, &g) == VP_EUNSUPPORTED);
    CHECK(vp_create_grid(nullptr, &g) == VP_EINVAL);
    CHECK(vp_step(nullptr, 0.1, 1) == VP_EINVAL);
    CHECK(vp_moments(nullptr, nullptr) == VP_EINVAL);
    CHECK(vp_destroy_grid(nullptr) == VP_OK);
    CHECK(vp_batch_create(nullptr, 0, nullptr, nullptr) == VP_EINVAL);
    CHECK(vp_set_fixed_point(nullptr, 0) == VP_EINVAL);
    CHECK(vp_get_run_state(nullptr, nullptr) == VP_EINVAL);
    vp4_grid* g4 = nullptr;
    vp4_grid_desc d4{};
    CHECK(vp4_create_grid(&d4, &g4) == VP_EINVAL);
    for (int s = -8; s <= 1; ++s) CHECK(vp_status_string(s) != nullptr && strlen(vp_status_string(s)) > 0);
    CHECK(strlen(vp_last_error()) > 0);
    // the source-box planner against brute force (pendulum, free, oscillator; three bases)
    long boxes = 0;
    for (int trial = 0; trial < 300; ++trial) {
        const int kind = (int)(U(rng) * 3.0);  // 0 free, 1 rotation, 2 pendulum
        const int basis = (int)(U(rng) * 3.0);
        vp_axis X{-M_PI, M_PI, 16 + (int)(U(rng) * 80), kind == 1 ? 0 : 1};
        vp_axis P{-3.0, 3.0, 16 + (int)(U(rng) * 80), 0};
        if (kind == 1) X = vp_axis{-3.0, 3.0, X.n, 0};
        vp_hamiltonian h{};
        h.kind = kind == 0 ? VP_H_FREE : kind == 1 ? VP_H_SHO_EXACT : VP_H_PENDULUM;
        h.a = 0.5 + 1.5 * U(rng);
        h.omega = 1.0;
        const double dt = 0.01 + 0.3 * U(rng);
        const int bx0 = (int)(U(rng) * X.n * 0.8), by0 = (int)(U(rng) * P.n * 0.8);
        const int bx1 = bx0 + 1 + (int)(U(rng) * (X.n - bx0 - 1)), by1 = by0 + 1 + (int)(U(rng) * (P.n - by0 - 1));
        int32_t box[4];
        CHECK(vp_plan_source_box(&X, &P, &h, basis, dt, 0.0, 0.0, bx0, bx1, by0, by1, box) == VP_OK);
        ++boxes;
        const double hx = (X.hi - X.lo) / (X.periodic ? X.n : X.n - 1), hp = (P.hi - P.lo) / (P.n - 1);
        const int reach = 2 + basis;  // taps floor(u) - reach + 1 .. floor(u) + reach
        for (int j = 0; j < P.n; ++j)
            for (int i = 0; i < X.n; ++i) {
                const double x0 = X.lo + i * hx, p0 = P.lo + j * hp;
                double xn, pn;
                if (kind == 0) {
                    xn = x0 + p0 * dt;
                    pn = p0;
                } else if (kind == 1) {
                    xn = x0 * cos(dt) + p0 * sin(dt);
                    pn = -x0 * sin(dt) + p0 * cos(dt);
                } else {
                    const double xh = x0 + 0.5 * dt * p0;
                    pn = p0 - h.a * sin(xh) * dt;
                    xn = xh + 0.5 * dt * pn;
                }
                const double u = (xn - X.lo) / hx, v = (pn - P.lo) / hp;
                const long cu = (long)floor(u), cv = (long)floor(v);
                // does any tap reach the tile (columns wrap on a periodic axis)?
                bool hits_rows = cv + reach >= by0 && cv - reach + 1 < by1;
                bool hits_cols = false;
                for (long c = cu - reach + 1; c <= cu + reach && !hits_cols; ++c) {
                    long cc = X.periodic ? ((c % X.n) + X.n) % X.n : c;
                    hits_cols = cc >= bx0 && cc < bx1;
                }
                if (!(hits_rows && hits_cols)) continue;
                // the node must lie in the box (columns unwrapped)
                bool in_cols = false;
                for (long k = -2; k <= 2 && !in_cols; ++k) {
                    const long ii = i + k * X.n;
                    in_cols = ii >= box[0] && ii < box[1];
                }
                if (!X.periodic) in_cols = i >= box[0] && i < box[1];
                CHECK(in_cols && j >= box[2] && j < box[3]);
                if (!(in_cols && j >= box[2] && j < box[3])) {
                    fprintf(stderr, "  kind %d basis %d node (%d, %d) box [%d %d %d %d] tile [%d %d %d %d]\n", kind,
                            basis, i, j, box[0], box[1], box[2], box[3], bx0, bx1, by0, by1);
                    return 1;
                }
            }
    }
    printf("host checks: %ld planned boxes checked, %d failures\n", boxes, failures);
    return failures ? 1 : 0;
}
