// Error reporting and argument validation shared by the entry points.
#include <cmath>

#include "pr_internal.hpp"

namespace pr {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

int check_sde(const pr_sde *s) {
    PR_REQUIRE(s != nullptr, "sde is NULL");
    PR_REQUIRE(valid_d(s->d_fast), "d_fast = %d not served (1, 2, 3, 4, 8, 16, 32)", s->d_fast);
    PR_REQUIRE(valid_precision(s->precision), "precision = %d (64 or 32)", s->precision);
    PR_REQUIRE(std::isfinite(s->eps) && s->eps > 0, "eps must be > 0");
    PR_REQUIRE(std::isfinite(s->beta) && s->beta > 0, "beta must be > 0");
    PR_REQUIRE(std::isfinite(s->lambda) && std::isfinite(s->c3) && std::isfinite(s->c1),
               "lambda, c3, c1 must be finite");
    return PR_OK;
}

int check_schedule(const pr_schedule *s) {
    PR_REQUIRE(s != nullptr, "schedule is NULL");
    PR_REQUIRE(s->n_slices >= 1, "n_slices must be >= 1");
    PR_REQUIRE(s->total_steps >= s->n_slices, "total_steps must be >= n_slices");
    PR_REQUIRE(s->total_steps <= 0xFFFFFFFFll, "total_steps must fit the 32-bit step counter");
    PR_REQUIRE(std::isfinite(s->dt) && s->dt > 0, "dt must be > 0");
    return PR_OK;
}

int check_grid(const pr_grid *g) {
    PR_REQUIRE(g != nullptr, "grid is NULL");
    PR_REQUIRE(g->n_cells >= 3 && g->n_cells <= 4096, "n_cells must be in [3, 4096]");
    PR_REQUIRE(std::isfinite(g->x_lo) && std::isfinite(g->x_hi) && g->x_lo < g->x_hi,
               "need finite x_lo < x_hi");
    PR_REQUIRE(g->n_q >= 2 && g->n_q <= 4096, "n_q must be in [2, 4096]");
    return PR_OK;
}

}  // namespace pr

extern "C" const char *pr_last_error(void) { return pr::g_err.c_str(); }

extern "C" int pr_version(void) { return 1; }
