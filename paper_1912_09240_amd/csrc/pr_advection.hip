// Coarse model of the linear-advection study (Sec. 6): Fbar(x) = x/eps,
// Dbar = 1/beta, tau_x = 1, on the finite-volume scheme of Sec. 2.2.2.
// rho_inf(x) ~ exp(-beta x/eps), so the coefficient a_i/g_j of the scheme is
//   Dbar/h^2 * rho_inf(x_i)/rho_inf(m_j) = Dbar/h^2 * exp(-(beta/eps)(x_i - m_j))
// with |x_i - m_j| = h/2.
#include <cmath>
#include <vector>

#include "pr_chem.hpp"

namespace pr {

int advection_coarse_create(double eps, double beta, const pr_schedule *sch, const pr_grid *grid, hipStream_t st,
                            Coarse **out) {
    const int I = grid->n_cells;
    const double h = (grid->x_hi - grid->x_lo) / I;
    const double base = (1.0 / beta) / (h * h);
    const double to_left = base * std::exp(-(beta / eps) * (0.5 * h));   // a_i / g_{i-1}: x_i - m_{i-1} = h/2
    const double to_right = base * std::exp(-(beta / eps) * (-0.5 * h));  // a_i / g_i:     x_i - m_i = -h/2
    std::vector<double> lo(I, 0.0), di(I, 0.0), up(I, 0.0);
    for (int i = 1; i < I; ++i) {
        di[i - 1] -= to_left;
        lo[i] += to_left;
        di[i] -= to_right;
        up[i - 1] += to_right;
    }
    return coarse_create_tridiag(lo, di, up, sch, grid, st, out);
}

}  // namespace pr

using namespace pr;

extern "C" int pr_advection_coarse_create(double eps, double beta, const pr_schedule *sched, const pr_grid *grid,
                                          void *stream, void **coarse) {
    clear_error();
    PR_REQUIRE(eps > 0.0 && beta > 0.0 && std::isfinite(eps) && std::isfinite(beta), "need eps > 0 and beta > 0");
    PR_CHECK(check_schedule(sched));
    PR_CHECK(check_grid(grid));
    PR_REQUIRE(coarse != nullptr, "coarse must be non-NULL");
    Coarse *p = nullptr;
    PR_CHECK(advection_coarse_create(eps, beta, sched, grid, as_stream(stream), &p));
    *coarse = p;
    return PR_OK;
}
