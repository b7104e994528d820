// Internal interface of the models beside the double-well SDE: the
// chemical-reaction system (Sec. 2.1.2: fine propagator, initial law, coarse
// propagator) and the linear-advection coarse model (Sec. 6); and the coarse
// constructor from a tridiagonal generator that every coarse model shares.
#pragma once

#include <vector>

#include "pr_internal.hpp"

namespace pr {

int check_chem(const pr_chem *c);
int chem_init_ensemble(const pr_chem *c, uint64_t seed, uint32_t inst, int64_t n, double *x, double *y,
                       hipStream_t st);
int chem_fine_propagate(const pr_chem *c, const pr_schedule *sch, uint64_t seed, uint32_t inst, int64_t n,
                        int slice_first, int slice_count, const double *xi, const double *yi, double *x, double *y,
                        hipStream_t st);
int chem_mean_fast(const pr_chem *c, double *ybar);
int chem_coarse_create(const pr_chem *c, const pr_schedule *sch, const pr_grid *grid, hipStream_t st, Coarse **out);

int advection_coarse_create(double eps, double beta, const pr_schedule *sch, const pr_grid *grid, hipStream_t st,
                            Coarse **out);
int coarse_n_slices(const Coarse *c);
int coarse_grid_cells(const Coarse *c);

// Coarse handle from the generator A (lo[i] = A[i][i-1], di[i] = A[i][i],
// up[i] = A[i][i+1]): E(tau) for every distinct slice length of sch.
int coarse_create_tridiag(const std::vector<double> &lo, const std::vector<double> &di,
                          const std::vector<double> &up, const pr_schedule *sch, const pr_grid *grid, hipStream_t st,
                          Coarse **out);

}  // namespace pr
