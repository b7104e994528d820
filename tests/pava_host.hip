// Host harness for the library's sparse pool-adjacent-violators pass (the
// same source the kernels inline), used by the CPU tests to compare it bit
// for bit with the oracle's stack form.
#include <vector>

#include "pr_coarse_dev.hpp"

// v[0..L) in place; returns the number of pools of more than one value.
extern "C" int pv_pava_sparse(double *v, int L) {
    std::vector<int> vio;
    for (int j = 0; j + 1 < L; ++j)
        if (v[j] > v[j + 1]) vio.push_back(j);
    if (vio.empty()) return 0;
    std::vector<double> S(L);
    std::vector<int> SC(L);
    int np = 0;
    pr::pava_sparse(v, L, vio.data(), (int)vio.size(), S.data(), SC.data(), &np);
    for (int b = 0; b < np; ++b) {
        const int c = SC[b] & 0xFFFF, st = SC[b] >> 16;
        const double mean = S[b] / (double)c;
        for (int t = 0; t < c; ++t) v[st + t] = mean;
    }
    return np;
}
