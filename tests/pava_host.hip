// Host harness for the library's sparse pool-adjacent-violators pass (the
// same source the kernels inline), used by the CPU tests to compare it bit
// for bit with the oracle's stack form.
#include <algorithm>
#include <vector>

#include "pr_coarse_dev.hpp"

// The library's comparison of two pool means, over arrays: out[i] = 1 when
// a[i]/ca[i] > b[i]/cb[i] as the library decides it.
extern "C" void pv_mean_above(const double *a, const int *ca, const double *b, const int *cb, int n, int *out) {
    for (int i = 0; i < n; ++i) out[i] = pr::mean_above(a[i], ca[i], b[i], cb[i]) ? 1 : 0;
}

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

// The stretch decomposition of the block pass, run serially: the input cut
// where every value before is below every value after, each stretch holding
// violations by pava_sparse_range, cuts that the serial pass would cross
// dropped until none is.  Returns the rounds.
extern "C" int pv_pava_stretches(double *v, int L) {
    std::vector<int> vio;
    for (int j = 0; j + 1 < L; ++j)
        if (v[j] > v[j + 1]) vio.push_back(j);
    const int nv = (int)vio.size();
    if (nv == 0) return 0;
    // cuts: max(v[0..b)) < min(v[b..L)); last cut at or before every position
    std::vector<double> pm(L), sm(L);
    for (int j = 0; j < L; ++j) pm[j] = j ? std::max(pm[j - 1], v[j]) : v[j];
    for (int j = L - 1; j >= 0; --j) sm[j] = j + 1 < L ? std::min(sm[j + 1], v[j]) : v[j];
    std::vector<int> last(L, 0);
    for (int b = 1; b < L; ++b) last[b] = pm[b - 1] < sm[b] ? b : last[b - 1];
    std::vector<int> cb, fv;
    for (int f = 0; f < nv; ++f)
        if (f == 0 || last[vio[f]] != last[vio[f - 1]]) {
            fv.push_back(f);
            cb.push_back(f == 0 ? 0 : last[vio[f]]);
        }
    cb.push_back(L);
    fv.push_back(nv);
    std::vector<double> S(L), fm, lm;
    std::vector<int> SC(L), np;
    int rounds = 0;
    while (true) {
        ++rounds;
        const int nc = (int)cb.size() - 1;
        fm.assign(nc, 0.0);
        lm.assign(nc, 0.0);
        np.assign(nc, 0);
        for (int k = 0; k < nc; ++k)
            np[k] = pr::pava_sparse_range(v, cb[k], cb[k + 1], vio.data() + fv[k], fv[k + 1] - fv[k], S.data(),
                                          SC.data(), &fm[k], &lm[k]);
        std::vector<int> ncb{cb[0]}, nfv{fv[0]};
        for (int k = 1; k < nc; ++k)
            if (!(lm[k - 1] > fm[k])) {
                ncb.push_back(cb[k]);
                nfv.push_back(fv[k]);
            }
        if ((int)ncb.size() == nc) break;
        ncb.push_back(L);
        nfv.push_back(nv);
        cb.swap(ncb);
        fv.swap(nfv);
    }
    const int nc = (int)cb.size() - 1;
    for (int k = 0; k < nc; ++k)
        for (int b = 0; b < np[k]; ++b) {
            const int c = SC[cb[k] + b] & 0xFFFF, st = SC[cb[k] + b] >> 16;
            const double mean = S[cb[k] + b] / (double)c;
            for (int t = 0; t < c; ++t) v[st + t] = mean;
        }
    return rounds;
}
