// Load balance from measured work-queue times (host only); the interface is described in
// balance.h.
#include "balance.h"

#include <algorithm>
#include <cmath>

namespace pdg {

double queue_imbalance(const std::vector<double> &load, int32_t nq) {
    double worst = 0.0, mean = 0.0;
    for (int ph = 0; ph < kPhases; ++ph) {
        double mx = 0.0, sum = 0.0;
        for (int q = 0; q < nq; ++q) {
            mx = std::max(mx, load[(size_t)ph * nq + q]);
            sum += load[(size_t)ph * nq + q];
        }
        worst += mx;
        mean += sum / nq;
    }
    return mean > 0.0 ? worst / mean - 1.0 : 0.0;
}

std::string check_schedule(int32_t n, int32_t nq, const int32_t *qb) {
    if (nq <= 0) return "n_queues must be positive";
    if (qb[0] != 0 || qb[nq] != n) return "queue_begin must start at 0 and end at n_elems";
    for (int q = 0; q < nq; ++q)
        if (qb[q + 1] < qb[q]) return "queue_begin must be non-decreasing";
    return {};
}

namespace {

// Solves the symmetric system A x = b of size k (row stride 4) by Gaussian elimination with
// partial pivoting; a tiny ridge keeps collinear type mixes solvable.
void solve_small(int k, const double A0[4][4], const double b0[4], double x[4]) {
    double A[4][5];
    double dmax = 0.0;
    for (int i = 0; i < k; ++i) dmax = std::max(dmax, A0[i][i]);
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j < k; ++j) A[i][j] = A0[i][j] + (i == j ? 1e-12 * dmax : 0.0);
        A[i][k] = b0[i];
    }
    for (int c = 0; c < k; ++c) {
        int p = c;
        for (int r = c + 1; r < k; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[p][c])) p = r;
        for (int j = 0; j <= k; ++j) std::swap(A[c][j], A[p][j]);
        const double d = A[c][c];
        for (int r = c + 1; r < k; ++r) {
            const double f = d != 0.0 ? A[r][c] / d : 0.0;
            for (int j = c; j <= k; ++j) A[r][j] -= f * A[c][j];
        }
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = A[i][k];
        for (int j = i + 1; j < k; ++j) s -= A[i][j] * x[j];
        x[i] = A[i][i] != 0.0 ? s / A[i][i] : 0.0;
    }
}

// Non-negative least squares over the types in `present`: min sum_q (sum_t C[q][t] c_t - t_q)^2
// with c >= 0, by the active-set rule of dropping the most negative coefficient and re-solving.
void fit_type_costs(const std::vector<int64_t> &C, const double *t, int32_t nq, const bool present[4],
                    double c[4]) {
    double G[4][4] = {}, r[4] = {};
    for (int q = 0; q < nq; ++q)
        for (int i = 0; i < 4; ++i) {
            const double ci = (double)C[(size_t)q * 4 + i];
            r[i] += ci * t[q];
            for (int j = 0; j < 4; ++j) G[i][j] += ci * (double)C[(size_t)q * 4 + j];
        }
    bool act[4];
    for (int i = 0; i < 4; ++i) { act[i] = present[i]; c[i] = 0.0; }
    for (int it = 0; it < 4; ++it) {
        int idx[4], k = 0;
        for (int i = 0; i < 4; ++i)
            if (act[i]) idx[k++] = i;
        if (k == 0) break;
        double A[4][4], b[4], x[4] = {};
        for (int i = 0; i < k; ++i) {
            b[i] = r[idx[i]];
            for (int j = 0; j < k; ++j) A[i][j] = G[idx[i]][idx[j]];
        }
        solve_small(k, A, b, x);
        int worst = -1;
        for (int i = 0; i < k; ++i)
            if (x[i] <= 0.0 && (worst < 0 || x[i] < x[worst])) worst = i;
        if (worst < 0) {
            for (int i = 0; i < k; ++i) c[idx[i]] = x[i];
            return;
        }
        act[idx[worst]] = false;
    }
}

}  // namespace

void attribute_costs(int32_t n, const int8_t *etype, int32_t nq, const int32_t *qb, const double *qms,
                     std::vector<double> &cost, double type_cost[kPhases * 4]) {
    std::vector<int64_t> C((size_t)nq * 4, 0);
    int64_t total[4] = {};
    for (int q = 0; q < nq; ++q)
        for (int e = qb[q]; e < qb[q + 1]; ++e) {
            ++C[(size_t)q * 4 + etype[e]];
            ++total[etype[e]];
        }
    bool present[4];
    for (int t = 0; t < 4; ++t) present[t] = total[t] > 0;
    cost.assign((size_t)kPhases * n, 0.0);
    for (int ph = 0; ph < kPhases; ++ph) {
        const double *t = qms + (size_t)ph * nq;
        double c[4];
        fit_type_costs(C, t, nq, present, c);
        double cmax = 0.0;
        for (int i = 0; i < 4; ++i) cmax = std::max(cmax, c[i]);
        if (cmax <= 0.0) {  // no usable fit: the mean cost per element for every type
            double tt = 0.0;
            for (int q = 0; q < nq; ++q) tt += t[q];
            cmax = tt / std::max<int64_t>(1, n);
            for (int i = 0; i < 4; ++i) c[i] = cmax;
        }
        // a type the fit drops still takes a small share of its queue's time
        for (int i = 0; i < 4; ++i) {
            c[i] = present[i] ? std::max(c[i], 1e-3 * cmax) : 0.0;
            type_cost[ph * 4 + i] = c[i];
        }
        double *ce = cost.data() + (size_t)ph * n;
        for (int q = 0; q < nq; ++q) {
            double den = 0.0;
            for (int e = qb[q]; e < qb[q + 1]; ++e) den += c[etype[e]];
            if (den <= 0.0) continue;
            for (int e = qb[q]; e < qb[q + 1]; ++e) ce[e] = t[q] * c[etype[e]] / den;
        }
    }
}

void cost_weights(int32_t n, const std::vector<double> &cost, uint32_t *weight) {
    std::vector<double> tot(n, 0.0);
    double sum = 0.0;
    for (int ph = 0; ph < kPhases; ++ph)
        for (int e = 0; e < n; ++e) tot[e] += cost[(size_t)ph * n + e];
    for (int e = 0; e < n; ++e) sum += tot[e];
    const double mean = sum / std::max(1, n);
    for (int e = 0; e < n; ++e) {
        const double w = mean > 0.0 ? std::round(1024.0 * tot[e] / mean) : 1024.0;
        weight[e] = (uint32_t)std::min(16777216.0, std::max(1.0, w));
    }
}

std::vector<double> queue_loads(int32_t n, const std::vector<double> &cost, int32_t nq, const int32_t *qb) {
    std::vector<double> L((size_t)kPhases * nq, 0.0);
    for (int ph = 0; ph < kPhases; ++ph)
        for (int q = 0; q < nq; ++q) {
            double s = 0.0;
            for (int e = qb[q]; e < qb[q + 1]; ++e) s += cost[(size_t)ph * n + e];
            L[(size_t)ph * nq + q] = s;
        }
    return L;
}

}  // namespace pdg
