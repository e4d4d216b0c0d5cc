// Host-only driver for the sanitizer test: builds the operator tables of every element type and
// degree and runs the load-balance attribution on random schedules, under AddressSanitizer and
// UndefinedBehaviorSanitizer (no device code is compiled or called).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2511_08020_amd/csrc/balance.h"
#include "../../paper_2511_08020_amd/csrc/pdg_internal.h"

namespace pdg {
void set_error(const std::string &) {}
}  // namespace pdg

int main() {
    using namespace pdg;
    double checksum = 0.0;
    for (int t = 0; t < 4; ++t)
        for (int N = 2; N <= kMaxN; ++N) {
            TypeTables tt;
            build_type_tables(t, N, tt);
            for (double v : tt.dhat[0]) checksum += v;
            for (double v : tt.dskew[0]) checksum += v;
            if (t != PDG_HEX) {
                for (double v : tt.Minv) checksum += v;
                for (double v : tt.MVtW) checksum += v;
                const std::vector<double> P = pack_rows(tt.MVtW, tt.m, tt.nn);
                for (double v : P) checksum += v;
            }
        }
    std::mt19937_64 rng(7);
    for (int rep = 0; rep < 50; ++rep) {
        const int n = 1 + (int)(rng() % 3000), nq = 1 + (int)(rng() % 300);
        std::vector<int8_t> et(n);
        for (auto &x : et) x = (int8_t)(rng() % 4);
        std::vector<int32_t> qb(nq + 1);
        qb[0] = 0;
        qb[nq] = n;
        for (int q = 1; q < nq; ++q) qb[q] = (int32_t)(rng() % (n + 1));
        std::sort(qb.begin() + 1, qb.end() - 1);
        std::vector<double> ms((size_t)kPhases * nq);
        for (auto &x : ms) x = (double)(rng() % 1000) * 1e-3;
        ms[0] += 1.0;
        if (!check_schedule(n, nq, qb.data()).empty()) return 2;
        std::vector<double> cost;
        double tc[kPhases * 4];
        attribute_costs(n, et.data(), nq, qb.data(), ms.data(), cost, tc);
        std::vector<uint32_t> w(n);
        cost_weights(n, cost, w.data());
        const std::vector<double> L = queue_loads(n, cost, nq, qb.data());
        checksum += queue_imbalance(L, nq) + w[0];
    }
    std::printf("ok %.6e\n", checksum);
    return std::isfinite(checksum) ? 0 : 1;
}
