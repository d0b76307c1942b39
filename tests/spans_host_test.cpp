// Host test of dare::SpanUnion (the server's device-time accounting): random spans reported in
// completion order with the tightest horizon the scheduler could state, against a brute-force
// union; built with g++ and AddressSanitizer/UBSan.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <utility>
#include <vector>

#include "dare_spans.h"

static double brute_union(std::vector<std::pair<double, double>> v) {
    std::sort(v.begin(), v.end());
    double u = 0.0, a = 0.0, b = -1e300;
    bool any = false;
    for (auto& iv : v) {
        if (!any || iv.first > b) {
            if (any) u += b - a;
            a = iv.first;
            b = iv.second;
            any = true;
        } else {
            b = std::max(b, iv.second);
        }
    }
    if (any) u += b - a;
    return u;
}

int main() {
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; ++trial) {
        const int streams = 1 + (int)(rng() % 4);
        const int n = 1 + (int)(rng() % 3000);
        // spans per stream, sequential on their stream, streams overlapping each other
        std::vector<std::pair<double, double>> all;
        std::vector<double> clock(streams, 0.0);
        std::uniform_real_distribution<double> gap(0.0, 2e-4), len(1e-6, 5e-4);
        std::vector<int> owner;
        for (int k = 0; k < n; ++k) {
            const int s = (int)(rng() % streams);
            const double t0 = clock[s] + gap(rng), t1 = t0 + len(rng);
            clock[s] = t1;
            all.emplace_back(t0, t1);
            owner.push_back(s);
        }
        // report in order of end; the horizon is the earliest start among spans not yet reported
        std::vector<int> order(n);
        for (int k = 0; k < n; ++k) order[k] = k;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return all[x].second < all[y].second; });
        std::vector<double> later_min(n + 1, 1e300);
        for (int r = n - 1; r >= 0; --r) later_min[r] = std::min(later_min[r + 1], all[order[r]].first);
        dare::SpanUnion u;
        double sum = 0.0;
        for (int r = 0; r < n; ++r) {
            const auto& iv = all[order[r]];
            u.add(iv.first, iv.second, later_min[r + 1]);
            sum += iv.second - iv.first;
        }
        const double want = brute_union(all), got = u.busy();
        if (std::fabs(got - want) > 1e-9 * std::max(1.0, want) || std::fabs(u.sum() - sum) > 1e-9) {
            std::printf("trial %d: union %.12g vs %.12g, sum %.12g vs %.12g\n", trial, got, want, u.sum(), sum);
            return 1;
        }
        if (n > 1000 && u.pending() > 600) {   // folding keeps the open list short
            std::printf("trial %d: %zu spans still open\n", trial, u.pending());
            return 1;
        }
    }
    // no horizon ever: nothing folds, the union is still right
    dare::SpanUnion u;
    std::vector<std::pair<double, double>> v;
    for (int k = 0; k < 1000; ++k) {
        const double t0 = (double)(k % 37) * 1e-3, t1 = t0 + 5e-4 + 1e-5 * (k % 5);
        v.emplace_back(t0, t1);
        u.add(t0, t1, -1e300);
    }
    if (std::fabs(u.busy() - brute_union(v)) > 1e-12) {
        std::printf("no-horizon union wrong\n");
        return 1;
    }
    std::printf("spans host test ok\n");
    return 0;
}
