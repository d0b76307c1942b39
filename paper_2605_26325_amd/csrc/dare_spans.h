// Union of time spans whose ends arrive in any order, kept compact: spans that no later span
// can overlap are folded into a running total.  Used by the server for the device time of its
// ticks' kernels (ticks on different streams overlap).  Plain C++, no HIP.
#pragma once

#include <algorithm>
#include <utility>
#include <vector>

namespace dare {

class SpanUnion {
public:
    // Add the span [t0, t1] (t1 >= t0).  The caller promises that no span added later starts
    // before `horizon`: every span that ends by then can be folded.
    void add(double t0, double t1, double horizon) {
        sum_ += t1 - t0;
        open_.emplace_back(t0, t1);
        if (open_.size() < kFoldAt) return;
        std::sort(open_.begin(), open_.end());
        std::vector<std::pair<double, double>> keep;
        double a = open_[0].first, b = open_[0].second;
        auto flush = [&](double x, double y) {
            if (y <= horizon) folded_ += y - x;
            else keep.emplace_back(x, y);
        };
        for (size_t k = 1; k < open_.size(); ++k) {
            if (open_[k].first <= b) {
                b = std::max(b, open_[k].second);
            } else {
                flush(a, b);
                a = open_[k].first;
                b = open_[k].second;
            }
        }
        flush(a, b);
        open_.swap(keep);
    }
    // Length of the union of every span added so far.
    double busy() const {
        std::vector<std::pair<double, double>> v(open_);
        std::sort(v.begin(), v.end());
        double u = folded_, b = -1e300;
        for (const auto& iv : v) {
            if (iv.second <= b) continue;
            u += iv.second - std::max(iv.first, b);
            b = iv.second;
        }
        return u;
    }
    double sum() const { return sum_; }
    size_t pending() const { return open_.size(); }

private:
    static constexpr size_t kFoldAt = 256;
    double sum_ = 0.0, folded_ = 0.0;
    std::vector<std::pair<double, double>> open_;
};

}  // namespace dare
