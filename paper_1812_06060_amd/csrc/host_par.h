// Host-side parallel loops for mesh preprocessing (std::thread workers over
// contiguous index ranges).  Every use writes disjoint outputs per index or
// sorts under a total order, so results never depend on the thread count.
// HG_HOST_THREADS sets the number of workers (default: the hardware's, at
// most 16).
#pragma once
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <exception>
#include <functional>
#include <thread>
#include <vector>

namespace hg {

inline int host_threads() {
    static const int n = [] {
        const char* e = std::getenv("HG_HOST_THREADS");
        int v = e ? std::atoi(e) : 0;
        if (v <= 0) v = std::min(16, (int)std::thread::hardware_concurrency());
        return std::max(1, std::min(v, 256));
    }();
    return n;
}

// f(begin, end, part) over `parts` contiguous ranges of [0, n) (part p covers
// [p*n/parts, (p+1)*n/parts)); the first exception of the lowest part is
// rethrown after all parts have finished.
template <class F>
void parallel_parts(int64_t n, int parts, F&& f) {
    if (n <= 0) return;
    parts = (int)std::max<int64_t>(1, std::min<int64_t>(parts, n));
    auto lo = [&](int p) { return (int64_t)((__int128)n * p / parts); };
    if (parts == 1) {
        f((int64_t)0, n, 0);
        return;
    }
    std::vector<std::exception_ptr> err(parts);
    auto part = [&](int p) {
        try {
            f(lo(p), lo(p + 1), p);
        } catch (...) {
            err[p] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    std::vector<int> inline_parts{0};   // parts run on the calling thread
    th.reserve(parts - 1);
    for (int p = 1; p < parts; ++p) {
        try {
            th.emplace_back(part, p);
        } catch (...) {   // no thread to be had: run the part here
            inline_parts.push_back(p);
        }
    }
    for (int p : inline_parts) part(p);
    for (auto& t : th) t.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

// f(begin, end) over ranges of [0, n) of at least `grain` indices each.
template <class F>
void parallel_for(int64_t n, int64_t grain, F&& f) {
    const int64_t by_grain = (n + std::max<int64_t>(grain, 1) - 1) / std::max<int64_t>(grain, 1);
    const int parts = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), by_grain));
    parallel_parts(n, parts, [&](int64_t b, int64_t e, int) { f(b, e); });
}

// Sorts v under cmp, a strict total order on its elements (so the result is
// the one std::sort gives): sorted runs per worker, then rounds of pairwise
// merges.
template <class T, class Cmp>
void parallel_sort(std::vector<T>& v, Cmp cmp) {
    const int64_t n = (int64_t)v.size();
    int parts = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / 65536));
    if (parts <= 1) {
        std::sort(v.begin(), v.end(), cmp);
        return;
    }
    std::vector<int64_t> bnd(parts + 1);
    for (int p = 0; p <= parts; ++p) bnd[p] = (int64_t)((__int128)n * p / parts);
    parallel_parts(parts, parts, [&](int64_t b, int64_t e, int) {
        for (int64_t p = b; p < e; ++p) std::sort(v.begin() + bnd[p], v.begin() + bnd[p + 1], cmp);
    });
    std::vector<T> buf(n);
    std::vector<T>* src = &v;
    std::vector<T>* dst = &buf;
    while (bnd.size() > 2) {
        const int runs = (int)bnd.size() - 1;
        const int pairs = runs / 2;
        std::vector<int64_t> nb;
        for (int r = 0; r < runs; r += 2) nb.push_back(bnd[r]);
        nb.push_back(n);
        parallel_parts(pairs + (runs & 1), pairs + (runs & 1), [&](int64_t b, int64_t e, int) {
            for (int64_t q = b; q < e; ++q) {
                const int r = (int)(2 * q);
                auto s0 = src->begin() + bnd[r], s1 = src->begin() + bnd[r + 1];
                if (r + 1 < runs) {
                    auto s2 = src->begin() + bnd[r + 2];
                    std::merge(s0, s1, s1, s2, dst->begin() + bnd[r], cmp);
                } else {
                    std::copy(s0, s1, dst->begin() + bnd[r]);
                }
            }
        });
        bnd.swap(nb);
        std::swap(src, dst);
    }
    if (src != &v) v.swap(*src);
}

}  // namespace hg
