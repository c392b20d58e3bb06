// MC64 maximum-product matching and scaling on the host (Alg. 3 step 1 of
// the paper, Sec. 3.3; Duff and Koster, SIAM J. Matrix Anal. Appl. 22
// (2001) 973).  The matching is the minimum-cost perfect assignment of rows
// to columns with costs c_ij = log(max_k |a_kj|) - log|a_ij| on the
// nonzeros, found by successive shortest augmenting paths (Dijkstra on
// reduced costs with a binary heap, after a greedy start on the tight
// entries).  The dual variables u (rows) and v (columns), with
// c_ij - u_i - v_j >= 0 and equality on the matching, give the scalings
// dr_i = exp(u_i) and dc_j = exp(v_j) / max_k |a_kj|, under which every
// |dr_i a_ij dc_j| <= 1 and the matched entries have magnitude 1.
// Sequential graph work on the sparse pattern, run once per pattern.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <limits>
#include <queue>
#include <utility>
#include <vector>

namespace sdsl {

bool mc64_match(int n, const int64_t* rp, const int* ci, const double* v, std::vector<int>& match,
                std::vector<double>& dr, std::vector<double>& dc) {
    const int64_t nnz = rp[n];
    std::vector<double> colmax(n, 0.0);
    for (int64_t p = 0; p < nnz; ++p) colmax[ci[p]] = std::max(colmax[ci[p]], std::fabs(v[p]));
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<double> cost(nnz, inf);
    for (int64_t p = 0; p < nnz; ++p)
        if (v[p] != 0.0) cost[p] = std::log(colmax[ci[p]]) - std::log(std::fabs(v[p]));
    // row potentials start at the row minima, column potentials at 0, so
    // every reduced cost is >= 0
    std::vector<double> u(n, inf), w(n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) u[i] = std::min(u[i], cost[p]);
    for (int i = 0; i < n; ++i)
        if (!(u[i] < inf)) return false;  // a row without nonzeros
    match.assign(n, -1);
    std::vector<int> owner(n, -1);  // column -> row
    for (int i = 0; i < n; ++i)     // greedy start on tight entries
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (cost[p] == u[i] && owner[ci[p]] < 0) {
                match[i] = ci[p];
                owner[ci[p]] = i;
                break;
            }
    std::vector<double> dist(n, inf);   // tentative column distances
    std::vector<int> from(n, -1);       // row that reached the column
    std::vector<char> done(n, 0);       // column finalised
    std::vector<int> touched, fin_cols;
    std::vector<std::pair<int, double>> fin_rows;
    using Item = std::pair<double, int>;
    for (int i0 = 0; i0 < n; ++i0) {
        if (match[i0] >= 0) continue;
        std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
        fin_rows.clear();
        fin_cols.clear();
        auto relax = [&](int r, double dr_) {
            fin_rows.push_back({r, dr_});
            for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
                if (!(cost[p] < inf)) continue;
                const int j = ci[p];
                if (done[j]) continue;
                const double nd = dr_ + std::max(0.0, cost[p] - u[r] - w[j]);
                if (nd < dist[j]) {
                    if (!(dist[j] < inf)) touched.push_back(j);
                    dist[j] = nd;
                    from[j] = r;
                    heap.push({nd, j});
                }
            }
        };
        relax(i0, 0.0);
        int jfree = -1;
        double D = 0.0;
        while (!heap.empty()) {
            const auto [d, j] = heap.top();
            heap.pop();
            if (done[j] || d > dist[j]) continue;
            done[j] = 1;
            fin_cols.push_back(j);
            if (owner[j] < 0) {
                jfree = j;
                D = d;
                break;
            }
            relax(owner[j], d);
        }
        if (jfree < 0) return false;  // no augmenting path: structurally singular
        // potentials: finalised rows rise by D - their distance, finalised
        // columns fall by D - theirs; the path's entries become tight
        for (const auto& [r, dr_] : fin_rows) u[r] += D - dr_;
        for (int j : fin_cols) w[j] -= D - dist[j];
        for (int j = jfree;;) {  // flip the path
            const int i = from[j];
            const int jn = match[i];
            match[i] = j;
            owner[j] = i;
            if (i == i0) break;
            j = jn;
        }
        for (int j : touched) {
            dist[j] = inf;
            from[j] = -1;
            done[j] = 0;
        }
        touched.clear();
    }
    dr.resize(n);
    dc.resize(n);
    for (int i = 0; i < n; ++i) dr[i] = std::exp(u[i]);
    for (int j = 0; j < n; ++j) dc[j] = colmax[j] > 0.0 ? std::exp(w[j]) / colmax[j] : 1.0;
    return true;
}

}  // namespace sdsl
