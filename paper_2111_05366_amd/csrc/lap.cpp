// Host linear assignment for the final projection of Alg. 3 (and the
// direction step of Alg. 1): maximise sum_i M[i][perm[i]] over permutations.
//
// Successive shortest augmenting paths (the Hungarian / Jonker-Volgenant
// family) on costs c = -M with row and column duals u, v: a greedy start
// matches each row to its cheapest column when that column is free; every
// row still free is matched by one Dijkstra search over reduced costs
// c_ij - u_i - v_j, a dual update and an augmentation along the found path.
// Among columns of equal tentative distance the lowest index is scanned
// first, so results are deterministic.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "common.h"

namespace goat {

int lap_max(int n, const double* M, int ld, int32_t* perm) {
    if (n < 1 || !M || !perm || ld < n) {
        set_error("goat_lap_max: bad arguments");
        return GOAT_EINVAL;
    }
    const double INF = std::numeric_limits<double>::infinity();
    for (size_t k = 0; k < (size_t)n * ld; ++k) {
        if ((k % ld) < (size_t)n && !std::isfinite(M[k])) {
            set_error("goat_lap_max: non-finite entry");
            return GOAT_EINVAL;
        }
    }

    std::vector<double> u(n, 0.0), v(n, 0.0), d(n);
    std::vector<int> col_of(n, -1), row_of(n, -1), pred(n);
    std::vector<char> row_seen(n), col_done(n);
    std::vector<int> seen_rows;
    seen_rows.reserve(n);

    // Greedy start: with column duals v = 0 each row may take its cheapest
    // column (lowest index on ties) if that column is still free; u_i is then
    // the row minimum, so reduced costs c_ij - u_i - v_j are >= 0 and vanish
    // on every matched pair.
    for (int i = 0; i < n; ++i) {
        const double* row = M + (size_t)i * ld;
        int jb = 0;
        for (int j = 1; j < n; ++j)
            if (row[j] > row[jb]) jb = j;
        if (row_of[jb] < 0) {
            row_of[jb] = i;
            col_of[i] = jb;
            u[i] = -row[jb];
        }
    }

    // column scans run on several host threads for large n
    const int nth = n >= 2048 ? std::max(1, omp_get_max_threads()) : 1;
    std::vector<double> tbest(nth, INF);
    std::vector<int> tj(nth, -1);
    int tcount = 1;
    for (int f = 0; f < n; ++f) {
        if (col_of[f] >= 0) continue;
        std::fill(d.begin(), d.end(), INF);
        std::fill(row_seen.begin(), row_seen.end(), 0);
        std::fill(col_done.begin(), col_done.end(), 0);
        seen_rows.clear();
        int i = f, sink = -1;
        double dmin = 0.0;
        while (sink < 0) {
            row_seen[i] = 1;
            seen_rows.push_back(i);
            const double ui = u[i];
            const double* row = M + (size_t)i * ld;
            int jbest = -1;
            double best = INF;
            if (nth <= 1) {
                for (int j = 0; j < n; ++j) {
                    if (col_done[j]) continue;
                    const double r = dmin - row[j] - ui - v[j];
                    if (r < d[j]) { d[j] = r; pred[j] = i; }
                    if (d[j] < best) { best = d[j]; jbest = j; }
                }
            } else {
                // each thread scans one contiguous column range; the ranges are
                // combined in order, so ties still go to the lowest index
#pragma omp parallel num_threads(nth)
                {
                    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
                    const int j0 = (int)((long long)n * t / nt), j1 = (int)((long long)n * (t + 1) / nt);
                    double b = INF;
                    int jb = -1;
                    for (int j = j0; j < j1; ++j) {
                        if (col_done[j]) continue;
                        const double r = dmin - row[j] - ui - v[j];
                        if (r < d[j]) { d[j] = r; pred[j] = i; }
                        if (d[j] < b) { b = d[j]; jb = j; }
                    }
                    tbest[t] = b;
                    tj[t] = jb;
                    if (t == 0) tcount = nt;
                }
                for (int t = 0; t < tcount; ++t)
                    if (tj[t] >= 0 && tbest[t] < best) { best = tbest[t]; jbest = tj[t]; }
            }
            if (jbest < 0 || best == INF) {
                set_error("goat_lap_max: no augmenting path (infeasible costs)");
                return GOAT_EINVAL;
            }
            dmin = best;
            col_done[jbest] = 1;
            if (row_of[jbest] < 0) sink = jbest;
            else i = row_of[jbest];
        }
        // dual update keeps reduced costs non-negative and zero on matches
        u[f] += dmin;
        for (int r : seen_rows)
            if (r != f) u[r] += dmin - d[col_of[r]];
        for (int j = 0; j < n; ++j)
            if (col_done[j]) v[j] -= dmin - d[j];
        // augment along the predecessor chain
        int j = sink;
        while (true) {
            const int r = pred[j];
            row_of[j] = r;
            const int prev = col_of[r];
            col_of[r] = j;
            if (r == f) break;
            j = prev;
        }
    }
    for (int i = 0; i < n; ++i) perm[i] = col_of[i];
    return GOAT_OK;
}

}  // namespace goat
