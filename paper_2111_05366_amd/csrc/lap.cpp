// Host linear assignment for the final projection of Alg. 3 (and the
// direction step of Alg. 1): maximise sum_i M[i][perm[i]] over permutations.
//
// Shortest augmenting paths with row/column duals (the Jonker-Volgenant
// family): costs c = -M; columns are first reduced to their minimum and
// each column's argmin row is matched when still free (complementary
// slackness holds for these pairs); every remaining free row is then matched
// by one Dijkstra search over reduced costs c_ij - u_i - v_j >= 0 followed by
// a dual update and an augmentation along the found path. Among columns of
// equal tentative distance the lowest index is scanned first.
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
    auto cost = [&](int i, int j) { return -M[(size_t)i * ld + j]; };
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

    // Column reduction and free argmin matches.
    for (int j = 0; j < n; ++j) {
        int imin = 0;
        double cmin = cost(0, j);
        for (int i = 1; i < n; ++i) {
            const double c = cost(i, j);
            if (c < cmin) { cmin = c; imin = i; }
        }
        v[j] = cmin;
        if (col_of[imin] < 0) {
            col_of[imin] = j;
            row_of[j] = imin;
        }
    }

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
            int jbest = -1;
            double best = INF;
            for (int j = 0; j < n; ++j) {
                if (col_done[j]) continue;
                const double r = dmin + cost(i, j) - ui - v[j];
                if (r < d[j]) { d[j] = r; pred[j] = i; }
                if (d[j] < best) { best = d[j]; jbest = j; }
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
