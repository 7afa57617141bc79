// Host planner: the balanced 2^d-tree of Sec. 2.1 and the hybrid block
// partition of Alg. 1 / eq:hybrid_admiss. Built with -ffp-contract=off so the
// box coordinates are the plain IEEE evaluation of ((p - lo) / side) * 2^L.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "hh_internal.h"

namespace hh {

// Tree depth: smallest L >= 0 with leaf_size * 2^(dL) >= n (the perfectly
// balanced relation of Sec. 2.1 read as a lower bound on L).
static int tree_depth(int64_t n, int d, int leaf_size) {
    int L = 0;
    while ((__int128)leaf_size * ((__int128)1 << (d * L)) < n) ++L;
    return L;
}

void box_coords(int64_t box, int level, int d, int64_t* c) {
    for (int k = 0; k < d; ++k) c[k] = 0;
    for (int b = 0; b < level; ++b) {
        int64_t digit = (box >> (d * (level - 1 - b))) & ((1 << d) - 1);
        for (int k = 0; k < d; ++k) c[k] = c[k] * 2 + ((digit >> (d - 1 - k)) & 1);
    }
}

static int64_t box_index(const int64_t* c, int level, int d) {
    int64_t key = 0;
    for (int b = level - 1; b >= 0; --b)
        for (int k = 0; k < d; ++k) key = key * 2 + ((c[k] >> b) & 1);
    return key;
}

// eq:H_admiss on tree boxes of equal side h: min diam = sqrt(d) h and
// dist = h sqrt(S), S = sum max(0, |c_i - c_j| - 1)^2. Exact geometric ties
// (d == eta^2 S) are admissible: the comparison carries a 2^-40 relative slack.
bool adm_s(const int64_t* ci, const int64_t* cj, int d, double eta) {
    int64_t S = 0;
    for (int k = 0; k < d; ++k) {
        int64_t g = std::llabs(ci[k] - cj[k]) - 1;
        if (g > 0) S += g * g;
    }
    return (double)d <= ((eta * eta) * (double)S) * (1.0 + 0x1p-40);
}

Plan make_plan(const double* pts, int64_t n, int d, double eta, int switch_level,
               int leaf_size) {
    if (n < 1) fail(HH_EINVAL, "n must be >= 1");
    if (d < 1 || d > 3) fail(HH_EINVAL, "d must be 1, 2 or 3");
    if (leaf_size < 1) fail(HH_EINVAL, "leaf_size must be >= 1");
    if (!(eta > 0) || !std::isfinite(eta)) fail(HH_EINVAL, "eta must be a positive finite number");
    for (int64_t i = 0; i < n * d; ++i)
        if (!std::isfinite(pts[i])) fail(HH_EINVAL, "points must be finite");
    Plan P;
    P.n = n;
    P.d = d;
    P.leaf_size = leaf_size;
    P.eta = eta;
    P.L = tree_depth(n, d, leaf_size);
    const int L = P.L;
    if ((int64_t)d * L > 30) fail(HH_ENOTSUP, "tree too deep (d * L > 30): raise leaf_size");
    if (switch_level == -1) switch_level = L > 0 ? L - 1 : 0;
    if (switch_level < 0 || switch_level > L)
        fail(HH_EINVAL, "switch_level must lie in [0, L] (L = " + std::to_string(L) + ") or be -1");
    P.ell = switch_level;

    // bounding cube: lower corner = coordinate minima, side = largest extent
    double lo[3], hi[3];
    for (int k = 0; k < d; ++k) lo[k] = hi[k] = pts[k];
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) {
            lo[k] = std::min(lo[k], pts[i * d + k]);
            hi[k] = std::max(hi[k], pts[i * d + k]);
        }
    double side = 0;
    for (int k = 0; k < d; ++k) side = std::max(side, hi[k] - lo[k]);
    if (side == 0.0) side = 1.0;
    const double cells = (double)((int64_t)1 << L);
    const int64_t top = ((int64_t)1 << L) - 1;
    std::vector<int64_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int k = 0; k < d; ++k) {
            volatile double q = (pts[i * d + k] - lo[k]) / side;
            volatile double s = q * cells;
            int64_t v = (int64_t)std::floor((double)s);
            c[k] = std::min(v, top);
        }
        key[i] = box_index(c, L, d);
    }
    P.perm.resize(n);
    std::iota(P.perm.begin(), P.perm.end(), 0);
    std::stable_sort(P.perm.begin(), P.perm.end(),
                     [&](int64_t a, int64_t b) { return key[a] < key[b]; });

    // cluster ranges per level
    P.ranges.resize(L + 1);
    for (int l = 0; l <= L; ++l) {
        int64_t nb = (int64_t)1 << (d * l);
        auto& r = P.ranges[l];
        r.assign(2 * nb, 0);
        int sh = d * (L - l);
        int64_t t = 0;
        for (int64_t b = 0; b < nb; ++b) {
            r[2 * b] = t;
            while (t < n && (key[P.perm[t]] >> sh) == b) ++t;
            r[2 * b + 1] = t;
        }
    }

    auto nonempty = [&](int l, int64_t b) { return P.ranges[l][2 * b + 1] > P.ranges[l][2 * b]; };
    auto push = [&](int l, int kind, int64_t i, int64_t j) {
        const auto& r = P.ranges[l];
        P.blocks.push_back(Blk{l, kind, i, j, r[2 * i], r[2 * i + 1], r[2 * j], r[2 * j + 1]});
    };

    // offsets (in boxes) that are not standard-admissible: a finite set, since
    // adm_s holds as soon as one |Delta_k| - 1 reaches sqrt(d) / eta.
    int R = 2 + (int)std::ceil(std::sqrt((double)d) / eta);
    std::vector<std::array<int64_t, 3>> near;
    {
        int64_t zero[3] = {0, 0, 0};
        int64_t o[3] = {0, 0, 0};
        int64_t span = 2 * R + 1, total = 1;
        for (int k = 0; k < d; ++k) total *= span;
        for (int64_t t = 0; t < total; ++t) {
            int64_t v = t;
            for (int k = 0; k < d; ++k) { o[k] = v % span - R; v /= span; }
            if (!adm_s(zero, o, d, eta)) near.push_back({o[0], o[1], o[2]});
        }
    }

    const int ell = P.ell;
    for (int l = 1; l <= L; ++l) {
        int64_t nb = (int64_t)1 << (d * l);
        int64_t side_l = (int64_t)1 << l, side_p = (int64_t)1 << (l - 1);
        for (int64_t i = 0; i < nb; ++i) {
            if (!nonempty(l, i)) continue;
            if (l <= ell) {
                // open pairs: children of the parent's inadmissible partners
                int64_t ci[3], pc[3], q[3], cj[3];
                box_coords(i, l, d, ci);
                box_coords(i >> d, l - 1, d, pc);
                for (const auto& o : near) {
                    bool inside = true;
                    for (int k = 0; k < d; ++k) {
                        q[k] = pc[k] + o[k];
                        if (q[k] < 0 || q[k] >= side_p) inside = false;
                    }
                    if (!inside) continue;
                    int64_t qb = box_index(q, l - 1, d);
                    for (int64_t ch = 0; ch < ((int64_t)1 << d); ++ch) {
                        int64_t j = (qb << d) | ch;
                        if (!nonempty(l, j)) continue;
                        box_coords(j, l, d, cj);
                        (void)side_l;
                        if (adm_s(ci, cj, d, eta)) push(l, HH_BLK_FAR, i, j);
                        else if (l == ell && j != i)
                            push(l, ell < L ? HH_BLK_NEAR : HH_BLK_DENSE_NEAR, i, j);
                    }
                }
            } else {
                int64_t first = (i >> d) << d;
                for (int64_t j = first; j < first + ((int64_t)1 << d); ++j)
                    if (j != i && nonempty(l, j)) push(l, HH_BLK_WEAK, i, j);
            }
        }
    }
    int64_t nbL = (int64_t)1 << (d * L);
    for (int64_t i = 0; i < nbL; ++i)
        if (nonempty(L, i)) push(L, HH_BLK_DIAG, i, i);
    std::sort(P.blocks.begin(), P.blocks.end(), [](const Blk& a, const Blk& b) {
        if (a.level != b.level) return a.level < b.level;
        if (a.bi != b.bi) return a.bi < b.bi;
        return a.bj < b.bj;
    });
    return P;
}

}  // namespace hh
