// Basis and hopping-table builder (host).
//
// Basis of one spin: every sites-bit word with n bits set, in ascending order
// (Siro & Harju, Sec. 2.1: site i is bit i, states ordered by the size of the
// binary number).  The words are enumerated with Gosper's next-combination
// step, and the position of a word in that list is its combinatorial rank
//     rank(s) = sum_{k=1..n} C(p_k, k),   p_1 < p_2 < ... the set bits of s,
// which equals the ascending-order index (combinatorial number system).
//
// Hopping table of one spin (Sec. 2.1 and Sec. 4.2): for each configuration s
// and each bond {i, j} with exactly one end occupied, the hop flips both bits;
// the sign is (-1)^n with n the same-spin electrons strictly between i and j.
// Rows are packed into ELL with width = max row length, entries ascending by
// column, stored column-major (Fig. ELL); padding is column 0, sign 0.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace hub {

uint64_t binomial(int n, int k)
{
    if (k < 0 || n < 0 || k > n)
        return 0;
    static uint64_t table[65][65];
    static bool ready = false;
    if (!ready) {
        for (int a = 0; a <= 64; a++) {
            table[a][0] = 1;
            for (int b = 1; b <= a; b++)
                table[a][b] = table[a - 1][b - 1] + (b <= a - 1 ? table[a - 1][b] : 0);
        }
        ready = true;
    }
    return table[n][k];
}

static inline uint32_t next_combination(uint32_t v)
{
    // Gosper: smallest larger word with the same number of set bits
    uint32_t low = v & (0u - v);
    uint32_t ripple = v + low;
    uint32_t ones = ((v ^ ripple) >> 2) / low;
    return ripple | ones;
}

void build_spin_table(int sites, const std::vector<int32_t> &edges, int n, SpinTable &out)
{
    out = SpinTable();
    out.n = n;
    out.dim = (int64_t)binomial(sites, n);
    out.states.resize((size_t)out.dim);
    if (n == 0) {
        out.states[0] = 0;
    } else {
        uint32_t v = (n == 32) ? 0xFFFFFFFFu : ((1u << n) - 1u);
        for (int64_t r = 0; r < out.dim; r++) {
            out.states[(size_t)r] = v;
            if (r + 1 < out.dim)
                v = next_combination(v);
        }
    }

    // rank lookup through per-position binomials
    uint64_t C[33][33];
    for (int a = 0; a <= 32; a++)
        for (int b = 0; b <= 32; b++)
            C[a][b] = binomial(a, b);
    auto rank = [&](uint32_t s) -> int64_t {
        uint64_t r = 0;
        int k = 1;
        while (s) {
            int p = __builtin_ctz(s);
            r += C[p][k++];
            s &= s - 1;
        }
        return (int64_t)r;
    };

    const int ne = (int)edges.size() / 2;
    struct Entry {
        int32_t col;
        int8_t sgn;
        uint16_t bond;
    };
    std::vector<std::vector<Entry>> rows((size_t)out.dim);
    int32_t width = 0;
    int64_t nnz = 0;
    for (int64_t r = 0; r < out.dim; r++) {
        uint32_t s = out.states[(size_t)r];
        auto &row = rows[(size_t)r];
        for (int e = 0; e < ne; e++) {
            int i = edges[2 * e], j = edges[2 * e + 1];
            if (((s >> i) ^ (s >> j)) & 1u) {
                int lo = std::min(i, j), hi = std::max(i, j);
                uint32_t between = (hi - lo > 1) ? (((1u << hi) - 1u) & ~((2u << lo) - 1u)) : 0u;
                int8_t sg = (__builtin_popcount(s & between) & 1) ? -1 : 1;
                row.push_back(Entry{(int32_t)rank(s ^ ((1u << i) | (1u << j))), sg, (uint16_t)e});
            }
        }
        std::sort(row.begin(), row.end(), [](const Entry &a, const Entry &b) { return a.col < b.col; });
        width = std::max<int32_t>(width, (int32_t)row.size());
        nnz += (int64_t)row.size();
    }
    out.width = width;
    out.nnz = nnz;
    out.col.assign((size_t)width * (size_t)out.dim, 0);
    out.sgn.assign((size_t)width * (size_t)out.dim, 0);
    out.bond.assign((size_t)width * (size_t)out.dim, 0);
    out.row_nnz.resize((size_t)out.dim);
    for (int64_t r = 0; r < out.dim; r++) {
        const auto &row = rows[(size_t)r];
        out.row_nnz[(size_t)r] = (uint16_t)row.size();
        for (size_t k = 0; k < row.size(); k++) {
            out.col[k * (size_t)out.dim + (size_t)r] = row[k].col;
            out.sgn[k * (size_t)out.dim + (size_t)r] = row[k].sgn;
            out.bond[k * (size_t)out.dim + (size_t)r] = row[k].bond;
        }
    }
}

}  // namespace hub
