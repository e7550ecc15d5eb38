// Host-side constant tables of the descriptor kernels.
//
// Clebsch-Gordan coefficients <j1 m1 j2 m2 | j m> are built by coupling:
// the stretched state |j1+j2, j1+j2> = |j1 j1>|j2 j2> is lowered with
// J- = J1- + J2-; each lower j starts from the vector of the M = j subspace
// orthogonal to all states of larger j (Gram-Schmidt), with the
// Condon-Shortley phase <j1 j1, j2 (j-j1) | j j> > 0, and is lowered in turn.
// This is a different route from the closed Racah sum.
//
// Table layout per descriptor triple, in its contraction orientation
// (A, B -> C) (doubled): a dense (A+1) x (C+1) block
// c[ma1*(C+1) + ma] = <a m1 b m2 | c m> with ma1 = a + m1, ma = c + m,
// m2 = m - m1 (zero where m2 is out of range).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <vector>

#include "ace.h"
#include "mala_internal.h"
#include "snap_core.h"

namespace mala {

namespace {

// coupled[J][ma][ma1] for fixed (J1, J2): coefficient of |ma1, ma2 = ma - ma1 + (J1+J2-J)/2>
struct Coupling {
    int J1, J2;
    // index (J, ma, ma1, ma2) flattened over the product basis
    std::vector<std::vector<std::vector<double>>> vec;  // [Jidx][ma] -> product-basis vector
};

inline int pidx(int J2, int a1, int a2) { return a1 * (J2 + 1) + a2; }

Coupling couple(int J1, int J2) {
    Coupling c;
    c.J1 = J1;
    c.J2 = J2;
    const int dim = (J1 + 1) * (J2 + 1);
    const int nJ = std::min(J1, J2) + 1;   // J = J1+J2, J1+J2-2, ..., |J1-J2|
    c.vec.assign(nJ, {});
    // lowering: J-|j,m> = sqrt((j+m)(j-m+1)) |j,m-1>; doubled: ma = j+m, so
    // (j+m)(j-m+1) = ma * (J - ma + 1) with J doubled.
    auto lower = [&](const std::vector<double>& v) {
        std::vector<double> out(dim, 0.0);
        for (int a1 = 0; a1 <= J1; ++a1)
            for (int a2 = 0; a2 <= J2; ++a2) {
                const double x = v[pidx(J2, a1, a2)];
                if (x == 0.0) continue;
                if (a1 >= 1) out[pidx(J2, a1 - 1, a2)] += x * sqrt((double)a1 * (J1 - a1 + 1));
                if (a2 >= 1) out[pidx(J2, a1, a2 - 1)] += x * sqrt((double)a2 * (J2 - a2 + 1));
            }
        return out;
    };
    for (int t = 0; t < nJ; ++t) {
        const int J = J1 + J2 - 2 * t;
        // top state: M = J/2, i.e. a1 + a2 = (J + J1 + J2)/2
        const int S = (J + J1 + J2) / 2;
        std::vector<double> top(dim, 0.0);
        // start from the product state with a1 = J1 (m1 = j1), orthogonalise
        top[pidx(J2, J1, S - J1)] = 1.0;
        for (int u = 0; u < t; ++u) {
            const int Ju = J1 + J2 - 2 * u;
            const std::vector<double>& w = c.vec[u][(Ju + J) / 2];   // |Ju, M = J/2>: ma = Ju/2 + J/2
            double dot = 0.0;
            for (int i = 0; i < dim; ++i) dot += w[i] * top[i];
            for (int i = 0; i < dim; ++i) top[i] -= dot * w[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < dim; ++i) nrm += top[i] * top[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < dim; ++i) top[i] /= nrm;
        if (top[pidx(J2, J1, S - J1)] < 0)
            for (int i = 0; i < dim; ++i) top[i] = -top[i];
        c.vec[t].assign(J + 1, std::vector<double>());
        c.vec[t][J] = top;
        for (int ma = J; ma >= 1; --ma) {
            std::vector<double> v = lower(c.vec[t][ma]);
            const double f = sqrt((double)ma * (J - ma + 1));
            for (int i = 0; i < dim; ++i) v[i] /= f;
            c.vec[t][ma - 1] = v;
        }
    }
    return c;
}

}  // namespace

// Returns the number of floats written, or -1 if cap is too small.  Triple t
// gets the block of its contraction orientation (A, B -> C) of zb_perm.
int build_cg_table(int twojmax, float* table, int* offsets, int cap) {
    int n = 0;
    std::vector<Coupling> cache((twojmax + 1) * (twojmax + 1));
    std::vector<bool> have(cache.size(), false);
    for (int t = 0; t < n_triples(twojmax); ++t) {
        const ZbPerm p = zb_perm(twojmax, t);
        const int A = p.a, B = p.b, C = p.c;
        const int key = A * (twojmax + 1) + B;
        if (!have[key]) {
            cache[key] = couple(A, B);
            have[key] = true;
        }
        const Coupling& c = cache[key];
        const int D = (A + B - C) / 2;       // also the index of C in the coupling's list
        offsets[t] = n;
        const int sz = (A + 1) * (C + 1);
        if (n + sz > cap) return -1;
        for (int ma1 = 0; ma1 <= A; ++ma1)
            for (int ma = 0; ma <= C; ++ma) {
                const int ma2 = ma - ma1 + D;
                double v = 0.0;
                if (ma2 >= 0 && ma2 <= B) v = c.vec[D][ma][pidx(B, ma1, ma2)];
                table[n + ma1 * (C + 1) + ma] = (float)v;
            }
        n += sz;
    }
    return n;
}

// The same blocks for every coupled pair (A, B -> C) of the descriptor
// adjoint (combo_of order).
int build_cg_table_adjoint(int twojmax, float* table, int* offsets, int cap) {
    int n = 0;
    std::vector<Coupling> cache((twojmax + 1) * (twojmax + 1));
    std::vector<bool> have(cache.size(), false);
    for (int k = 0; k < n_combos(twojmax); ++k) {
        const Combo cb = combo_of(twojmax, k);
        const int A = cb.a, B = cb.b, C = cb.c;
        const int key = A * (twojmax + 1) + B;
        if (!have[key]) {
            cache[key] = couple(A, B);
            have[key] = true;
        }
        const Coupling& c = cache[key];
        const int D = (A + B - C) / 2;
        offsets[k] = n;
        const int sz = (A + 1) * (C + 1);
        if (n + sz > cap) return -1;
        for (int ma1 = 0; ma1 <= A; ++ma1)
            for (int ma = 0; ma <= C; ++ma) {
                const int ma2 = ma - ma1 + D;
                double v = 0.0;
                if (ma2 >= 0 && ma2 <= B) v = c.vec[D][ma][pidx(B, ma1, ma2)];
                table[n + ma1 * (C + 1) + ma] = (float)v;
            }
        n += sz;
    }
    return n;
}

// Work units of the adjoint contraction: output level C (c_lo..c_hi) and
// column mb, each summing Z^C(A, B)[., mb] over the coupled pairs of C.
// Assigned to the waves of a block by longest processing time; wave_units[w*stride] = count,
// followed by the units (C * 32 + mb).
void plan_y_units(int twojmax, int c_lo, int c_hi, int n_waves, int* wave_units, int stride) {
    std::vector<std::pair<double, int>> jobs;
    for (int C = c_lo; C <= c_hi; ++C)
        for (int mb = 0; mb <= C; ++mb) {
            double cost = 0.0;
            for (int k = combo_first(twojmax, C); k < n_combos(twojmax) && combo_of(twojmax, k).c == C; ++k) {
                const Combo cb = combo_of(twojmax, k);
                const int A = cb.a, B = cb.b, D = (A + B - C) / 2, HR = C / 2;
                int t = 0;
                for (int ma = 0; ma <= HR; ++ma)
                    for (int ma1 = 0; ma1 <= A; ++ma1)
                        if (zb_pair_ok(A, B, C, ma, ma1) && (C % 2 || ma < HR || mb <= HR)) ++t;
                const int lo = mb + D - B > 0 ? mb + D - B : 0, hi = A < mb + D ? A : mb + D;
                cost += (hi - lo + 1) * (4.0 * t + zy_scale_ops(A, B, C) + 6.0) + 2.0 * t + 4.0;
            }
            jobs.push_back({cost, C * 32 + mb});
        }
    std::stable_sort(jobs.begin(), jobs.end(),
                     [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
                         return a.first > b.first;
                     });
    std::vector<double> load(n_waves, 0.0);
    std::vector<std::vector<int>> lists(n_waves);
    for (auto& jb : jobs) {
        int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[w] += jb.first;
        lists[w].push_back(jb.second);
    }
    for (int w = 0; w < n_waves; ++w) {
        wave_units[w * stride] = (int)lists[w].size();
        for (size_t i = 0; i < lists[w].size(); ++i) wave_units[w * stride + 1 + i] = lists[w][i];
    }
}

// Rank-3 grid ACE tables.  The descriptors (multisets of three (n, l)
// pairs, key p = n (lmax+1) + l, p1 <= p2 <= p3, l1+l2+l3 even and triangle,
// in that order) are grouped by (p1, p2, l3).  A group's partial sums
//   P(m3) = sum_m1 (l1 l2 l3; m1, -m1-m3, m3) A_{n1 l1 m1} A_{n2 l2 -m1-m3}
// are formed once and every descriptor of the group is
//   B = sum_m3 P(m3) A_{n3 l3 m3}.
// A is stored for m >= 0 only (A_{l,-m} = (-1)^m conj(A_{l,m})) at n*15 +
// l(l+1)/2 + |m|.  The kernel evaluates a group with code specialised for
// its (l1, l2, l3), so the 3j symbols of each such combination form one block
// of coefficients shared by all groups of that combination, in the order
// m3 = -l3..l3, m1 = -l1..l1 with |m1 + m3| <= l2 (zeros included).  Per group:
// groups[8g..8g+7] = {offset of its coefficient block, l3, first output,
// output count, l1*25 + l2*5 + l3, storage base of (n1, l1), of (n2, l2), 0};
// outputs pack the storage base n3*15 + l3(l3+1)/2 (bits 0-6) and the
// descriptor's rank-3 position (bits 7 and up).  The 3j symbol comes from the
// coupled states of couple(): (l1 l2 l3; m1 m2 m3) = (-1)^(l1-l2-m3)
// <l1 m1 l2 m2 | l3 -m3> / sqrt(2 l3 + 1).
int build_ace_tables(int nmax, int lmax, std::vector<int>& groups, std::vector<int>& groups_dm,
                     std::vector<float>& coef) {
    groups.clear();
    groups_dm.clear();
    coef.clear();
    std::vector<Coupling> cache(25 * 25);
    std::vector<bool> have(cache.size(), false);
    auto three_j = [&](int l1, int l2, int l3, int m1, int m2, int m3) {
        const int J1 = 2 * l1, J2 = 2 * l2, J = 2 * l3;
        const int key = J1 * 25 + J2;
        if (!have[key]) {
            cache[key] = couple(J1, J2);
            have[key] = true;
        }
        const Coupling& c = cache[key];
        const int D = (J1 + J2 - J) / 2;
        const int ma = l3 - m3, ma1 = l1 + m1, ma2 = l2 + m2;     // <l1 m1 l2 m2 | l3, -m3>
        const double cg = c.vec[D][ma][pidx(J2, ma1, ma2)];
        const int ph = l1 - l2 - m3;
        return ((ph % 2 + 2) % 2 ? -1.0 : 1.0) * cg / sqrt(2.0 * l3 + 1.0);
    };
    const int np = nmax * (lmax + 1);
    // rank-3 position of every descriptor, in the output order
    std::vector<int> pos_of(np * np * np, -1);
    int nd = 0;
    for (int p1 = 0; p1 < np; ++p1)
        for (int p2 = p1; p2 < np; ++p2)
            for (int p3 = p2; p3 < np; ++p3) {
                const int l1 = p1 % (lmax + 1), l2 = p2 % (lmax + 1), l3 = p3 % (lmax + 1);
                if (l3 < abs(l1 - l2) || l3 > l1 + l2 || (l1 + l2 + l3) % 2) continue;
                pos_of[(p1 * np + p2) * np + p3] = nd++;
            }
    std::vector<int> block_of(125, -1);
    struct Pair {
        std::vector<std::array<int, kAceGroupInts>> groups;
        int col0 = -1, ncol = 0;
        long cost = 0;
    };
    std::vector<Pair> pairs;
    for (int p1 = 0; p1 < np; ++p1)
        for (int p2 = p1; p2 < np; ++p2) {
            Pair pr;
            for (int l3 = 0; l3 <= lmax; ++l3) {
                const int n1 = p1 / (lmax + 1), l1 = p1 % (lmax + 1), n2 = p2 / (lmax + 1), l2 = p2 % (lmax + 1);
                if (l3 < abs(l1 - l2) || l3 > l1 + l2 || (l1 + l2 + l3) % 2) continue;
                std::vector<int> outs;
                for (int n3 = 0; n3 < nmax; ++n3) {
                    const int p3 = n3 * (lmax + 1) + l3;
                    if (p3 < p2) continue;
                    outs.push_back((n3 * 15 + l3 * (l3 + 1) / 2) | (pos_of[(p1 * np + p2) * np + p3] << 7));
                }
                if (outs.empty()) continue;
                const int combo = l1 * 25 + l2 * 5 + l3;
                int terms = 0;                   // structural terms (m3, m1) of the combination
                for (int m3 = -l3; m3 <= l3; ++m3)
                    for (int m1 = -l1; m1 <= l1; ++m1)
                        terms += abs(m1 + m3) <= l2;
                if (block_of[combo] < 0) {
                    block_of[combo] = (int)coef.size();
                    for (int m3 = -l3; m3 <= l3; ++m3)
                        for (int m1 = -l1; m1 <= l1; ++m1) {
                            const int m2 = -m1 - m3;
                            if (abs(m2) > l2) continue;
                            coef.push_back((float)three_j(l1, l2, l3, m1, m2, m3));
                        }
                }
                // header: coefficient block, l3, output count, combination, the
                // two A row bases, the outputs (one per n3 <= nmax <= 4), then
                // the pair's columns (filled below)
                std::array<int, kAceGroupInts> g{};
                g[0] = block_of[combo];
                g[1] = l3;
                g[2] = (int)outs.size();
                g[3] = combo;
                g[4] = n1 * 15 + l1 * (l1 + 1) / 2;
                g[5] = n2 * 15 + l2 * (l2 + 1) / 2;
                for (size_t i = 0; i < outs.size(); ++i) {
                    g[6 + i] = outs[i];
                    const int pos = outs[i] >> 7;
                    if (pr.col0 < 0 || pos < pr.col0) pr.col0 = pos;
                    ++pr.ncol;
                }
                pr.cost += terms + (long)outs.size() * (2 * l3 + 1);
                pr.groups.push_back(g);
            }
            if (pr.groups.empty()) continue;
            // the kernel stages a pair's outputs by column - col0: they must be
            // exactly the columns col0 .. col0 + ncol - 1
            std::vector<int> cols;
            for (const auto& g : pr.groups)
                for (int i = 0; i < g[2]; ++i) cols.push_back(g[6 + i] >> 7);
            std::sort(cols.begin(), cols.end());
            for (size_t i = 0; i < cols.size(); ++i)
                if (cols[i] != pr.col0 + (int)i) return -1;
            if (pr.ncol > kAceMaxPairCols) return -1;
            for (const auto& g : pr.groups)                     // (p1, p2, l3) order
                for (int i = 0; i < kAceGroupInts; ++i) groups_dm.push_back(g[i]);
            pairs.push_back(pr);
        }
    // whole pairs to the waves, longest first to the least loaded (LPT)
    std::vector<int> order(pairs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pairs[a].cost > pairs[b].cost; });
    std::vector<long> load(kAce3Waves, 0);
    std::vector<std::vector<int>> wave_pairs(kAce3Waves);
    for (int i : order) {
        const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[w] += pairs[i].cost;
        wave_pairs[w].push_back(i);
    }
    std::vector<std::vector<std::array<int, kAceGroupInts>>> lists(kAce3Waves);
    size_t longest = 0;
    for (int w = 0; w < kAce3Waves; ++w) {
        std::sort(wave_pairs[w].begin(), wave_pairs[w].end());
        for (int i : wave_pairs[w]) {
            const Pair& pr = pairs[i];
            for (size_t k = 0; k < pr.groups.size(); ++k) {
                std::array<int, kAceGroupInts> g = pr.groups[k];
                g[10] = pr.col0;
                g[11] = pr.ncol | ((k + 1 == pr.groups.size() ? 1 : 0) << 8);
                lists[w].push_back(g);
            }
        }
        longest = std::max(longest, lists[w].size());
    }
    std::array<int, kAceGroupInts> empty{};
    empty[3] = -1;
    for (size_t k = 0; k < longest; ++k)
        for (int w = 0; w < kAce3Waves; ++w) {
            const std::array<int, kAceGroupInts>& g = k < lists[w].size() ? lists[w][k] : empty;
            for (int i = 0; i < kAceGroupInts; ++i) groups.push_back(g[i]);
        }
    return nd;
}

// Rank-4 grid ACE (Eq. ace_grid with four factors, one intermediate
// coupling L): for keys p = n (lmax4+1) + l,
//   B(p1 p2 p3 p4; L) = sum over m of <l1 m1 l2 m2 | L M> <l3 m3 l4 m4 | L -M>
//                       (-1)^(L-M)/sqrt(2L+1) A_p1 A_p2 A_p3 A_p4.
// The set: multisets p1 <= p2 <= p3 <= p4 with an even l-sum; for each, the
// couplings L (in increasing order) whose coefficients, summed over the
// permutations that exchange equal keys, are linearly independent of those
// kept before (Gram-Schmidt on the coefficient tensors).
// Evaluation: with the coupled pairs P_a(M) = sum_m1 <l1 m1 l2 m2|L M>
// A_p1,m1 A_p2,m2 (a = (p1 p2), m2 = M - m1) and A_{l,-m} = (-1)^m conj A_{l,m},
// P_a(-M) = (-1)^(l1+l2-L+M) conj P_a(M); for an even l-sum the descriptor is
//   B = (-1)^(l3+l4-L) (-1)^L / sqrt(2L+1)
//       [Re P_a(0) conj P_b(0) + 2 sum_{M>=1} Re P_a(M) conj P_b(M)],
// so only M >= 0 of every pair is formed.  Tables per L: pair units
// (coefficient block, (l1, l2, L) combination, LDS slot of P_a(0), storage
// bases of the two keys), one Clebsch-Gordan block per combination, and
// descriptors (slot of P_a(0), slot of P_b(0), output position, factor).
namespace {

struct Ace4Cg {
    std::vector<Coupling> cache = std::vector<Coupling>(25 * 25);
    std::vector<bool> have = std::vector<bool>(25 * 25, false);
    // <l1 m1 l2 m2 | L M> from the coupled states of couple()
    double operator()(int l1, int m1, int l2, int m2, int L, int M) {
        if (m1 + m2 != M || abs(m1) > l1 || abs(m2) > l2 || abs(M) > L || L < abs(l1 - l2) || L > l1 + l2)
            return 0.0;
        const int key = 2 * l1 * 25 + 2 * l2;
        if (!have[key]) {
            cache[key] = couple(2 * l1, 2 * l2);
            have[key] = true;
        }
        return cache[key].vec[l1 + l2 - L][L + M][pidx(2 * l2, l1 + m1, l2 + m2)];
    }
};

}  // namespace

int ace4_descriptor_set(int nmax4, int lmax4, std::vector<int>& desc) {
    desc.clear();
    Ace4Cg cg;
    const int nl = lmax4 + 1, np = nmax4 * nl;
    for (int p1 = 0; p1 < np; ++p1)
        for (int p2 = p1; p2 < np; ++p2)
            for (int p3 = p2; p3 < np; ++p3)
                for (int p4 = p3; p4 < np; ++p4) {
                    const int ps[4] = {p1, p2, p3, p4};
                    const int l[4] = {p1 % nl, p2 % nl, p3 % nl, p4 % nl};
                    if ((l[0] + l[1] + l[2] + l[3]) % 2) continue;
                    const int d1 = 2 * l[1] + 1, d2 = 2 * l[2] + 1, d3 = 2 * l[3] + 1;
                    const int dim = (2 * l[0] + 1) * d1 * d2 * d3;
                    // permutations of the four slots that map every key onto an equal key
                    std::vector<std::array<int, 4>> perms;
                    std::array<int, 4> q = {0, 1, 2, 3};
                    do {
                        bool ok = true;
                        for (int i = 0; i < 4; ++i) ok = ok && ps[q[i]] == ps[i];
                        if (ok) perms.push_back(q);
                    } while (std::next_permutation(q.begin(), q.end()));
                    std::vector<std::vector<double>> kept;
                    const int Llo = std::max(abs(l[0] - l[1]), abs(l[2] - l[3]));
                    const int Lhi = std::min(l[0] + l[1], l[2] + l[3]);
                    for (int L = Llo; L <= Lhi; ++L) {
                        std::vector<double> T(dim, 0.0);
                        auto at = [&](const int (&m)[4]) {
                            return (((m[0] + l[0]) * d1 + m[1] + l[1]) * d2 + m[2] + l[2]) * d3 + m[3] + l[3];
                        };
                        for (int m1 = -l[0]; m1 <= l[0]; ++m1)
                            for (int m2 = -l[1]; m2 <= l[1]; ++m2)
                                for (int m3 = -l[2]; m3 <= l[2]; ++m3) {
                                    const int m4 = -m1 - m2 - m3, M = m1 + m2;
                                    if (abs(m4) > l[3] || abs(M) > L) continue;
                                    const double c = cg(l[0], m1, l[1], m2, L, M) * cg(l[2], m3, l[3], m4, L, -M) *
                                                     (((L - M) & 1) ? -1.0 : 1.0) / sqrt(2.0 * L + 1.0);
                                    if (c == 0.0) continue;
                                    const int m[4] = {m1, m2, m3, m4};
                                    // symmetrised: the coefficient lands on every slot order
                                    // that exchanges equal keys
                                    for (const auto& pr : perms) {
                                        int mp[4];
                                        for (int i = 0; i < 4; ++i) mp[pr[i]] = m[i];
                                        T[at(mp)] += c / (double)perms.size();
                                    }
                                }
                        double n0 = 0.0;
                        for (double x : T) n0 += x * x;
                        for (const auto& k : kept) {            // Gram-Schmidt against the kept ones
                            double dot = 0.0;
                            for (int i = 0; i < dim; ++i) dot += k[i] * T[i];
                            for (int i = 0; i < dim; ++i) T[i] -= dot * k[i];
                        }
                        double n1 = 0.0;
                        for (double x : T) n1 += x * x;
                        if (n0 > 0.0 && n1 > 1e-18 * std::max(1.0, n0)) {
                            const double inv = 1.0 / sqrt(n1);
                            for (double& x : T) x *= inv;
                            kept.push_back(T);
                            for (int i = 0; i < 4; ++i) desc.push_back(ps[i]);
                            desc.push_back(L);
                        }
                    }
                }
    return (int)(desc.size() / 5);
}

int build_ace4_tables(int nmax4, int lmax4, std::vector<int>& l_units, std::vector<int4>& units,
                      std::vector<float>& coef, std::vector<int>& l_descs, std::vector<int4>& descs,
                      int& max_slots) {
    std::vector<int> set;
    const int n4 = ace4_descriptor_set(nmax4, lmax4, set);
    Ace4Cg cg;
    const int nl = lmax4 + 1;
    l_units.assign(1, 0);
    l_descs.assign(1, 0);
    units.clear();
    coef.clear();
    descs.clear();
    max_slots = 0;
    // per L: the pairs it needs, in first-use order, each with L+1 slots,
    // and its descriptors (first pair slot, second pair slot, output, l3+l4)
    struct LPart {
        std::vector<std::pair<int, int>> pairs;
        std::vector<std::array<int, 4>> dl;
        int slots() const { return (int)pairs.size(); }
    };
    std::vector<LPart> part(2 * lmax4 + 1);
    for (int L = 0; L <= 2 * lmax4; ++L) {
        LPart& P = part[L];
        auto slot_of = [&](int pa, int pb) {
            for (size_t i = 0; i < P.pairs.size(); ++i)
                if (P.pairs[i].first == pa && P.pairs[i].second == pb) return (int)i * (L + 1);
            P.pairs.push_back({pa, pb});
            return (int)(P.pairs.size() - 1) * (L + 1);
        };
        for (int k = 0; k < n4; ++k) {
            const int* d = &set[5 * k];
            if (d[4] != L) continue;
            P.dl.push_back({slot_of(d[0], d[1]), slot_of(d[2], d[3]), k, (d[2] % nl + d[3] % nl)});
        }
    }
    // phases: several L share one pass (one pair formation, one evaluation,
    // two barriers) while their slots fit the LDS budget and their entries
    // the staged table; first fit, largest L first
    const int slot_cap = (int)(kAce4LdsBudget / (sizeof(float) * 2 * 64));
    std::vector<int> order;
    for (int L = 0; L <= 2 * lmax4; ++L)
        if (!part[L].dl.empty()) order.push_back(L);
    auto slots_of = [&](int L) { return part[L].slots() * (L + 1); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return slots_of(a) > slots_of(b); });
    std::vector<std::vector<int>> phases;
    std::vector<int> ph_slots, ph_descs;
    for (int L : order) {
        size_t i = 0;
        for (; i < phases.size(); ++i)
            if (ph_slots[i] + slots_of(L) <= slot_cap && ph_descs[i] + (int)part[L].dl.size() <= kAce4MaxDescsL)
                break;
        if (i == phases.size()) {
            phases.push_back({});
            ph_slots.push_back(0);
            ph_descs.push_back(0);
        }
        phases[i].push_back(L);
        ph_slots[i] += slots_of(L);
        ph_descs[i] += (int)part[L].dl.size();
    }
    std::vector<int> block_of(4 * 4 * 7, -1);        // (l1, l2, L) with l <= 3, L <= 6
    for (auto& ph : phases) {
        std::sort(ph.begin(), ph.end());
        std::vector<std::array<int, 5>> dl;           // slot a, slot b, output, l3+l4, L
        int base = 0;
        for (int L : ph) {
            const LPart& P = part[L];
            for (const auto& x : P.dl) dl.push_back({x[0] + base, x[1] + base, x[2], x[3], L});
            // one unit per pair: P_a(M) for M = 0..L by code specialised for
            // (l1, l2, L), with the Clebsch-Gordan coefficients of that
            // combination in one block, ordered M = 0..L, m1 = -l1..l1 with
            // |M - m1| <= l2 (zeros included)
            for (size_t i = 0; i < P.pairs.size(); ++i) {
                const int pa = P.pairs[i].first, pb = P.pairs[i].second;
                const int n1 = pa / nl, l1 = pa % nl, n2 = pb / nl, l2 = pb % nl;
                const int combo = (l1 * 4 + l2) * 7 + L;
                if (block_of[combo] < 0) {
                    block_of[combo] = (int)coef.size();
                    for (int M = 0; M <= L; ++M)
                        for (int m1 = -l1; m1 <= l1; ++m1) {
                            const int m2 = M - m1;
                            if (abs(m2) > l2) continue;
                            coef.push_back((float)cg(l1, m1, l2, m2, L, M));
                        }
                }
                const int base1 = n1 * 15 + l1 * (l1 + 1) / 2, base2 = n2 * 15 + l2 * (l2 + 1) / 2;
                units.push_back(make_int4(block_of[combo], combo, base + (int)i * (L + 1), base1 | (base2 << 8)));
            }
            base += slots_of(L);
        }
        // descriptors sharing their first pair next to each other
        std::stable_sort(dl.begin(), dl.end(), [](const std::array<int, 5>& x, const std::array<int, 5>& y) {
            return x[0] < y[0];
        });
        for (const auto& x : dl) {
            const double f = ((x[3] & 1) ? -1.0 : 1.0) / sqrt(2.0 * x[4] + 1.0);   // (-1)^(l3+l4-L) (-1)^L
            float ff = (float)f;
            int fb;
            memcpy(&fb, &ff, 4);
            descs.push_back(make_int4(x[0] | (x[4] << 16), x[1], x[2], fb));
        }
        max_slots = std::max(max_slots, base);
        l_units.push_back((int)units.size());
        l_descs.push_back((int)descs.size());
    }
    return n4;
}

// Longest-processing-time assignment of triples to the waves of a block.
// wave_triples[w*stride] = count, followed by the triple indices.
void plan_zb_waves(int twojmax, int n_waves, int* wave_triples, int stride) {
    std::vector<std::pair<double, int>> jobs;
    for (int t = 0; t < n_triples(twojmax); ++t) {
        const ZbPerm p = zb_perm(twojmax, t);
        jobs.push_back({zb_cost(p.a, p.b, p.c), t});
    }
    std::stable_sort(jobs.begin(), jobs.end(),
                     [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
                         return a.first > b.first;
                     });
    std::vector<double> load(n_waves, 0.0);
    std::vector<std::vector<int>> lists(n_waves);
    for (auto& jb : jobs) {
        int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[w] += jb.first;
        lists[w].push_back(jb.second);
    }
    for (int w = 0; w < n_waves; ++w) {
        std::sort(lists[w].begin(), lists[w].end());
        wave_triples[w * stride] = (int)lists[w].size();
        for (size_t i = 0; i < lists[w].size(); ++i) wave_triples[w * stride + 1 + i] = lists[w][i];
    }
}

}  // namespace mala
