// Graph-based compression with a target average block density mu (Sec. 2.2, Alg. 1).
//
// Supernodes start as the classes of rows with identical patterns.  Every supernode X, in
// ascending order of its smallest row, tries the supernodes adjacent to it in the quotient
// graph of A + A^T (fixed when its turn starts, ascending smallest row), skipping those
// merged away and merges beyond VBARMS_MAX_BLOCK rows, and keeps a merge when the average
// block density of the whole ordering -- nnz(A) over the elements of the blocks that hold
// an entry or lie on the diagonal -- stays >= mu (tested as nnz >= mu * elements in FP64).
// Blocks are ordered by their smallest row, rows ascending inside.
//
// The acceptance of every merge depends on the density left by all earlier merges, so
// the merge loop is sequential by construction; it runs on the host over the pattern.  The
// block elements are kept exactly (integers) and updated per merge from the block rows and
// block columns of the two supernodes, instead of being recounted.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

#include "factor.h"

namespace vb {

namespace {

// union of two sorted label lists with X and Z both mapped to X (result sorted, unique)
void merge_strip(const std::vector<int> &a, const std::vector<int> &b, int X, int Z, std::vector<int> &out) {
    out.clear();
    out.reserve(a.size() + b.size());
    for (int v : a) out.push_back(v == Z ? X : v);
    for (int v : b) out.push_back(v == Z ? X : v);
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
}

// replaces Z by X in a sorted label list (keeping it sorted and unique)
void relabel(std::vector<int> &v, int X, int Z) {
    auto it = std::lower_bound(v.begin(), v.end(), Z);
    if (it == v.end() || *it != Z) return;
    v.erase(it);
    auto jt = std::lower_bound(v.begin(), v.end(), X);
    if (jt == v.end() || *jt != X) v.insert(jt, X);
}

}  // namespace

std::vector<int> graph_compress_host(int n, const std::vector<int64_t> &rp, const std::vector<int> &ci, double mu,
                                     std::vector<int> &perm) {
    const int64_t nnz = rp[n];
    // identical patterns: rows sorted by (length, pattern, row); equal neighbours join the
    // class of the first, which is its smallest row
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    auto less_pattern = [&](int a, int b) {
        const int64_t la = rp[a + 1] - rp[a], lb = rp[b + 1] - rp[b];
        if (la != lb) return la < lb;
        for (int64_t k = 0; k < la; ++k) {
            const int ca = ci[rp[a] + k], cb = ci[rp[b] + k];
            if (ca != cb) return ca < cb;
        }
        return a < b;
    };
    std::sort(order.begin(), order.end(), less_pattern);
    std::vector<int> lab(n);
    for (int t = 0; t < n; ++t) {
        const int i = order[t];
        lab[i] = i;
        if (t == 0) continue;
        const int j = order[t - 1];
        const int64_t li = rp[i + 1] - rp[i], lj = rp[j + 1] - rp[j];
        if (li > 0 && li == lj && std::equal(ci.begin() + rp[i], ci.begin() + rp[i + 1], ci.begin() + rp[j]))
            lab[i] = lab[j];
    }
    std::vector<int64_t> sz(n, 0);
    for (int i = 0; i < n; ++i) sz[lab[i]]++;
    std::vector<std::vector<int>> members(n);
    for (int i = 0; i < n; ++i) members[lab[i]].push_back(i);
    // block rows (BR) and block columns (BC) of every supernode, both including the diagonal
    std::vector<std::vector<int>> br(n), bc(n);
    for (int i = 0; i < n; ++i) {
        const int I = lab[i];
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int J = lab[ci[k]];
            br[I].push_back(J);
            bc[J].push_back(I);
        }
    }
    int64_t elems = 0;
    for (int S = 0; S < n; ++S) {
        if (sz[S] == 0) continue;
        br[S].push_back(S);
        bc[S].push_back(S);
        std::sort(br[S].begin(), br[S].end());
        br[S].erase(std::unique(br[S].begin(), br[S].end()), br[S].end());
        std::sort(bc[S].begin(), bc[S].end());
        bc[S].erase(std::unique(bc[S].begin(), bc[S].end()), bc[S].end());
        for (int J : br[S]) elems += sz[S] * sz[J];
    }
    std::vector<int> first(n);
    std::iota(first.begin(), first.end(), 0);
    std::vector<int> cand, nbr, nbc;
    for (int X = 0; X < n; ++X) {
        if (sz[X] == 0 || lab[X] != X) continue;  // not a supernode, or merged away
        // quotient-graph neighbours of X when its turn starts, ascending smallest row
        cand.clear();
        std::set_union(br[X].begin(), br[X].end(), bc[X].begin(), bc[X].end(), std::back_inserter(cand));
        cand.erase(std::remove(cand.begin(), cand.end(), X), cand.end());
        std::sort(cand.begin(), cand.end(), [&](int a, int b) { return first[a] < first[b]; });
        for (int Z : cand) {
            if (sz[Z] == 0) continue;
            if (sz[X] + sz[Z] > VBARMS_MAX_BLOCK) continue;
            const int64_t sS = sz[X] + sz[Z];
            // elements of the blocks that change: the block rows of X and Z, and their block
            // columns outside X and Z
            int64_t old_el = 0, new_el = 0;
            for (int J : br[X]) old_el += sz[X] * sz[J];
            for (int J : br[Z]) old_el += sz[Z] * sz[J];
            for (int I : bc[X])
                if (I != X && I != Z) old_el += sz[I] * sz[X];
            for (int I : bc[Z])
                if (I != X && I != Z) old_el += sz[I] * sz[Z];
            merge_strip(br[X], br[Z], X, Z, nbr);
            merge_strip(bc[X], bc[Z], X, Z, nbc);
            for (int J : nbr) new_el += sS * (J == X ? sS : sz[J]);
            for (int I : nbc)
                if (I != X) new_el += sz[I] * sS;
            const int64_t el = elems - old_el + new_el;
            if (!((double)nnz >= mu * (double)el)) continue;
            // merge Z into X
            elems = el;
            for (int I : bc[Z])
                if (I != X && I != Z) relabel(br[I], X, Z);
            for (int J : br[Z])
                if (J != X && J != Z) relabel(bc[J], X, Z);
            br[X].swap(nbr);
            bc[X].swap(nbc);
            std::vector<int>().swap(br[Z]);
            std::vector<int>().swap(bc[Z]);
            for (int i : members[Z]) lab[i] = X;
            members[X].insert(members[X].end(), members[Z].begin(), members[Z].end());
            std::vector<int>().swap(members[Z]);
            sz[X] = sS;
            sz[Z] = 0;
            first[X] = std::min(first[X], first[Z]);
        }
    }
    // blocks by smallest row, rows ascending inside
    std::vector<int> sups;
    for (int S = 0; S < n; ++S)
        if (sz[S] > 0) sups.push_back(S);
    std::sort(sups.begin(), sups.end(), [&](int a, int b) { return first[a] < first[b]; });
    std::vector<int> bptr(1, 0);
    perm.clear();
    perm.reserve(n);
    for (int S : sups) {
        std::vector<int> &m = members[S];
        std::sort(m.begin(), m.end());
        perm.insert(perm.end(), m.begin(), m.end());
        bptr.push_back((int)perm.size());
    }
    return bptr;
}

}  // namespace vb
