// Angle-based compression (Sec. 2.1) on the GPU.
//
// The sequential definition opens a group at every unassigned row i (ascending) and adds
// each later unassigned row j with cos(r_i, r_j) >= tau.  Its seeds are exactly the
// lexicographically first maximal independent set of the similarity graph, and every
// other row belongs to its smallest similar seed.  The GPU computes:
//   1. identical-pattern classes with a 64-bit pattern checksum (Ashcraft's checksum
//      idea, Eq. checksum, with an order-independent mixing function) verified by exact
//      comparison; identical rows provably share a group for any tau, so only class
//      representatives enter the cosine test (at tau = 1 the classes are the groups);
//   2. the lower similarity lists: for every representative j, the counts
//      c = |r_i & r_j| for representatives i < j reached through a shared column, held
//      in an LDS hash table, tested as c*c >= tau^2 |r_i||r_j| (exact integer-valued
//      FP64 compare, no square root);
//   3. the lexicographically first independent set by monotone parallel rounds;
//   4. groups in seed order with ascending members.
#include <algorithm>
#include <climits>

#include "common.h"

namespace vb {

namespace {

constexpr unsigned long long kEmpty = ~0ull;

__device__ inline unsigned long long mix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void k_row_key(int n, const int64_t *rowptr, const int *col, unsigned long long *key, int *len) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long h = 0;
    int64_t b = rowptr[i], e = rowptr[i + 1];
    for (int64_t k = b; k < e; ++k) h += mix64((unsigned long long)col[k] + 1ull);
    h ^= mix64((unsigned long long)(e - b) * 0x2545F4914F6CDD1Dull);
    if (h == kEmpty) h ^= 1ull;
    key[i] = h;
    len[i] = (int)(e - b);
}

__global__ void k_class_insert(int n, const unsigned long long *key, const int *len, unsigned long long *tkey,
                               int *tval, unsigned cap_mask) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || len[i] == 0) return;
    unsigned long long k = key[i];
    unsigned h = (unsigned)(mix64(k) & cap_mask);
    for (;;) {
        unsigned long long old = atomicCAS(&tkey[h], kEmpty, k);
        if (old == kEmpty || old == k) {
            atomicMin(&tval[h], i);
            return;
        }
        h = (h + 1) & cap_mask;
    }
}

__global__ void k_class_rep(int n, const int64_t *rowptr, const int *col, const unsigned long long *key,
                            const int *len, const unsigned long long *tkey, const int *tval, unsigned cap_mask,
                            int *rep, int *collision) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (len[i] == 0) { rep[i] = i; return; }
    unsigned long long k = key[i];
    unsigned h = (unsigned)(mix64(k) & cap_mask);
    while (tkey[h] != k) h = (h + 1) & cap_mask;
    int u = tval[h];
    if (u == i) { rep[i] = i; return; }
    bool same = len[u] == len[i];
    if (same) {
        const int *a = col + rowptr[i];
        const int *b = col + rowptr[u];
        for (int t = 0; t < len[i]; ++t)
            if (a[t] != b[t]) { same = false; break; }
    }
    rep[i] = same ? u : i;
    if (!same) atomicExch(collision, 1);
}

__global__ void k_flag_eq(int n, const int *a, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = a[i] == i;
}
__global__ void k_list_from_flag(int n, const int *flag, const int *idx, int *list) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) list[idx[i]] = i;
}

// column counts of the representatives' patterns
__global__ void k_rep_colcount(int nr, const int *replist, const int64_t *rowptr, const int *col, int *ccnt) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    int i = replist[r];
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) atomicAdd(&ccnt[col[k]], 1);
}
__global__ void k_rep_colfill(int nr, const int *replist, const int64_t *rowptr, const int *col,
                              const int64_t *cptr, int *cfill, int *crow) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    int i = replist[r];
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        int c = col[k];
        crow[cptr[c] + atomicAdd(&cfill[c], 1)] = r;  // representative index
    }
}

// Upper bound on the candidates of representative r (with repetitions).
__global__ void k_sim_bound(int nr, const int *replist, const int64_t *rowptr, const int *col, const int64_t *cptr,
                            int64_t *bound) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    int i = replist[r];
    int64_t s = 0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s += cptr[col[k] + 1] - cptr[col[k]];
    bound[r] = s;
}

constexpr int kSimThreads = 256;
constexpr int kSimCap = 4096;  // LDS table; a row with more than kSimCap/2 candidates moves to global memory

// Counts |r_i & r_j| for every representative i < j sharing a column with j, then tests the
// cosine.  pass 0 counts similar pairs, pass 1 writes them.  At most `limit` distinct
// candidates are inserted (limit + blockDim.x < cap keeps an empty slot for every probe);
// beyond that *full is set and the caller discards the row.
__device__ void sim_row(int r, const int *replist, const int64_t *rowptr, const int *col, const int *len,
                        const int64_t *cptr, const int *crow, double tau2, int *tkeys, int *tcnt, int cap, int limit,
                        int pass, int *ecnt, const int64_t *eptr, int *elist, int *wcount, int *distinct,
                        int *full) {
    const int t = threadIdx.x;
    for (int h = t; h < cap; h += blockDim.x) { tkeys[h] = -1; tcnt[h] = 0; }
    if (t == 0) { *wcount = 0; *distinct = 0; *full = 0; }
    __syncthreads();
    const int j = replist[r];
    const int64_t b = rowptr[j], e = rowptr[j + 1];
    const unsigned mask = (unsigned)cap - 1u;
    // one wavefront per column, lanes over the representatives holding that column
    const int wave = t >> 6, lane = t & 63, nwave = blockDim.x >> 6;
    for (int64_t k = b + wave; k < e; k += nwave) {
        int c = col[k];
        for (int64_t q = cptr[c] + lane; q < cptr[c + 1]; q += 64) {
            int i = crow[q];
            if (i >= r) continue;
            if (__atomic_load_n(full, __ATOMIC_RELAXED)) break;
            unsigned h = ((unsigned)i * 2654435761u) & mask;
            for (;;) {
                int old = atomicCAS(&tkeys[h], -1, i);
                if (old == -1 || old == i) {
                    atomicAdd(&tcnt[h], 1);
                    if (old == -1 && atomicAdd(distinct, 1) + 1 >= limit) atomicExch(full, 1);
                    break;
                }
                h = (h + 1) & mask;
            }
        }
    }
    __syncthreads();
    if (*full) return;
    const double lj = (double)len[j];
    for (int h = t; h < cap; h += blockDim.x) {
        int i = tkeys[h];
        if (i < 0) continue;
        double c = (double)tcnt[h];
        double lhs = c * c;
        double rhs = tau2 * ((double)len[replist[i]] * lj);
        if (lhs >= rhs) {
            int slot = atomicAdd(wcount, 1);
            if (pass == 1) elist[eptr[r] + slot] = i;
        }
    }
    __syncthreads();
    if (pass == 0 && t == 0) ecnt[r] = *wcount;
}

// pass 0 marks rows that do not fit the LDS table in big[]; pass 1 skips them
__global__ void __launch_bounds__(kSimThreads) k_sim_lds(int nr, const int *replist, const int64_t *rowptr,
                                                         const int *col, const int *len, const int64_t *cptr,
                                                         const int *crow, double tau2, int pass, int *ecnt,
                                                         const int64_t *eptr, int *elist, int *big) {
    __shared__ int tkeys[kSimCap];
    __shared__ int tcnt[kSimCap];
    __shared__ int wcount, distinct, full;
    int r = blockIdx.x;
    if (r >= nr) return;
    if (pass == 1 && big[r]) return;
    sim_row(r, replist, rowptr, col, len, cptr, crow, tau2, tkeys, tcnt, kSimCap, kSimCap / 2, pass, ecnt, eptr,
            elist, &wcount, &distinct, &full);
    if (pass == 0 && threadIdx.x == 0) big[r] = full;
}

// rows that overflowed the LDS table: per-workgroup tables in global memory, sized from the
// candidate bound so they never overflow
__global__ void __launch_bounds__(kSimThreads) k_sim_global(int nbig, const int *biglist, const int *replist,
                                                            const int64_t *rowptr, const int *col, const int *len,
                                                            const int64_t *cptr, const int *crow, double tau2, int pass,
                                                            int *ecnt, const int64_t *eptr, int *elist, int *gkeys,
                                                            int *gcnt, int cap) {
    __shared__ int wcount, distinct, full;
    int slot = blockIdx.x;
    int *tk = gkeys + (int64_t)slot * cap;
    int *tc = gcnt + (int64_t)slot * cap;
    for (int q = slot; q < nbig; q += gridDim.x) {
        sim_row(biglist[q], replist, rowptr, col, len, cptr, crow, tau2, tk, tc, cap, cap / 2, pass, ecnt, eptr, elist,
                &wcount, &distinct, &full);
        __syncthreads();
    }
}

// Lexicographically first independent set by rounds (state 1 in, 2 out).  Decisions are
// monotone, so a state read while another thread writes it only speeds convergence.
// visits_before: true when u comes before v in the visiting order: ascending index, or with
// weights, descending weight and ascending index among equal weights
__device__ inline bool visits_before(int u, int v, const double *prio) {
    if (!prio) return u < v;
    const double wu = prio[u], wv = prio[v];
    return wu > wv || (wu == wv && u < v);
}

// Neighbours of v visited before v (from one or two adjacency lists, duplicates kept),
// counted (pass 0) and listed (pass 1); the rounds then read only these.
__global__ void k_lfmis_before(int nv, const int64_t *eptr, const int *elist, const int64_t *eptr2, const int *elist2,
                               const double *prio, const int64_t *bptr, int *bcnt, int *blist) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    int c = 0;
    int64_t o = bptr ? bptr[v] : 0;
    for (int pass = 0; pass < 2; ++pass) {
        const int64_t *ep = pass == 0 ? eptr : eptr2;
        const int *el = pass == 0 ? elist : elist2;
        if (!el) continue;
        for (int64_t e = ep[v]; e < ep[v + 1]; ++e) {
            const int u = el[e];
            if (u == v || !visits_before(u, v, prio)) continue;
            if (blist) blist[o + c] = u;
            ++c;
        }
    }
    if (!blist) bcnt[v] = c;
}

// One round over the vertices of `list` (count nl): a vertex enters when all its earlier
// neighbours are out and leaves when one of them is in.  The states of eight neighbours are
// loaded before any is examined, so a round costs a few dependent loads per vertex.
__global__ void k_lfmis_round(int nl, const int *list, const int64_t *bptr, const int *blist, int *state) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nl) return;
    const int v = list[q];
    if (__atomic_load_n(&state[v], __ATOMIC_RELAXED) != 0) return;
    bool any_in = false, all_out = true;
    const int64_t e1 = bptr[v + 1];
    for (int64_t e0 = bptr[v]; e0 < e1 && !any_in; e0 += 8) {
        int st[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) st[u] = e0 + u < e1 ? blist[e0 + u] : -1;
#pragma unroll
        for (int u = 0; u < 8; ++u) st[u] = st[u] >= 0 ? __atomic_load_n(&state[st[u]], __ATOMIC_RELAXED) : 2;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            any_in = any_in || st[u] == 1;
            all_out = all_out && st[u] == 2;
        }
    }
    if (any_in) __atomic_store_n(&state[v], 2, __ATOMIC_RELAXED);
    else if (all_out) __atomic_store_n(&state[v], 1, __ATOMIC_RELAXED);
}

__global__ void k_assign_rep(int nr, const int *replist, const int64_t *eptr, const int *elist, const int *state,
                             int *seedrep) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    if (state[r] == 1) { seedrep[r] = replist[r]; return; }
    int best = INT_MAX;
    for (int64_t e = eptr[r]; e < eptr[r + 1]; ++e) {
        int u = elist[e];
        if (state[u] == 1 && u < best) best = u;
    }
    seedrep[r] = replist[best];
}
__global__ void k_assign_row(int n, const int *rep, const int *repidx, const int *seedrep, int *seed) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) seed[i] = seedrep[repidx[rep[i]]];
}

__global__ void k_group_size(int n, const int *seed, const int *sidx, int *gsize) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&gsize[sidx[seed[i]]], 1);
}
__global__ void k_group_scatter(int n, const int *seed, const int *sidx, const int *bptr, int *cursor, int *perm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = sidx[seed[i]];
    perm[bptr[b] + atomicAdd(&cursor[b], 1)] = i;
}
__global__ void k_group_sort(int p, const int *bptr, int *perm) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p) return;
    int lo = bptr[b], hi = bptr[b + 1];
    for (int x = lo + 1; x < hi; ++x) {
        int v = perm[x];
        int y = x - 1;
        while (y >= lo && perm[y] > v) { perm[y + 1] = perm[y]; --y; }
        perm[y + 1] = v;
    }
}

// undecided vertices of list_in appended to list_out (one atomic per wavefront)
__global__ void k_lfmis_compact(int nl, const int *list_in, const int *state, int *list_out, int *cnt_out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = q < nl ? list_in[q] : -1;
    const bool keep = v >= 0 && state[v] == 0;
    const int lane = threadIdx.x & 63;
    const unsigned long long mask = __ballot(keep);
    const int tot = __popcll(mask);
    int base = 0;
    if (tot > 0) {
        const int leader = __ffsll((long long)mask) - 1;
        if (lane == leader) base = atomicAdd(cnt_out, tot);
        base = __shfl(base, leader, 64);
    }
    if (keep) list_out[base + __popcll(mask & ((1ull << lane) - 1ull))] = v;
}

}  // namespace

// Lexicographically first MIS by rounds; shared with the independent-set step.  Every
// round visits only the vertices that were undecided at the last compaction (every
// `batch` rounds): a decision never changes, so skipping decided vertices changes nothing.
void lfmis(int nv, const int64_t *eptr, const int *elist, const int64_t *eptr2, const int *elist2, const double *prio,
           int *state, hipStream_t s) {
    fill_i32(state, 0, nv, s);
    if (nv == 0) return;
    // each vertex's earlier-visited neighbours, listed once
    DBuf<int> bcnt(nv);
    DBuf<int64_t> bptr(nv + 1);
    k_lfmis_before<<<grid_for(nv, 256), 256, 0, s>>>(nv, eptr, elist, eptr2, elist2, prio, nullptr, bcnt.p, nullptr);
    VB_LAUNCH_CHECK();
    const int64_t nb = scan_i32_to_i64(bcnt.p, bptr.p, nv, s);
    DBuf<int> blist(std::max<int64_t>(nb, 1));
    k_lfmis_before<<<grid_for(nv, 256), 256, 0, s>>>(nv, eptr, elist, eptr2, elist2, prio, bptr.p, nullptr, blist.p);
    VB_LAUNCH_CHECK();
    DBuf<int> lists(2 * (size_t)nv), cnt(2);
    iota_i32(lists.p, nv, s);
    int nl = nv, cur = 0;
    const int batch = 8;
    for (int round = 0;; round += batch) {
        const int *lin = lists.p + (size_t)cur * nv;
        for (int b = 0; b < batch; ++b) {
            k_lfmis_round<<<grid_for(nl, 256), 256, 0, s>>>(nl, lin, bptr.p, blist.p, state);
            VB_LAUNCH_CHECK();
        }
        int *lout = lists.p + (size_t)(1 - cur) * nv;
        fill_i32(cnt.p, 0, 1, s);
        k_lfmis_compact<<<grid_for(nl, 256), 256, 0, s>>>(nl, lin, state, lout, cnt.p);
        VB_LAUNCH_CHECK();
        nl = read_one(cnt.p, s);
        if (nl == 0) break;
        cur = 1 - cur;
        if (round > 4 * nv + 64) fail(VBARMS_ERR_HIP, "independent-set rounds did not converge");
    }
}

namespace {

// seed[i] = representative row of i's identical-pattern class; returns true on a checksum
// collision between different patterns (the classes are then incomplete, which only
// costs speed: the cosine test below still groups identical rows together)
bool pattern_classes(int n, const int64_t *rowptr, const int *col, int *len, int *rep, hipStream_t s) {
    DBuf<unsigned long long> key(n);
    k_row_key<<<grid_for(n, 256), 256, 0, s>>>(n, rowptr, col, key.p, len);
    VB_LAUNCH_CHECK();
    unsigned cap = 1024;
    while (cap < 2u * (unsigned)n) cap <<= 1;
    DBuf<unsigned long long> tkey(cap);
    DBuf<int> tval(cap), coll(1);
    fill_val<unsigned long long>(tkey.p, kEmpty, cap, s);
    fill_i32(tval.p, INT_MAX, cap, s);
    fill_i32(coll.p, 0, 1, s);
    k_class_insert<<<grid_for(n, 256), 256, 0, s>>>(n, key.p, len, tkey.p, tval.p, cap - 1);
    VB_LAUNCH_CHECK();
    k_class_rep<<<grid_for(n, 256), 256, 0, s>>>(n, rowptr, col, key.p, len, tkey.p, tval.p, cap - 1, rep, coll.p);
    VB_LAUNCH_CHECK();
    return read_one(coll.p, s) != 0;
}

// lower similarity lists between representatives, then the first independent set and the
// assignment of every row to its smallest similar seed
void similarity_groups(int n, const int64_t *rowptr, const int *col, const int *len, const int *rep, double tau,
                       int *seed, hipStream_t s) {
    DBuf<int> flag(n), repidx(n + 1);
    k_flag_eq<<<grid_for(n, 256), 256, 0, s>>>(n, rep, flag.p);
    VB_LAUNCH_CHECK();
    int nr = scan_i32(flag.p, repidx.p, n, s);
    DBuf<int> replist(std::max(nr, 1));
    k_list_from_flag<<<grid_for(n, 256), 256, 0, s>>>(n, flag.p, repidx.p, replist.p);
    VB_LAUNCH_CHECK();
    // pattern transpose restricted to representatives
    DBuf<int> ccnt(n), cfill(n);
    DBuf<int64_t> cptr(n + 1);
    fill_i32(ccnt.p, 0, n, s);
    fill_i32(cfill.p, 0, n, s);
    k_rep_colcount<<<grid_for(nr, 256), 256, 0, s>>>(nr, replist.p, rowptr, col, ccnt.p);
    VB_LAUNCH_CHECK();
    int64_t nnzr = scan_i32_to_i64(ccnt.p, cptr.p, n, s);
    DBuf<int> crow(std::max<int64_t>(nnzr, 1));
    k_rep_colfill<<<grid_for(nr, 256), 256, 0, s>>>(nr, replist.p, rowptr, col, cptr.p, cfill.p, crow.p);
    VB_LAUNCH_CHECK();
    // similarity counts in LDS; rows that overflow move to global-memory tables
    DBuf<int64_t> eptr(nr + 1);
    DBuf<int> ecnt(std::max(nr, 1)), big(std::max(nr, 1)), bigidx(nr + 1);
    const double tau2 = tau * tau;
    DBuf<int> elist;
    k_sim_lds<<<nr, kSimThreads, 0, s>>>(nr, replist.p, rowptr, col, len, cptr.p, crow.p, tau2, 0, ecnt.p, eptr.p,
                                         elist.p, big.p);
    VB_LAUNCH_CHECK();
    int nbig = scan_i32(big.p, bigidx.p, nr, s);
    DBuf<int> biglist(std::max(nbig, 1));
    int gcap = 1, gslots = 1;
    DBuf<int> gkeys, gcnt;
    if (nbig > 0) {
        k_list_from_flag<<<grid_for(nr, 256), 256, 0, s>>>(nr, big.p, bigidx.p, biglist.p);
        VB_LAUNCH_CHECK();
        DBuf<int64_t> bound(std::max(nr, 1));
        k_sim_bound<<<grid_for(nr, 256), 256, 0, s>>>(nr, replist.p, rowptr, col, cptr.p, bound.p);
        VB_LAUNCH_CHECK();
        std::vector<int64_t> hb;
        std::vector<int> hbig;
        to_host(hb, bound.p, nr, s);
        to_host(hbig, big.p, nr, s);
        int64_t mb = 0;
        for (int r = 0; r < nr; ++r)
            if (hbig[r]) mb = std::max(mb, hb[r]);
        while (gcap < 2 * mb + 2 * kSimThreads) gcap <<= 1;
        gslots = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(nbig, 1024), (int64_t(1) << 27) / gcap));
        gkeys.alloc((size_t)gslots * gcap);
        gcnt.alloc((size_t)gslots * gcap);
        k_sim_global<<<gslots, kSimThreads, 0, s>>>(nbig, biglist.p, replist.p, rowptr, col, len, cptr.p, crow.p, tau2,
                                                    0, ecnt.p, eptr.p, elist.p, gkeys.p, gcnt.p, gcap);
        VB_LAUNCH_CHECK();
    }
    int64_t ne = scan_i32_to_i64(ecnt.p, eptr.p, nr, s);
    elist.alloc(std::max<int64_t>(ne, 1));
    k_sim_lds<<<nr, kSimThreads, 0, s>>>(nr, replist.p, rowptr, col, len, cptr.p, crow.p, tau2, 1, ecnt.p, eptr.p,
                                         elist.p, big.p);
    VB_LAUNCH_CHECK();
    if (nbig > 0) {
        k_sim_global<<<gslots, kSimThreads, 0, s>>>(nbig, biglist.p, replist.p, rowptr, col, len, cptr.p, crow.p, tau2,
                                                    1, ecnt.p, eptr.p, elist.p, gkeys.p, gcnt.p, gcap);
        VB_LAUNCH_CHECK();
    }
    DBuf<int> state(std::max(nr, 1)), seedrep(std::max(nr, 1));
    lfmis(nr, eptr.p, elist.p, nullptr, nullptr, nullptr, state.p, s);
    k_assign_rep<<<grid_for(nr, 256), 256, 0, s>>>(nr, replist.p, eptr.p, elist.p, state.p, seedrep.p);
    VB_LAUNCH_CHECK();
    k_assign_row<<<grid_for(n, 256), 256, 0, s>>>(n, rep, repidx.p, seedrep.p, seed);
    VB_LAUNCH_CHECK();
    VB_HIP(hipStreamSynchronize(s));
}

// groups in seed order, members ascending; returns bptr on the host
std::vector<int> make_groups(int n, const int *seed, int *perm, hipStream_t s) {
    DBuf<int> flag(n), sidx(n + 1);
    k_flag_eq<<<grid_for(n, 256), 256, 0, s>>>(n, seed, flag.p);
    VB_LAUNCH_CHECK();
    int p = scan_i32(flag.p, sidx.p, n, s);
    DBuf<int> gsize(p), bptr(p + 1), cursor(p);
    fill_i32(gsize.p, 0, p, s);
    fill_i32(cursor.p, 0, p, s);
    k_group_size<<<grid_for(n, 256), 256, 0, s>>>(n, seed, sidx.p, gsize.p);
    VB_LAUNCH_CHECK();
    scan_i32(gsize.p, bptr.p, p, s, false);
    k_group_scatter<<<grid_for(n, 256), 256, 0, s>>>(n, seed, sidx.p, bptr.p, cursor.p, perm);
    VB_LAUNCH_CHECK();
    k_group_sort<<<grid_for(p, 256), 256, 0, s>>>(p, bptr.p, perm);
    VB_LAUNCH_CHECK();
    std::vector<int> bptr_h;
    to_host(bptr_h, bptr.p, p + 1, s);
    return bptr_h;
}

}  // namespace

// perm (device, n) receives new position -> original row; returns bptr on the host.
std::vector<int> compress_gpu(int n, const int64_t *rowptr, const int *col, double tau, int *perm, hipStream_t s) {
    if (n == 0) return std::vector<int>{0};
    DBuf<int> len(n), rep(n), seed(n);
    bool collision = pattern_classes(n, rowptr, col, len.p, rep.p, s);
    if (tau >= 1.0 && !collision) {
        // identical patterns are exactly the groups at tau = 1
        VB_HIP(hipMemcpyAsync(seed.p, rep.p, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    } else {
        similarity_groups(n, rowptr, col, len.p, rep.p, tau, seed.p, s);
    }
    return make_groups(n, seed.p, perm, s);
}

}  // namespace vb
