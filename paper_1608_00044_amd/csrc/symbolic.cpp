// Host symbolic analysis (see symbolic.hpp).
//
// Algorithms: Liu's path-compressed elimination-tree construction; a
// depth-first postorder; column counts from row subtrees with the skeleton
// leaf test and least common ancestors found by a disjoint-set forest; the
// supernodal row structure built by merging each supernode's own entries of C
// with the row lists of its child supernodes.  None of this is shared with the
// CPU oracle, which builds the structure by its set definition.
#include "symbolic.hpp"

#include <algorithm>
#include <cstring>
#include <functional>
#include <new>
#include <numeric>
#include <system_error>
#include <thread>

namespace spc {

int32_t validate_input(int64_t n, const int64_t* colptr, const int32_t* rowind,
                       const int32_t* perm) {
    if (n < 0 || n > INT32_MAX - 1) return ERR_ARG;
    if (n == 0) return OK;
    if (!colptr) return ERR_ARG;
    if (colptr[0] != 0) return ERR_PATTERN;
    if (colptr[n] > 0 && !rowind) return ERR_ARG;
    for (int64_t j = 0; j < n; ++j) {
        int64_t a = colptr[j], b = colptr[j + 1];
        if (b < a) return ERR_PATTERN;
        int64_t prev = -1;
        for (int64_t p = a; p < b; ++p) {
            int64_t i = rowind[p];
            if (i < j || i >= n || i <= prev) return ERR_PATTERN;
            prev = i;
        }
    }
    if (perm) {
        std::vector<uint8_t> hit((size_t)n, 0);
        for (int64_t k = 0; k < n; ++k) {
            int32_t v = perm[k];
            if (v < 0 || v >= n || hit[v]) return ERR_ARG;
            hit[v] = 1;
        }
    }
    return OK;
}

namespace {

// C = lower(P A P^T): entry (i, j) of A moves to (max(pinv i, pinv j), min(...)).
void permute_lower(Symbolic& S, const int64_t* colptr, const int32_t* rowind) {
    const int64_t n = S.n, nnz = S.nnz_a;
    std::vector<int32_t> pinv((size_t)n);
    for (int64_t k = 0; k < n; ++k) pinv[S.perm[k]] = (int32_t)k;
    S.Cp.assign((size_t)n + 1, 0);
    std::vector<int32_t> newr((size_t)nnz), newc((size_t)nnz);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            int32_t a = pinv[rowind[p]], b = pinv[j];
            newr[p] = std::max(a, b);
            newc[p] = std::min(a, b);
            S.Cp[newc[p] + 1]++;
        }
    for (int64_t j = 0; j < n; ++j) S.Cp[j + 1] += S.Cp[j];
    std::vector<int64_t> src((size_t)nnz);
    std::vector<int64_t> next(S.Cp.begin(), S.Cp.end() - 1);
    for (int64_t p = 0; p < nnz; ++p) src[next[newc[p]]++] = p;
    S.Ci.resize((size_t)nnz);
    S.amap.resize((size_t)nnz);
    for (int64_t j = 0; j < n; ++j) {
        auto b = src.begin() + S.Cp[j], e = src.begin() + S.Cp[j + 1];
        std::sort(b, e, [&](int64_t x, int64_t y) { return newr[x] < newr[y]; });
        for (int64_t q = S.Cp[j]; q < S.Cp[j + 1]; ++q) {
            S.Ci[q] = newr[src[q]];
            S.amap[src[q]] = q;
        }
    }
}

// Elimination tree (Section II-B): parent(j) is the first off-diagonal row of
// column j of L.  Liu's algorithm: for each row i, follow every k < i with
// C_ik != 0 up its path-compressed ancestor chain; the chain's top, if not yet
// attached, becomes a child of i.
void etree(Symbolic& S, const std::vector<int64_t>& Rp, const std::vector<int32_t>& Rj) {
    const int64_t n = S.n;
    S.parent.assign((size_t)n, -1);
    std::vector<int32_t> anc((size_t)n, -1);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = Rp[i]; p < Rp[i + 1]; ++p) {
            int32_t r = Rj[p];
            while (r != -1 && r < i) {
                int32_t up = anc[r];
                anc[r] = (int32_t)i;
                if (up == -1) S.parent[r] = (int32_t)i;
                r = up;
            }
        }
    }
}

void postorder(Symbolic& S) {
    const int64_t n = S.n;
    std::vector<int32_t> head((size_t)n, -1), nxt((size_t)n, -1);
    for (int64_t j = n - 1; j >= 0; --j) {  // children lists in increasing order
        int32_t p = S.parent[j];
        if (p != -1) { nxt[j] = head[p]; head[p] = (int32_t)j; }
    }
    S.post.clear();
    S.post.reserve((size_t)n);
    std::vector<int32_t> stack;
    for (int64_t r = 0; r < n; ++r) {
        if (S.parent[r] != -1) continue;
        stack.push_back((int32_t)r);
        while (!stack.empty()) {
            int32_t v = stack.back();
            if (head[v] != -1) {
                int32_t c = head[v];
                head[v] = nxt[c];
                stack.push_back(c);
            } else {
                stack.pop_back();
                S.post.push_back(v);
            }
        }
    }
}

// Column counts: colcount(j) = number of rows i whose row subtree contains j.
// Each row subtree is the union of the etree paths from its leaves up to i;
// with the leaves taken in postorder, +1 at every leaf and -1 at the least
// common ancestor of consecutive leaves (and -1 above i) sum, over the subtree
// of any node, to the indicator of membership.  A neighbour j of row i is a
// leaf iff no earlier neighbour lies in j's subtree, i.e. iff first(j) is past
// the postorder index of the previous neighbour.
void column_counts(Symbolic& S) {
    const int64_t n = S.n;
    std::vector<int32_t> first((size_t)n, -1), pidx((size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        int32_t v = S.post[k];
        pidx[v] = (int32_t)k;
        while (v != -1 && first[v] == -1) { first[v] = (int32_t)k; v = S.parent[v]; }
    }
    std::vector<int64_t> delta((size_t)n, 0);
    std::vector<int32_t> prevnbr((size_t)n, -1), prevleaf((size_t)n, -1), dsu((size_t)n);
    std::iota(dsu.begin(), dsu.end(), 0);
    auto find = [&](int32_t x) {
        int32_t r = x;
        while (dsu[r] != r) r = dsu[r];
        while (dsu[x] != r) { int32_t t = dsu[x]; dsu[x] = r; x = t; }
        return r;
    };
    for (int64_t k = 0; k < n; ++k) {
        int32_t j = S.post[k];
        for (int64_t p = S.Cp[j]; p < S.Cp[j + 1]; ++p) {
            int32_t i = S.Ci[p];
            if (i == j) continue;
            if (first[j] > prevnbr[i]) {
                delta[j] += 1;
                if (prevleaf[i] != -1) delta[find(prevleaf[i])] -= 1;
                prevleaf[i] = j;
            }
            prevnbr[i] = (int32_t)k;
        }
        if (S.parent[j] != -1) dsu[j] = S.parent[j];
    }
    for (int64_t i = 0; i < n; ++i) {
        if (prevleaf[i] == -1) delta[i] += 1;  // row subtree is {i} alone
        if (S.parent[i] != -1) delta[S.parent[i]] -= 1;
    }
    for (int64_t k = 0; k < n; ++k) {
        int32_t j = S.post[k];
        if (S.parent[j] != -1) delta[S.parent[j]] += delta[j];
    }
    S.colcount.resize((size_t)n);
    S.nnz_l = 0;
    S.flops = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        S.colcount[j] = (int32_t)delta[j];
        S.nnz_l += delta[j];
        S.flops += (double)delta[j] * (double)delta[j];
    }
}

// Supernodes (Section II-B), non-fundamental form: column j+1 joins column
// j's supernode iff parent(j) = j+1 and colcount(j) = colcount(j+1) + 1.  Runs
// wider than the cap (Section III-B) become ceil(w / cap) near-equal pieces,
// earlier pieces one column wider when w does not divide evenly.
void partition(Symbolic& S) {
    const int64_t n = S.n;
    const int32_t cap = S.opt.sn_cap;
    S.sn_ptr.clear();
    int64_t j = 0;
    while (j < n) {
        int64_t e = j + 1;
        while (e < n && S.parent[e - 1] == e && S.colcount[e - 1] == S.colcount[e] + 1) ++e;
        const int64_t w = e - j, pieces = (w + cap - 1) / cap;
        const int64_t q = w / pieces, rem = w % pieces;
        int64_t c = j;
        for (int64_t t = 0; t < pieces; ++t) {
            S.sn_ptr.push_back((int32_t)c);
            c += q + (t < rem);
        }
        j = e;
    }
    S.sn_ptr.push_back((int32_t)n);
}

// Relaxed amalgamation.  A supernode may be folded into its supernodal parent
// when the parent begins at the next column, the union stays within the cap,
// and the explicit zeros z of the union (stored minus exact entries over its
// columns) satisfy z <= ratio * T, T being its stored entries; a folded column
// j stores (last(parent) - j + 1) + r_parent entries.  Passes over the
// supernodes in increasing column order repeat until one folds nothing.
void amalgamate(Symbolic& S) {
    const double ratio = S.opt.amalg_ratio;
    const int64_t ns = (int64_t)S.sn_ptr.size() - 1;
    if (ratio <= 0.0 || ns <= 1) return;
    const int64_t n = S.n;
    struct Node { int32_t lo, hi; int64_t zeros, total; bool live; };
    std::vector<Node> nd((size_t)ns);
    std::vector<int32_t> own((size_t)n);
    const auto& cc = S.colcount;
    for (int64_t s = 0; s < ns; ++s) {
        Node& x = nd[s];
        x.lo = S.sn_ptr[s];
        x.hi = S.sn_ptr[s + 1] - 1;
        x.live = true;
        x.zeros = x.total = 0;
        const int64_t r = cc[x.hi] - 1;
        for (int32_t c = x.lo; c <= x.hi; ++c) {
            const int64_t st = (int64_t)(x.hi - c + 1) + r;
            x.zeros += st - cc[c];
            x.total += st;
            own[c] = (int32_t)s;
        }
    }
    for (bool changed = true; changed;) {
        changed = false;
        for (int64_t s = 0; s < ns; ++s) {
            Node& a = nd[s];
            if (!a.live) continue;
            const int32_t pcol = S.parent[a.hi];
            if (pcol < 0) continue;
            Node& b = nd[own[pcol]];
            if (b.lo != a.hi + 1) continue;
            if ((int64_t)(a.hi - a.lo + 1) + (b.hi - b.lo + 1) > S.opt.sn_cap) continue;
            const int64_t rb = cc[b.hi] - 1;
            int64_t z = b.zeros, T = b.total;
            for (int32_t c = a.lo; c <= a.hi; ++c) {
                const int64_t st = (int64_t)(b.hi - c + 1) + rb;
                z += st - cc[c];
                T += st;
            }
            if (!((double)z <= ratio * (double)T)) continue;
            const int32_t bidx = own[pcol];
            for (int32_t c = a.lo; c <= a.hi; ++c) own[c] = bidx;
            b.lo = a.lo;
            b.zeros = z;
            b.total = T;
            a.live = false;
            changed = true;
        }
    }
    std::vector<int32_t> np;
    for (int64_t s = 0; s < ns; ++s)
        if (nd[s].live) np.push_back(nd[s].lo);
    np.push_back((int32_t)n);
    S.sn_ptr.swap(np);
}

int32_t structures(Symbolic& S) {
    const int64_t n = S.n, ns = (int64_t)S.sn_ptr.size() - 1;
    S.nsup = ns;
    S.col_owner.resize((size_t)n);
    for (int64_t s = 0; s < ns; ++s)
        for (int32_t c = S.sn_ptr[s]; c < S.sn_ptr[s + 1]; ++c) S.col_owner[c] = (int32_t)s;
    S.sn_parent.assign((size_t)ns, -1);
    for (int64_t s = 0; s < ns; ++s) {
        int32_t pc = S.parent[S.sn_ptr[s + 1] - 1];
        S.sn_parent[s] = pc < 0 ? -1 : S.col_owner[pc];
    }
    std::vector<int32_t> chead((size_t)ns, -1), cnext((size_t)ns, -1);
    for (int64_t s = ns - 1; s >= 0; --s) {
        int32_t p = S.sn_parent[s];
        if (p >= 0) { cnext[s] = chead[p]; chead[p] = (int32_t)s; }
    }
    // rows of each supernode: own columns, then the merged rows below
    S.rowptr.assign((size_t)ns + 1, 0);
    S.rows.clear();
    std::vector<int32_t> mark((size_t)n, -1), below;
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t lo = S.sn_ptr[s], hi = S.sn_ptr[s + 1] - 1;
        below.clear();
        for (int32_t c = lo; c <= hi; ++c)
            for (int64_t p = S.Cp[c]; p < S.Cp[c + 1]; ++p) {
                int32_t i = S.Ci[p];
                if (i > hi && mark[i] != s) { mark[i] = (int32_t)s; below.push_back(i); }
            }
        for (int32_t c = chead[s]; c != -1; c = cnext[c]) {
            const int32_t wc = S.width(c);
            for (int64_t p = S.rowptr[c] + wc; p < S.rowptr[c + 1]; ++p) {
                int32_t i = S.rows[p];
                if (i > hi && mark[i] != s) { mark[i] = (int32_t)s; below.push_back(i); }
            }
        }
        std::sort(below.begin(), below.end());
        for (int32_t c = lo; c <= hi; ++c) S.rows.push_back(c);
        S.rows.insert(S.rows.end(), below.begin(), below.end());
        S.rowptr[s + 1] = (int64_t)S.rows.size();
        // a correct etree makes the stored count of the last column exact
        if ((int64_t)below.size() != (int64_t)S.colcount[hi] - 1) return ERR_PATTERN;
    }
    return OK;
}

void layout(Symbolic& S) {
    const int64_t ns = S.nsup;
    S.off.resize((size_t)ns);
    S.ld.resize((size_t)ns);
    S.arena = 0;
    S.nnz_stored = 0;
    S.flops_stored = 0.0;
    S.max_w = S.max_r = 0;
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t w = S.width(s), m = S.nrows(s), r = m - w;
        S.off[s] = S.arena;
        S.ld[s] = (int32_t)m;
        S.arena += m * w;
        S.max_w = std::max<int32_t>(S.max_w, (int32_t)w);
        S.max_r = std::max<int32_t>(S.max_r, (int32_t)r);
        for (int64_t c = 0; c < w; ++c) {
            const double st = (double)(w - c + r);
            S.nnz_stored += (int64_t)st;
            S.flops_stored += st * st;
        }
    }
}

// Position of global row g inside supernode t's row list (g must be present).
int64_t find_row(const Symbolic& S, int64_t t, int32_t g) {
    const int32_t lo = S.sn_ptr[t], hi = S.sn_ptr[t + 1] - 1;
    if (g >= lo && g <= hi) return g - lo;
    auto b = S.rows.begin() + S.rowptr[t] + (hi - lo + 1), e = S.rows.begin() + S.rowptr[t + 1];
    auto it = std::lower_bound(b, e, g);
    if (it == e || *it != g) return -1;
    return (int64_t)(hi - lo + 1) + (it - b);
}

int32_t slots(Symbolic& S) {
    const int64_t n = S.n;
    std::vector<int64_t> cslot((size_t)S.nnz_a);
    for (int64_t j = 0; j < n; ++j) {
        const int64_t s = S.col_owner[j];
        const int64_t lc = j - S.sn_ptr[s];
        for (int64_t q = S.Cp[j]; q < S.Cp[j + 1]; ++q) {
            int64_t lr = find_row(S, s, S.Ci[q]);
            if (lr < 0) return ERR_PATTERN;
            cslot[q] = S.off[s] + lr + lc * S.ld[s];
        }
    }
    S.slot.resize((size_t)S.nnz_a);
    for (int64_t p = 0; p < S.nnz_a; ++p) S.slot[p] = cslot[S.amap[p]];
    return OK;
}

// Update pairs (tasks U/A of Section III-A) and their relative indices.
int32_t pairs(Symbolic& S) {
    const int64_t ns = S.nsup;
    S.pair_ptr.assign((size_t)ns + 1, 0);
    S.pairs.clear();
    S.rel.clear();
    int64_t rel_off = 0;
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t w = S.width(s), r = S.nbelow(s);
        const int32_t* B = S.rows.data() + S.rowptr[s] + w;
        int32_t i = 0;
        while (i < r) {
            const int32_t t = S.col_owner[B[i]];
            int32_t e = i;
            while (e < r && S.col_owner[B[e]] == t) ++e;
            Pair pr{(int32_t)s, t, i, e, rel_off};
            // merge walk: B[i..r) and t's row list are both sorted
            const int32_t tlo = S.sn_ptr[t], thi = S.sn_ptr[t + 1] - 1, wt = thi - tlo + 1;
            const int32_t* TB = S.rows.data() + S.rowptr[t] + wt;
            const int64_t tr = S.nbelow(t);
            int64_t q = 0;
            for (int32_t k = i; k < r; ++k) {
                const int32_t g = B[k];
                if (g <= thi) { S.rel.push_back(g - tlo); continue; }
                while (q < tr && TB[q] < g) ++q;
                if (q == tr || TB[q] != g) return ERR_PATTERN;  // containment violated
                S.rel.push_back((int32_t)(wt + q));
            }
            rel_off += r - i;
            S.pairs.push_back(pr);
            i = e;
        }
        S.pair_ptr[s + 1] = (int64_t)S.pairs.size();
    }
    return OK;
}

void levels(Symbolic& S) {
    const int64_t ns = S.nsup;
    S.level.assign((size_t)ns, 0);
    int32_t top = -1;
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t p = S.sn_parent[s];
        if (p >= 0) S.level[p] = std::max(S.level[p], S.level[s] + 1);
        top = std::max(top, S.level[s]);
    }
    const int32_t nl = top + 1;
    S.level_ptr.assign((size_t)nl + 1, 0);
    for (int64_t s = 0; s < ns; ++s) S.level_ptr[S.level[s] + 1]++;
    for (int32_t l = 0; l < nl; ++l) S.level_ptr[l + 1] += S.level_ptr[l];
    S.level_sn.resize((size_t)ns);
    std::vector<int32_t> fill(S.level_ptr.begin(), S.level_ptr.end() - 1);
    for (int64_t s = 0; s < ns; ++s) S.level_sn[fill[S.level[s]]++] = (int32_t)s;
}

}  // namespace

int32_t analyze(int64_t n, const int64_t* colptr, const int32_t* rowind, const int32_t* perm,
                const Options& opt, Symbolic* out) {
    if (!out) return ERR_ARG;
    if (opt.sn_cap < 1 || !(opt.amalg_ratio >= 0.0) || opt.amalg_ratio > 1.0) return ERR_ARG;
    int32_t st = validate_input(n, colptr, rowind, perm);
    if (st != OK) return st;
    Symbolic& S = *out;
    S = Symbolic();
    S.n = n;
    S.opt = opt;
    S.batch_ptr = {0, n};
    S.nnz_a = n ? colptr[n] : 0;
    S.perm.resize((size_t)n);
    for (int64_t k = 0; k < n; ++k) S.perm[k] = perm ? perm[k] : (int32_t)k;
    permute_lower(S, colptr, rowind);
    // row lists of the strictly lower part (for Liu's algorithm)
    std::vector<int64_t> Rp((size_t)n + 1, 0);
    std::vector<int32_t> Rj;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t p = S.Cp[j]; p < S.Cp[j + 1]; ++p)
            if (S.Ci[p] != j) Rp[S.Ci[p] + 1]++;
    for (int64_t i = 0; i < n; ++i) Rp[i + 1] += Rp[i];
    Rj.resize((size_t)Rp[n]);
    {
        std::vector<int64_t> nx(Rp.begin(), Rp.end() - 1);
        for (int64_t j = 0; j < n; ++j)
            for (int64_t p = S.Cp[j]; p < S.Cp[j + 1]; ++p)
                if (S.Ci[p] != j) Rj[nx[S.Ci[p]]++] = (int32_t)j;
    }
    etree(S, Rp, Rj);
    postorder(S);
    column_counts(S);
    partition(S);
    amalgamate(S);
    if ((st = structures(S)) != OK) return st;
    layout(S);
    if ((st = slots(S)) != OK) return st;
    if ((st = pairs(S)) != OK) return st;
    levels(S);
    return OK;
}

namespace {

// Where member B of a batch goes in the joined analysis: its first row and
// column, input entry, supernode, row-list entry, pair, relative index and
// arena element.
struct MemberOffsets {
    int64_t o = 0, e = 0, s = 0, r = 0, p = 0, rel = 0, arena = 0;
};

// Writes member analysis B into its slices of the joined analysis A (sized
// beforehand).  Every index of B moves by the matching offset; relative
// indices and segment bounds are local to a supernode and stay.
void place_member(Symbolic& A, const Symbolic& B, const MemberOffsets& m) {
    const auto shift = [](int32_t* dst, const std::vector<int32_t>& src, int64_t by,
                          bool keep_neg) {
        for (size_t k = 0; k < src.size(); ++k)
            dst[k] = keep_neg && src[k] < 0 ? src[k] : (int32_t)(src[k] + by);
    };
    shift(A.perm.data() + m.o, B.perm, m.o, false);
    for (int64_t j = 0; j < B.n; ++j) A.Cp[m.o + j + 1] = m.e + B.Cp[j + 1];
    shift(A.Ci.data() + m.e, B.Ci, m.o, false);
    for (int64_t q = 0; q < B.nnz_a; ++q) {
        A.amap[m.e + q] = m.e + B.amap[q];
        A.slot[m.e + q] = m.arena + B.slot[q];
    }
    shift(A.parent.data() + m.o, B.parent, m.o, true);
    std::copy(B.colcount.begin(), B.colcount.end(), A.colcount.begin() + m.o);
    shift(A.post.data() + m.o, B.post, m.o, false);
    shift(A.col_owner.data() + m.o, B.col_owner, m.s, false);
    for (int64_t s = 0; s < B.nsup; ++s) {
        A.sn_ptr[m.s + s + 1] = (int32_t)(m.o + B.sn_ptr[s + 1]);
        A.rowptr[m.s + s + 1] = m.r + B.rowptr[s + 1];
        A.pair_ptr[m.s + s + 1] = m.p + B.pair_ptr[s + 1];
        A.off[m.s + s] = m.arena + B.off[s];
    }
    shift(A.sn_parent.data() + m.s, B.sn_parent, m.s, true);
    std::copy(B.ld.begin(), B.ld.end(), A.ld.begin() + m.s);
    std::copy(B.level.begin(), B.level.end(), A.level.begin() + m.s);
    shift(A.rows.data() + m.r, B.rows, m.o, false);
    for (size_t k = 0; k < B.pairs.size(); ++k) {
        Pair p = B.pairs[k];
        p.src += (int32_t)m.s;
        p.tgt += (int32_t)m.s;
        p.rel_off += m.rel;
        A.pairs[m.p + k] = p;
    }
    std::copy(B.rel.begin(), B.rel.end(), A.rel.begin() + m.rel);
}

// Runs fn(k) for k in [0, count) on up to nt threads (member k on thread
// k mod nt); where a thread cannot be started its members run on the caller.
template <class Fn>
void for_members(int32_t count, int nt, Fn fn) {
    auto work = [&](int t) {
        for (int32_t k = t; k < count; k += nt) fn(k);
    };
    std::vector<std::thread> pool;
    int started = 1;
    try {
        for (; started < nt; ++started) pool.emplace_back(work, started);
    } catch (const std::system_error&) {
    }
    for (int t = started; t < nt; ++t) work(t);
    work(0);
    for (auto& th : pool) th.join();
}

}  // namespace

int32_t analyze_batch(int32_t count, const int64_t* n, const int64_t* const* colptr,
                      const int32_t* const* rowind, const int32_t* const* perm,
                      const Options& opt, int threads, Symbolic* out) {
    if (!out || count < 0) return ERR_ARG;
    std::vector<Symbolic> part((size_t)count);
    std::vector<int32_t> st((size_t)count, OK);
    const int nt = std::max(1, std::min<int>(threads, count));
    for_members(count, nt, [&](int32_t k) {
        try {
            st[k] = analyze(n[k], colptr[k], rowind[k], perm ? perm[k] : nullptr, opt, &part[k]);
        } catch (const std::bad_alloc&) {
            st[k] = ERR_OOM;
        } catch (...) {  // nothing may leave a worker thread
            st[k] = ERR_ARG;
        }
    });
    for (int32_t k = 0; k < count; ++k)
        if (st[k] != OK) return st[k];
    Symbolic& A = *out;
    A = Symbolic();
    A.opt = opt;
    std::vector<MemberOffsets> at((size_t)count + 1);
    int32_t nl = 0;
    A.batch_ptr.assign(1, 0);
    for (int32_t k = 0; k < count; ++k) {
        const Symbolic& B = part[k];
        MemberOffsets m = at[k];
        m.o += B.n;
        m.e += B.nnz_a;
        m.s += B.nsup;
        m.r += (int64_t)B.rows.size();
        m.p += (int64_t)B.pairs.size();
        m.rel += (int64_t)B.rel.size();
        m.arena += B.arena;
        at[k + 1] = m;
        A.batch_ptr.push_back(m.o);
        A.nnz_l += B.nnz_l;
        A.flops += B.flops;
        A.nnz_stored += B.nnz_stored;
        A.flops_stored += B.flops_stored;
        A.max_w = std::max(A.max_w, B.max_w);
        A.max_r = std::max(A.max_r, B.max_r);
        nl = std::max<int32_t>(nl, (int32_t)B.level_ptr.size() - 1);
    }
    const MemberOffsets& T = at[count];
    A.n = T.o;
    A.nnz_a = T.e;
    A.nsup = T.s;
    A.arena = T.arena;
    const size_t N = (size_t)T.o, E = (size_t)T.e, NS = (size_t)T.s;
    // the joined arrays are sized side by side: their first touch (zero fill
    // and page faults) costs more than the copy that follows
    const std::function<void()> sizing[] = {
        [&] { A.perm.resize(N); }, [&] { A.Cp.assign(N + 1, 0); }, [&] { A.Ci.resize(E); },
        [&] { A.amap.resize(E); }, [&] { A.slot.resize(E); }, [&] { A.parent.resize(N); },
        [&] { A.colcount.resize(N); }, [&] { A.post.resize(N); },
        [&] { A.col_owner.resize(N); }, [&] { A.sn_ptr.assign(NS + 1, 0); },
        [&] { A.rowptr.assign(NS + 1, 0); }, [&] { A.pair_ptr.assign(NS + 1, 0); },
        [&] { A.off.resize(NS); }, [&] { A.sn_parent.resize(NS); }, [&] { A.ld.resize(NS); },
        [&] { A.level.resize(NS); }, [&] { A.rows.resize((size_t)T.r); },
        [&] { A.pairs.resize((size_t)T.p); }, [&] { A.rel.resize((size_t)T.rel); }};
    const int32_t nsizing = (int32_t)(sizeof(sizing) / sizeof(sizing[0]));
    std::vector<int32_t> oom((size_t)nsizing, 0);
    for_members(nsizing, std::min<int>(nt, nsizing), [&](int32_t k) {
        try {
            sizing[k]();
        } catch (...) {  // bad_alloc or length_error: either way the join cannot be held
            oom[k] = 1;
        }
    });
    if (std::find(oom.begin(), oom.end(), 1) != oom.end()) return ERR_OOM;
    for_members(count, nt, [&](int32_t k) {
        place_member(A, part[k], at[k]);
        part[k] = Symbolic();
    });
    // level sets: level l of the whole holds every member's level l, members
    // in order, each member's supernodes already increasing
    A.level_ptr.assign((size_t)nl + 1, 0);
    for (int32_t lv : A.level) A.level_ptr[lv + 1]++;
    for (int32_t l = 0; l < nl; ++l) A.level_ptr[l + 1] += A.level_ptr[l];
    A.level_sn.resize(NS);
    std::vector<int32_t> fill(A.level_ptr.begin(), A.level_ptr.end() - 1);
    for (size_t s = 0; s < NS; ++s) A.level_sn[fill[A.level[s]]++] = (int32_t)s;
    return OK;
}

}  // namespace spc
