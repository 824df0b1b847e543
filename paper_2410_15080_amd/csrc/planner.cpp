// Host planner: validation, FLOP-greedy path, per-step index tables,
// absorption of coefficient tensors into operand loads, and the memory plans
// of the per-step and fused executors.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <climits>
#include <map>
#include <sstream>

#include "htn_core.hpp"

namespace htn {

static Error make_err(htn_status s, const std::string &m) { return Error{s, m}; }

void validate_structure(const Net &n) {
    const int L = (int)n.dims.size();
    for (int l = 0; l < L; ++l)
        if (n.dims[l] < 1) throw make_err(HTN_E_SHAPE, "label " + std::to_string(l) + " has extent < 1");
    std::vector<char> carried(L, 0);
    for (int i = 0; i < n.n_t; ++i) {
        const auto &ls = n.labels[i];
        if (ls.empty()) throw make_err(HTN_E_SHAPE, "tensor " + std::to_string(i) + " has rank 0");
        double sz = 1.0;
        for (size_t a = 0; a < ls.size(); ++a) {
            if (ls[a] < 0 || ls[a] >= L)
                throw make_err(HTN_E_LABEL, "tensor " + std::to_string(i) + ": label out of range");
            for (size_t b = 0; b < a; ++b)
                if (ls[b] == ls[a])
                    throw make_err(HTN_E_LABEL, "tensor " + std::to_string(i) + ": label repeated");
            sz *= (double)n.dims[ls[a]];
            carried[ls[a]] = 1;
        }
        if (sz > 2147483647.0)
            throw make_err(HTN_E_SHAPE, "tensor " + std::to_string(i) + " has more than 2^31-1 elements");
    }
    double osz = 1.0;
    for (size_t a = 0; a < n.out_labels.size(); ++a) {
        int l = n.out_labels[a];
        if (l < 0 || l >= L) throw make_err(HTN_E_LABEL, "output label out of range");
        for (size_t b = 0; b < a; ++b)
            if (n.out_labels[b] == l) throw make_err(HTN_E_LABEL, "output label repeated");
        if (!carried[l]) throw make_err(HTN_E_LABEL, "output label " + std::to_string(l) + " is carried by no tensor");
        osz *= (double)n.dims[l];
    }
    if (osz > 2147483647.0) throw make_err(HTN_E_SHAPE, "output has more than 2^31-1 elements");
}

static double prod_dims(const Net &n, const std::vector<int> &ls) {
    double p = 1.0;
    for (int l : ls) p *= (double)n.dims[l];
    return p;
}

static std::vector<int> sorted_union(const std::vector<int> &a, const std::vector<int> &b) {
    std::vector<int> u;
    std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(u));
    return u;
}

static bool contains(const std::vector<int> &v, int x) { return std::find(v.begin(), v.end(), x) != v.end(); }

// splitmix64: a small deterministic generator for path sampling.
struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// Greedy pairwise order.  Candidates are live pairs that share a label; a
// pair's cost is its multiplication count (product of the extents of the
// union of the two label sets).  Without a generator the cheapest pair is
// taken (ties: smaller result, then lower (i, j)) -- the FLOP-greedy path.
// With a generator a pair is drawn with probability proportional to
// exp(-(log2 cost - log2 min cost) / temperature) (Boltzmann-sampled greedy).
// When no pair shares a label the two smallest live tensors are joined.
// *total receives the path's multiplication count and *peak its largest
// intermediate.
static std::vector<std::pair<int, int>> greedy_core(const Net &n, Rng *rng, double temperature, double *total,
                                                   double *peak) {
    const int N = n.n_t;
    const int L = (int)n.dims.size();
    std::vector<std::vector<int>> lab(2 * N);
    std::vector<char> alive(2 * N, 0);
    std::vector<int> ref(L, 0);
    std::vector<char> is_out(L, 0);
    for (int l : n.out_labels) is_out[l] = 1;
    for (int i = 0; i < N; ++i) {
        lab[i] = n.labels[i];
        std::sort(lab[i].begin(), lab[i].end());
        alive[i] = 1;
        for (int l : lab[i]) ref[l]++;
    }
    std::vector<std::pair<int, int>> path;
    int next = N, n_alive = N;
    double tot = 0.0, pk = 0.0;
    std::vector<std::vector<int>> holders(L);
    struct Cand {
        double cost, os;
        int i, j;
        int absorb;  // 1: an input scaled by another input (a1 absorption)
    };
    // ids holding an input (possibly with absorbed factors): absorbing one
    // into another is a scaling of a load, not a kernel step
    std::vector<char> is_input(2 * N, 0);
    for (int i = 0; i < N; ++i) is_input[i] = 1;
    std::vector<Cand> cands;
    auto eval = [&](int i, int j, Cand &c, std::vector<int> *kept_out) {
        std::vector<int> u = sorted_union(lab[i], lab[j]);
        c.cost = prod_dims(n, u);
        c.i = i;
        c.j = j;
        double os = 1.0;
        for (int l : u) {
            int r = ref[l] - (int)contains(lab[i], l) - (int)contains(lab[j], l);
            if (is_out[l] || r > 0) {
                os *= (double)n.dims[l];
                if (kept_out) kept_out->push_back(l);
            }
        }
        c.os = os;
        // absorption: both are inputs, one label set holds the other, and no
        // label of extent above 1 is summed
        c.absorb = 0;
        if (is_input[i] && is_input[j] &&
            (std::includes(lab[i].begin(), lab[i].end(), lab[j].begin(), lab[j].end()) ||
             std::includes(lab[j].begin(), lab[j].end(), lab[i].begin(), lab[i].end()))) {
            c.absorb = 1;
            for (int l : u) {
                const int r = ref[l] - (int)contains(lab[i], l) - (int)contains(lab[j], l);
                if (!is_out[l] && r <= 0 && n.dims[l] > 1) c.absorb = 0;
            }
        }
    };
    auto take = [&](int i, int j) {
        Cand c;
        std::vector<int> kept;
        eval(i, j, c, &kept);
        tot += c.cost;
        pk = std::max(pk, c.os);
        path.push_back({i, j});
        for (int l : lab[i]) ref[l]--;
        for (int l : lab[j]) ref[l]--;
        alive[i] = alive[j] = 0;
        lab[next] = kept;
        for (int l : kept) ref[l]++;
        alive[next] = 1;
        is_input[next] = is_input[i] && is_input[j] && c.absorb;
        ++next;
        --n_alive;
    };
    while (n_alive > 1) {
        for (auto &h : holders) h.clear();
        for (int i = 0; i < next; ++i)
            if (alive[i])
                for (int l : lab[i]) holders[l].push_back(i);
        cands.clear();
        for (int l = 0; l < L; ++l) {
            const auto &h = holders[l];
            for (size_t x = 0; x < h.size(); ++x)
                for (size_t y = x + 1; y < h.size(); ++y) {
                    Cand c;
                    eval(std::min(h[x], h[y]), std::max(h[x], h[y]), c, nullptr);
                    cands.push_back(c);
                }
        }
        // the same pair can appear under several shared labels
        std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) {
            if (a.cost != b.cost) return a.cost < b.cost;
            if (a.os != b.os) return a.os < b.os;
            if (a.i != b.i) return a.i < b.i;
            return a.j < b.j;
        });
        cands.erase(std::unique(cands.begin(), cands.end(),
                                [](const Cand &a, const Cand &b) { return a.i == b.i && a.j == b.j; }),
                    cands.end());
        int bi, bj;
        if (cands.empty()) {
            std::vector<std::pair<double, int>> sz;
            for (int i = 0; i < next; ++i)
                if (alive[i]) sz.push_back({prod_dims(n, lab[i]), i});
            std::sort(sz.begin(), sz.end());
            bi = std::min(sz[0].second, sz[1].second);
            bj = std::max(sz[0].second, sz[1].second);
        } else if (!rng || cands.size() == 1) {
            // among the cheapest pairs an absorption goes first
            const Cand *c = &cands[0];
            for (const Cand &x : cands) {
                if (x.cost != cands[0].cost) break;
                if (x.absorb) {
                    c = &x;
                    break;
                }
            }
            bi = c->i;
            bj = c->j;
        } else {
            const double lmin = std::log2(cands[0].cost);
            double wsum = 0.0;
            std::vector<double> wts(cands.size());
            for (size_t k = 0; k < cands.size(); ++k) {
                wts[k] = std::exp(-(std::log2(cands[k].cost) - lmin) / temperature);
                wsum += wts[k];
            }
            double r = rng->uniform() * wsum;
            size_t k = 0;
            while (k + 1 < cands.size() && r >= wts[k]) r -= wts[k++];
            // a drawn step that ties with an absorption defers to it (an
            // absorption is a scaling of a load, never a kernel step)
            if (!cands[k].absorb)
                for (const Cand &x : cands) {
                    if (x.cost > cands[k].cost) break;
                    if (x.cost == cands[k].cost && x.absorb) {
                        k = (size_t)(&x - cands.data());
                        break;
                    }
                }
            bi = cands[k].i;
            bj = cands[k].j;
        }
        take(bi, bj);
    }
    if (total) *total = tot;
    if (peak) *peak = pk;
    return path;
}

std::vector<std::pair<int, int>> greedy_path(const Net &n) { return greedy_core(n, nullptr, 1.0, nullptr, nullptr); }

std::vector<std::vector<std::pair<int, int>>> candidate_paths(const Net &n, int n_samples, uint64_t seed) {
    std::vector<std::vector<std::pair<int, int>>> out;
    out.push_back(greedy_path(n));
    static const double temps[] = {0.25, 0.5, 1.0, 2.0};
    Rng rng(seed * 0x9e3779b97f4a7c15ull + 12345);
    for (int k = 0; k < n_samples; ++k) out.push_back(greedy_core(n, &rng, temps[k % 4], nullptr, nullptr));
    return out;
}

// Cheapest of the FLOP-greedy path and n_samples Boltzmann-sampled greedy
// paths (by multiplication count, among those within the intermediate cap);
// ties keep the earlier candidate, so the result is never worse than
// FLOP-greedy.
std::vector<std::pair<int, int>> sampled_path(const Net &n, int n_samples, uint64_t seed) {
    double best_m = 0.0;
    std::vector<std::pair<int, int>> best;
    Rng rng(seed * 0x9e3779b97f4a7c15ull + 12345);
    static const double temps[] = {0.25, 0.5, 1.0, 2.0};
    for (int k = -1; k < n_samples; ++k) {
        double m, pk;
        auto p = k < 0 ? greedy_core(n, nullptr, 1.0, &m, &pk) : greedy_core(n, &rng, temps[k % 4], &m, &pk);
        if (pk > (double)n.max_intermediate && k >= 0) continue;
        if (best.empty() || m < best_m) {
            best = p;
            best_m = m;
        }
    }
    return best;
}

Net structure_copy(const Net &n) {
    Net t;
    t.n_t = n.n_t;
    t.labels = n.labels;
    t.dims = n.dims;
    t.out_labels = n.out_labels;
    t.sizes = n.sizes;
    t.storage = n.storage;
    t.compute = n.compute;
    t.final_sum = n.final_sum;
    t.exec = n.exec;
    t.max_intermediate = n.max_intermediate;
    t.fused_lds_budget = n.fused_lds_budget;
    t.fused_threads = n.fused_threads;
    t.fused_max_mults = n.fused_max_mults;
    t.batch_fused_max_mults = n.batch_fused_max_mults;
    t.allow_mfma = n.allow_mfma;
    t.path_samples = n.path_samples;
    t.path_seed = n.path_seed;
    t.slice_mode = n.slice_mode;
    t.queue_mode = n.queue_mode;
    return t;
}

void check_path(const Net &n, const std::vector<std::pair<int, int>> &p) {
    const int N = n.n_t;
    if ((int)p.size() != N - 1)
        throw make_err(HTN_E_PATH, "path must have n_tensors-1 = " + std::to_string(N - 1) + " steps, got " +
                                       std::to_string(p.size()));
    std::vector<char> used(2 * N, 0);
    for (size_t t = 0; t < p.size(); ++t) {
        int i = p[t].first, j = p[t].second;
        int lim = N + (int)t;
        if (i < 0 || j < 0 || i >= lim || j >= lim)
            throw make_err(HTN_E_PATH, "step " + std::to_string(t) + ": id not yet defined");
        if (i == j) throw make_err(HTN_E_PATH, "step " + std::to_string(t) + ": operand used twice");
        if (used[i] || used[j]) throw make_err(HTN_E_PATH, "step " + std::to_string(t) + ": id consumed twice");
        used[i] = used[j] = 1;
    }
}

// ---------------------------------------------------------------- tables

static std::vector<int64_t> strides_of(const Net &n, const std::vector<int> &ls) {
    std::vector<int64_t> s(ls.size());
    int64_t acc = 1;
    for (int k = (int)ls.size() - 1; k >= 0; --k) {
        s[k] = acc;
        acc *= n.dims[ls[k]];
    }
    return s;
}

static int64_t stride_in(const std::vector<int> &ls, const std::vector<int64_t> &st, int l) {
    for (size_t k = 0; k < ls.size(); ++k)
        if (ls[k] == l) return st[k];
    return 0;
}

// Split a label group into (hi, lo): lo is the longest suffix whose extent
// product stays <= kTabLoMax (at least one label when the group is not
// empty).  Append the (A, B) offset tables of both halves to `tab`.
static void group_tables(const Net &n, const std::vector<int> &group, const std::vector<int64_t> &sa,
                         const std::vector<int64_t> &sb, std::vector<int32_t> &tab, int64_t &n_hi, int64_t &n_lo,
                         int64_t &t_hi, int64_t &t_lo) {
    const int G = (int)group.size();
    int split = G;  // labels [split, G) form the low half
    int64_t p = 1;
    while (split > 0 && (split == G || p * n.dims[group[split - 1]] <= kTabLoMax)) {
        p *= n.dims[group[split - 1]];
        --split;
    }
    auto emit = [&](int from, int to, int64_t &count, int64_t &off) {
        count = 1;
        for (int k = from; k < to; ++k) count *= n.dims[group[k]];
        off = (int64_t)tab.size() / 2;
        std::vector<int64_t> dig(to - from, 0);
        for (int64_t e = 0; e < count; ++e) {
            int64_t oa = 0, ob = 0;
            for (int k = from; k < to; ++k) {
                oa += dig[k - from] * sa[k];
                ob += dig[k - from] * sb[k];
            }
            tab.push_back((int32_t)oa);
            tab.push_back((int32_t)ob);
            for (int k = to - 1; k >= from; --k) {
                if (++dig[k - from] < n.dims[group[k]]) break;
                dig[k - from] = 0;
            }
        }
    };
    emit(0, split, n_hi, t_hi);
    emit(split, G, n_lo, t_lo);
}

static int pow2floor(int64_t x) {
    int r = 1;
    while ((int64_t)r * 2 <= x) r *= 2;
    return r;
}

static int pow2ceil(int64_t x) {
    int r = 1;
    while (r < x && r < (1 << 20)) r *= 2;
    return r;
}

// -------------------------------------------------------------- allocator

// First-fit allocator over [0, inf) used for both the device workspace
// (bytes) and the LDS image of the fused kernel (elements).
struct FirstFit {
    std::map<int64_t, int64_t> used;  // off -> size
    int64_t peak = 0;
    int64_t alloc(int64_t size, int64_t align) {
        int64_t off = 0;
        for (auto &kv : used) {
            if (off + size <= kv.first) break;
            off = (kv.first + kv.second + align - 1) / align * align;
        }
        used[off] = size;
        peak = std::max(peak, off + size);
        return off;
    }
    void release(int64_t off) { used.erase(off); }
};

// ------------------------------------------------------------ build_plan

enum { OP_END = 0, OP_LOAD = 1, OP_STEP = 2, OP_SYNC = 3, OP_TSTEP = 4, OP_COPY = 6 };

// One-level offset table over a label group (pairs, .x = offset).
static void flat_table(const Net &n, const std::vector<int> &group, const std::vector<int64_t> &st,
                       std::vector<int32_t> &tab, int64_t &off) {
    off = (int64_t)tab.size() / 2;
    int64_t count = (int64_t)prod_dims(n, group);
    std::vector<int64_t> dig(group.size(), 0);
    for (int64_t e = 0; e < count; ++e) {
        int64_t o = 0;
        for (size_t k = 0; k < group.size(); ++k) o += dig[k] * st[k];
        tab.push_back((int32_t)o);
        tab.push_back(0);
        for (int k = (int)group.size() - 1; k >= 0; --k) {
            if (++dig[k] < n.dims[group[k]]) break;
            dig[k] = 0;
        }
    }
}

// Register tile of a tiled step: TM x TN outputs per thread on a GX x GY
// thread grid (GX * GY = threads).  The kernel runs U = 16 / (TM*TN)
// (at most 8, at least 1) independent partial sums over k.  Modelled time
// of a thread, in FMA-issue slots: passes * (30 + blocks * max(24, U *
// (TM*TN + (TM+TN)/2)) + tail * 24) with blocks = floor(K / U) and
// tail = K mod U: a k-block cannot finish faster than one LDS round trip
// (~24 slots), so large tiles and few passes win when K is small.
static void choose_tile(StepPlan &s, int threads) {
    double best = 0;
    for (int tm : {1, 2, 4})
        for (int tn : {1, 2, 4})
            for (int gx = 1; gx <= threads; gx *= 2) {
                const int gy = threads / gx;
                const double passes = std::ceil((double)s.tM / (gx * tm)) * std::ceil((double)s.tN / (gy * tn));
                const int u = tm * tn >= 16 ? 1 : (tm * tn >= 8 ? 2 : (tm * tn >= 4 ? 4 : 8));
                const double blocks = std::floor((double)s.tK / u), tail = (double)(s.tK % u);
                const double per = 30.0 + blocks * std::max(24.0, u * (tm * tn + 0.5 * (tm + tn))) + tail * 24.0;
                const double cost = passes * per;
                if (best == 0 || cost < best - 1e-9) {
                    best = cost;
                    s.TM = tm;
                    s.TN = tn;
                    s.GX = gx;
                }
            }
}

// Steps that are dense matrix products go to the matrix cores: every summed
// label is carried by both operands (K), the kept labels split into batch
// (both), M (A only) and N (B only), and the product is large enough.  The
// result is laid out [batch][M][N]; for the final step the output labels
// must already be in that grouped order.
constexpr double kMfmaMinMults = 4194304.0;

static void classify_mfma(const Net &n, StepPlan &s, const std::vector<int> &al, const std::vector<int> &bl,
                          const std::vector<int> &kept, const std::vector<int> &sums, bool last) {
    s.mfma = 0;
    if (!n.allow_mfma || s.mults < kMfmaMinMults) return;
    for (int l : sums)
        if (!contains(al, l) || !contains(bl, l)) return;
    auto kept_has = [&](int l) { return std::binary_search(kept.begin(), kept.end(), l); };
    std::vector<int> gb, gm, gn, gk;
    for (int l : al) {
        if (kept_has(l))
            (contains(bl, l) ? gb : gm).push_back(l);
        else
            gk.push_back(l);
    }
    for (int l : bl)
        if (kept_has(l) && !contains(al, l)) gn.push_back(l);
    const int64_t M = (int64_t)prod_dims(n, gm), N = (int64_t)prod_dims(n, gn), K = (int64_t)prod_dims(n, gk);
    if (M < 64 || N < 64 || K < 8) return;
    if (last) {
        // output order must read batch..., M..., N...
        const auto &o = n.out_labels;
        size_t p = 0;
        std::vector<int> ob, om, on;
        for (; p < o.size() && contains(gb, o[p]); ++p) ob.push_back(o[p]);
        for (; p < o.size() && contains(gm, o[p]); ++p) om.push_back(o[p]);
        for (; p < o.size() && contains(gn, o[p]); ++p) on.push_back(o[p]);
        if (p != o.size() || ob.size() != gb.size() || om.size() != gm.size() || on.size() != gn.size()) return;
        gb = ob;
        gm = om;
        gn = on;
    }
    s.mfma = 1;
    s.g_batch = gb;
    s.g_m = gm;
    s.g_n = gn;
    s.g_k = gk;
    s.gb = (int64_t)prod_dims(n, gb);
    s.gm = M;
    s.gn = N;
    s.gk = K;
    s.c_labels = gb;
    s.c_labels.insert(s.c_labels.end(), gm.begin(), gm.end());
    s.c_labels.insert(s.c_labels.end(), gn.begin(), gn.end());
    s.sum_labels = gk;
}

FoldLayout fold_layout(const Net &n, const Plan &P, const std::vector<int> &chain) {
    constexpr int kAx = 8, kOuter = 4, kStages = 8;
    constexpr int64_t kTileMax = 1024, kLdsMax = 81920;
    FoldLayout F;
    if (chain.empty() || (int)chain.size() > kStages) return F;
    auto row_major = [&](const std::vector<int> &labels) {
        std::vector<int64_t> st(labels.size(), 1);
        for (int k = (int)labels.size() - 2; k >= 0; --k) st[k] = st[k + 1] * n.dims[labels[k + 1]];
        return st;
    };
    // the chain's source: the head's larger operand; its labels are the axes
    const StepPlan &h = P.steps[chain[0]];
    if (h.a < 0 || h.b < 0) return F;
    F.x = P.values[h.a].size >= P.values[h.b].size ? h.a : h.b;
    const std::vector<int> &xl = P.values[F.x].labels;
    std::vector<int64_t> xs = row_major(xl);
    {
        // an input without folded scales is read in place: the strides of
        // its original tensor (labels it has beyond X's have extent 1)
        const Value &XV = P.values[F.x];
        if (XV.input && XV.scales.empty() && XV.base >= 0) {
            const std::vector<int> &bl = n.labels[XV.base];
            const std::vector<int64_t> bs = row_major(bl);
            std::vector<int64_t> raw(xl.size(), -1);
            bool ok = true;
            for (size_t j = 0; j < xl.size(); ++j) {
                for (size_t q = 0; q < bl.size(); ++q)
                    if (bl[q] == xl[j]) raw[j] = bs[q];
                if (raw[j] < 0) ok = false;
            }
            for (int l : bl)
                if (!contains(xl, l) && n.dims[l] != 1) ok = false;
            if (ok) {
                xs = raw;
                F.x_raw = true;
            }
        }
    }
    std::vector<int> cur = xl;
    std::vector<char> folded(xl.size(), 0);
    int prev = F.x;
    for (int k : chain) {
        const StepPlan &s = P.steps[k];
        const int m = s.a == prev ? s.b : (s.b == prev ? s.a : -1);
        if (m < 0 || s.sum_labels.size() != 1) return F;
        const Value &M = P.values[m];
        if (!M.input || M.labels.size() != 2) return F;
        const int l = s.sum_labels[0];
        const int lp = M.labels[0] == l ? M.labels[1] : M.labels[0];
        int ax = -1;
        for (size_t j = 0; j < cur.size(); ++j)
            if (cur[j] == l) ax = (int)j;
        if (ax < 0) return F;
        // the matrix is read raw: strides of its original tensor
        const std::vector<int> &ml = n.labels[M.base];
        const std::vector<int64_t> ms = row_major(ml);
        if (ml.size() != 2) return F;
        F.fold_ax.push_back(ax);
        F.fold_ext.push_back((int)n.dims[lp]);
        F.m_tensor.push_back(M.base);
        F.m_in.push_back(ml[0] == l ? ms[0] : ms[1]);
        F.m_out.push_back(ml[0] == l ? ms[1] : ms[0]);
        cur[ax] = lp;
        folded[ax] = 1;
        prev = s.c;
    }
    F.y = prev;
    const std::vector<int> &yl = P.values[F.y].labels;
    const std::vector<int64_t> ys = row_major(yl);
    if (yl.size() != xl.size()) return F;
    std::vector<int64_t> dst_of(xl.size(), -1);
    for (size_t j = 0; j < xl.size(); ++j)
        for (size_t q = 0; q < yl.size(); ++q)
            if (yl[q] == cur[j]) dst_of[j] = ys[q];
    for (int64_t d : dst_of)
        if (d < 0) return F;
    // largest in-tile size over the stages for the current in-tile axes
    std::vector<char> tile(xl.size(), 1);
    auto d_max = [&]() {
        std::vector<int64_t> e(xl.size());
        for (size_t j = 0; j < xl.size(); ++j) e[j] = n.dims[xl[j]];
        auto size = [&]() {
            int64_t p = 1;
            for (size_t j = 0; j < xl.size(); ++j)
                if (tile[j]) p *= e[j];
            return p;
        };
        int64_t mx = size();
        for (size_t st = 0; st < F.fold_ax.size(); ++st) {
            e[F.fold_ax[st]] = F.fold_ext[st];
            mx = std::max(mx, size());
        }
        return mx;
    };
    // move the largest carried axes out of the tile until it is small
    while (d_max() > kTileMax) {
        int best = -1;
        for (size_t j = 0; j < xl.size(); ++j)
            if (tile[j] && !folded[j] && (best < 0 || n.dims[xl[j]] > n.dims[xl[best]])) best = (int)j;
        if (best < 0) return F;
        tile[best] = 0;
    }
    // in-tile axes by falling destination stride (stores run along the
    // fastest), outer axes by falling source stride (loads run along it)
    std::vector<int> in_ax, out_ax;
    for (size_t j = 0; j < xl.size(); ++j) (tile[j] ? in_ax : out_ax).push_back((int)j);
    std::stable_sort(in_ax.begin(), in_ax.end(), [&](int p, int q) { return dst_of[p] > dst_of[q]; });
    std::stable_sort(out_ax.begin(), out_ax.end(), [&](int p, int q) { return xs[p] > xs[q]; });
    if ((int)in_ax.size() > kAx || (int)out_ax.size() > kOuter) return F;
    std::vector<int> pos(xl.size(), -1);
    for (size_t q = 0; q < in_ax.size(); ++q) pos[in_ax[q]] = (int)q;
    for (size_t q = 0; q < in_ax.size(); ++q) {
        const int j = in_ax[q];
        F.ext0.push_back((int)n.dims[xl[j]]);
        F.ext1.push_back((int)n.dims[cur[j]]);
        F.s_src.push_back(xs[j]);
        F.s_dst.push_back(dst_of[j]);
    }
    for (int &a : F.fold_ax) a = pos[a];
    for (int j : out_ax) {
        F.o_ext.push_back((int)n.dims[xl[j]]);
        F.o_src.push_back(xs[j]);
        F.o_dst.push_back(dst_of[j]);
        F.n_outer *= n.dims[xl[j]];
    }
    F.d_max = (int)d_max();
    const int64_t es = dtype_size(inter_dtype(n.compute));
    // 16 outer indices per tile: 128-byte runs of an FP64 source axis
    F.tf = 16;
    while (F.tf > 1 && 2 * (int64_t)F.d_max * (F.tf + 1) * es > kLdsMax) F.tf /= 2;
    while (F.tf > 1 && F.tf / 2 >= F.n_outer) F.tf /= 2;
    F.lds_bytes = 2 * (int64_t)F.d_max * (F.tf + 1) * es;
    F.ok = F.lds_bytes <= kLdsMax;
    return F;
}

void build_plan(Net &n) {
    const int N = n.n_t;
    const int L = (int)n.dims.size();
    Plan P;
    const auto &path = n.path;
    P.values.resize(N + path.size() + 1);
    std::vector<int> ref(L, 0);
    std::vector<char> is_out(L, 0);
    for (int l : n.out_labels) is_out[l] = 1;
    for (int i = 0; i < N; ++i) {
        Value &v = P.values[i];
        v.labels = n.labels[i];
        v.size = n.sizes[i];
        v.input = true;
        v.base = i;
        for (int l : v.labels) ref[l]++;
    }
    // input values whose data went into another value's load (absorbed or
    // moved); the others are loaded by their own consumer and may carry
    // further folded factors
    std::vector<char> folded(N + path.size() + 1, 0);
    for (size_t t = 0; t < path.size(); ++t) {
        const int i = path[t].first, j = path[t].second, c = N + (int)t;
        const Value A = P.values[i], B = P.values[j];
        std::vector<int> sa = A.labels, sb = B.labels;
        std::sort(sa.begin(), sa.end());
        std::sort(sb.begin(), sb.end());
        std::vector<int> u = sorted_union(sa, sb);
        for (int l : A.labels) ref[l]--;
        for (int l : B.labels) ref[l]--;
        std::vector<int> kept_set, sums;
        for (int l : u) (is_out[l] || ref[l] > 0 ? kept_set : sums).push_back(l);
        StepPlan s;
        s.a = i;
        s.b = j;
        s.c = c;
        s.a_labels = A.labels;
        s.b_labels = B.labels;
        s.mults = prod_dims(n, u);
        P.mults += s.mults;
        const bool last = (t + 1 == path.size());
        // Summing a label of extent 1 changes no value and no layout: such a
        // label may stay on a value (it is summed by a later step at no cost).
        bool sums_trivial = true;
        for (int l : sums) sums_trivial = sums_trivial && n.dims[l] == 1;
        // A scalar factor (an input of one element, such as a CT truncated
        // to one kept index) that meets an intermediate multiplies the whole
        // network: it is applied exactly once by folding it into the load of
        // an input (loads happen before any label is summed, so the order of
        // the path does not matter), and the intermediate's producer writes
        // this step's result directly.  Larger coefficient tensors that meet
        // an intermediate stay kernel steps: folding them would force the
        // carrier input, often loaded straight from its tensor, through the
        // materialisation launch (measured slower on grid batches); path
        // selection absorbs them first instead.
        auto sub_of = [&](const Value &x, const Value &y) {
            for (int l : x.labels)
                if (!contains(y.labels, l) && !std::binary_search(sums.begin(), sums.end(), l)) return false;
            return true;
        };
        int scl = -1, oth = -1;
        if (sums_trivial && A.input != B.input && !last) {
            scl = A.input ? i : j;
            oth = scl == i ? j : i;
            if (!sub_of(P.values[scl], P.values[oth]) || P.values[scl].size != 1) scl = -1;
        }
        if (scl >= 0) {
            const Value &S = P.values[scl];
            int carrier = -1;
            for (int k = 0; k < c; ++k) {
                const Value &K = P.values[k];
                if (!K.input || folded[k] || k == scl) continue;
                if (K.scales.size() + 1 + S.scales.size() > (size_t)kMaxScales) continue;
                bool carries = true;
                for (int l : S.labels) carries = carries && (n.dims[l] == 1 || contains(K.labels, l));
                if (!carries) continue;
                if (carrier < 0 || (P.values[carrier].size == 1 && K.size > 1)) carrier = k;
            }
            if (carrier >= 0) {
                P.values[carrier].scales.push_back(S.base);
                for (int x : S.scales) P.values[carrier].scales.push_back(x);
                folded[scl] = 1;
                Value &C = P.values[c];
                C = P.values[oth];
                P.steps[C.producer].c = c;
                s.absorbed = true;
                s.c_labels = C.labels;
                P.n_absorbed++;
                for (int l : kept_set) ref[l]++;
                s.final_step = false;
                P.steps.push_back(s);
                continue;
            }
        }
        // Absorption: both operands are (possibly already scaled) inputs, one
        // label set contains the other (or the smaller is a scalar whose
        // labels the larger carries or this step sums) and nothing of extent
        // above 1 is summed, so the result is the larger input scaled
        // entry-wise by the smaller one.
        int tgt = -1, sml = -1;
        if (A.input && B.input && sums_trivial && (A.size == 1) != (B.size == 1)) {
            // a scalar factor: its labels all have extent 1 (carried by the
            // other operand or summed here)
            tgt = A.size == 1 ? j : i;
            sml = tgt == i ? j : i;
            bool carried = true;
            for (int l : P.values[sml].labels)
                carried = carried && (contains(P.values[tgt].labels, l) || std::binary_search(sums.begin(), sums.end(), l));
            if (!carried || P.values[tgt].scales.size() + 1 + P.values[sml].scales.size() > (size_t)kMaxScales)
                tgt = -1;
        }
        if (tgt < 0 && A.input && B.input && sums_trivial) {
            bool b_in_a = std::includes(sa.begin(), sa.end(), sb.begin(), sb.end());
            bool a_in_b = std::includes(sb.begin(), sb.end(), sa.begin(), sa.end());
            if (b_in_a && (!a_in_b || A.size >= B.size)) {
                tgt = i;
                sml = j;
            } else if (a_in_b) {
                tgt = j;
                sml = i;
            }
            if (tgt >= 0 && P.values[tgt].scales.size() + 1 + P.values[sml].scales.size() > (size_t)kMaxScales)
                tgt = -1;
        }
        Value &C = P.values[c];
        if (tgt >= 0) {
            s.absorbed = true;
            folded[tgt] = folded[sml] = 1;
            C = P.values[tgt];
            C.scales.push_back(P.values[sml].base);
            for (int x : P.values[sml].scales) C.scales.push_back(x);
            s.c_labels = C.labels;
            P.n_absorbed++;
        } else {
            classify_mfma(n, s, A.labels, B.labels, kept_set, sums, last);
            if (s.mfma) {
                // result laid out [batch][M][N]
            } else if (last) {
                s.c_labels = n.out_labels;
            } else {
                for (int l : A.labels)
                    if (std::binary_search(kept_set.begin(), kept_set.end(), l)) s.c_labels.push_back(l);
                for (int l : B.labels)
                    if (std::binary_search(kept_set.begin(), kept_set.end(), l) && !contains(A.labels, l))
                        s.c_labels.push_back(l);
            }
            if (!s.mfma) {
                for (int l : A.labels)
                    if (std::binary_search(sums.begin(), sums.end(), l)) s.sum_labels.push_back(l);
                for (int l : B.labels)
                    if (std::binary_search(sums.begin(), sums.end(), l) && !contains(A.labels, l))
                        s.sum_labels.push_back(l);
            }
            C.labels = s.c_labels;
            C.input = false;
            C.producer = (int)P.steps.size();
            C.size = (int64_t)prod_dims(n, C.labels);
            P.peak = std::max(P.peak, (double)C.size);
            if ((double)C.size > (double)n.max_intermediate)
                throw make_err(HTN_E_OOM, "step " + std::to_string(t) + " creates " + std::to_string(C.size) +
                                              " elements, above the cap " + std::to_string(n.max_intermediate));
        }
        C.size = (int64_t)prod_dims(n, C.labels);
        for (int l : kept_set) ref[l]++;
        s.final_step = last && !s.absorbed;
        P.steps.push_back(s);
    }
    int fin = path.empty() ? 0 : N + (int)path.size() - 1;
    if (P.values[fin].input) {
        // Everything folded into one input (or a single tensor): finish with
        // a unary step that applies the scales, sums non-output labels and
        // lays the result out in output order.
        StepPlan s;
        s.a = fin;
        s.b = -1;
        s.c = N + (int)path.size();
        s.a_labels = P.values[fin].labels;
        s.c_labels = n.out_labels;
        for (int l : s.a_labels)
            if (!is_out[l]) s.sum_labels.push_back(l);
        s.synthetic = true;
        s.final_step = true;
        Value &C = P.values[s.c];
        C.labels = s.c_labels;
        C.input = false;
        C.producer = (int)P.steps.size();
        C.size = (int64_t)prod_dims(n, C.labels);
        P.steps.push_back(s);
        fin = s.c;
    } else {
        P.values.resize(N + path.size());
    }
    P.final_value = fin;
    for (size_t k = 0; k < P.steps.size(); ++k)
        if (!P.steps[k].absorbed) P.kernel_steps.push_back((int)k);

    // Fused-kernel phases.  A step's level is one more than the levels of
    // the steps producing its operands (inputs: 0); steps of one level are
    // independent, so up to W = threads / 64 of them share a phase, each on
    // its own power-of-two number of waves (more waves to more work).
    {
        const int W = std::max(1, n.fused_threads / 64);
        std::vector<int> level_of(P.values.size(), 0);
        std::vector<std::vector<int>> by_level;
        for (size_t q = 0; q < P.kernel_steps.size(); ++q) {
            StepPlan &s = P.steps[P.kernel_steps[q]];
            int lv = 0;
            for (int id : {s.a, s.b})
                if (id >= 0 && !P.values[id].input) lv = std::max(lv, level_of[id]);
            lv += 1;
            if (s.c >= 0) level_of[s.c] = lv;
            if ((int)by_level.size() < lv) by_level.resize(lv);
            by_level[lv - 1].push_back((int)q);
        }
        // Sharing a phase keeps more values live at once; a phase closes
        // early when its footprint (intermediates carried over from earlier
        // phases + the phase's loaded inputs and results) would pass ~70 %
        // of the LDS budget, so that sharing does not push values out of
        // LDS.
        const double es = (double)dtype_size(inter_dtype(n.compute));
        const double budget = 0.7 * (double)n.fused_lds_budget / es;
        double carry = 0.0;  // intermediates produced and not yet consumed
        std::vector<std::vector<int>> groups;
        for (auto &lv : by_level) {
            std::vector<int> cur;
            double foot = 0.0, made = 0.0, used = 0.0;
            auto close = [&]() {
                if (cur.empty()) return;
                groups.push_back(cur);
                carry += made - used;
                cur.clear();
                foot = made = used = 0.0;
            };
            for (int q : lv) {
                const StepPlan &s = P.steps[P.kernel_steps[q]];
                double in_sz = 0.0, inter_sz = 0.0;
                for (int id : {s.a, s.b})
                    if (id >= 0) (P.values[id].input ? in_sz : inter_sz) += (double)P.values[id].size;
                const double out_sz = s.c >= 0 ? (double)P.values[s.c].size : 0.0;
                if (!cur.empty() && ((int)cur.size() == W || carry + foot + in_sz + out_sz > budget)) close();
                cur.push_back(q);
                foot += in_sz + out_sz;
                made += out_sz;
                used += inter_sz;
            }
            close();
        }
        P.fused_phases.clear();
        for (auto &g : groups) {
                std::vector<int> ph = g;
                // waves: one each, then double the busiest while they fit
                std::vector<int> nw(ph.size(), 1);
                int used = (int)ph.size();
                for (;;) {
                    int best = -1;
                    double bw = -1.0;
                    for (size_t j = 0; j < ph.size(); ++j) {
                        const double w = P.steps[P.kernel_steps[ph[j]]].mults / nw[j];
                        if (used + nw[j] <= W && w > bw) {
                            bw = w;
                            best = (int)j;
                        }
                    }
                    if (best < 0) break;
                    used += nw[best];
                    nw[best] *= 2;
                }
                int w0 = 0;
                for (size_t j = 0; j < ph.size(); ++j) {
                    StepPlan &s = P.steps[P.kernel_steps[ph[j]]];
                    s.f_w0 = w0;
                    s.f_nw = nw[j];
                    w0 += nw[j];
                }
                P.fused_phases.push_back(ph);
            }
    }

    // Layout pass.  Each value is consumed by exactly one kernel step, so its
    // physical label order can be chosen for that consumer: operands of a
    // register-tiled step are laid out [K][M] and [K][N] with the same K
    // order.  Intermediates take the layout when their producer writes them;
    // inputs are permuted when they are loaded (or materialised).
    auto set_layout = [&](int v, const std::vector<int> &order) {
        Value &val = P.values[v];
        if (val.input) {
            val.labels = order;
            return true;
        }
        StepPlan &prod = P.steps[val.producer];
        if (prod.mfma || prod.final_step) return false;
        val.labels = order;
        prod.c_labels = order;
        return true;
    };
    // An intermediate consumed by a matrix-core step is written by its
    // producer directly in the packed order [batch][M][K] / [batch][N][K]
    // (as BF16 when the compute type is BF16: the producer rounds where the
    // pack would have), so that no pack launch is needed.  Only for
    // networks above the batch limit of the fused kernel (those run step by
    // step in every executor choice except an explicit HTN_EXEC_FUSED);
    // below it the register-tiled layout of the fused kernel keeps
    // precedence.
    const bool packed_layouts = P.mults > n.batch_fused_max_mults;
    if (packed_layouts)
        for (int k : P.kernel_steps) {
            StepPlan &s = P.steps[k];
            if (!s.mfma) continue;
            auto packed = [&](const std::vector<int> &mid) {
                std::vector<int> o = s.g_batch;
                o.insert(o.end(), mid.begin(), mid.end());
                o.insert(o.end(), s.g_k.begin(), s.g_k.end());
                return o;
            };
            if (!P.values[s.a].input) set_layout(s.a, packed(s.g_m));
            if (!P.values[s.b].input) set_layout(s.b, packed(s.g_n));
        }
    for (int k : P.kernel_steps) {
        StepPlan &s = P.steps[k];
        if (s.b < 0) continue;
        if (s.mfma && packed_layouts) continue;  // operands keep the packed order
        if (s.final_step && n.final_sum == HTN_SUM_COMPENSATED) continue;
        std::vector<int> al = P.values[s.a].labels, bl = P.values[s.b].labels;
        std::vector<int> K, M, Nn;
        bool ok = true;
        for (int l : s.sum_labels)
            if (!contains(al, l) || !contains(bl, l)) ok = false;
        for (int l : al)
            if (!contains(s.sum_labels, l)) {
                if (contains(bl, l)) ok = false;  // batch label
                M.push_back(l);
            }
        for (int l : bl)
            if (!contains(s.sum_labels, l)) Nn.push_back(l);
        if (!ok) continue;
        if (M.size() > 8 || Nn.size() > 8) continue;  // digit descriptors hold up to 8 labels
        const int64_t mM = (int64_t)prod_dims(n, M), nN = (int64_t)prod_dims(n, Nn);
        if (mM * nN < 64 * s.f_nw) continue;  // fewer outputs than threads: split the sums instead
        K = s.sum_labels;
        std::sort(K.begin(), K.end());
        std::sort(M.begin(), M.end());
        std::sort(Nn.begin(), Nn.end());
        std::vector<int> wa = K, wb = K;
        wa.insert(wa.end(), M.begin(), M.end());
        wb.insert(wb.end(), Nn.begin(), Nn.end());
        // Both operands must accept the layout (an MFMA or final producer
        // keeps its own); otherwise fall back to the table-driven step.
        auto can = [&](int v) { return P.values[v].input || !(P.steps[P.values[v].producer].mfma); };
        if (!can(s.a) || !can(s.b)) continue;
        set_layout(s.a, wa);
        set_layout(s.b, wb);
        s.tile = 1;
        s.tM = mM;
        s.tN = nN;
        s.tK = (int64_t)prod_dims(n, K);
        s.t_gm = M;
        s.t_gn = Nn;
        s.t_gk = K;
    }
    for (int k : P.kernel_steps) {
        StepPlan &s = P.steps[k];
        s.a_labels = P.values[s.a].labels;
        if (s.b >= 0) s.b_labels = P.values[s.b].labels;
        if (!s.final_step) s.c_labels = P.values[s.c].labels;
        if (s.tile) s.sum_labels = s.t_gk;
    }

    // Offset tables and lane counts of every kernel step.
    for (int k : P.kernel_steps) {
        StepPlan &s = P.steps[k];
        auto sta = strides_of(n, s.a_labels);
        std::vector<int64_t> stb = s.b >= 0 ? strides_of(n, s.b_labels) : std::vector<int64_t>();
        std::vector<int64_t> oa, ob, ua, ub;
        for (int l : s.c_labels) {
            oa.push_back(stride_in(s.a_labels, sta, l));
            ob.push_back(s.b >= 0 ? stride_in(s.b_labels, stb, l) : 0);
        }
        for (int l : s.sum_labels) {
            ua.push_back(stride_in(s.a_labels, sta, l));
            ub.push_back(s.b >= 0 ? stride_in(s.b_labels, stb, l) : 0);
        }
        group_tables(n, s.c_labels, oa, ob, P.tables, s.n_ohi, s.n_olo, s.t_ohi, s.t_olo);
        group_tables(n, s.sum_labels, ua, ub, P.tables, s.n_shi, s.n_slo, s.t_shi, s.t_slo);
        if (s.tile) {
            // C offsets of (m, n): tables over the M and N groups
            auto stc = strides_of(n, s.c_labels);
            std::vector<int64_t> cm, cn;
            for (int l : s.t_gm) cm.push_back(stride_in(s.c_labels, stc, l));
            for (int l : s.t_gn) cn.push_back(stride_in(s.c_labels, stc, l));
            flat_table(n, s.t_gm, cm, P.tables, s.t_cm);
            flat_table(n, s.t_gn, cn, P.tables, s.t_cn);
            auto digits = [&](const std::vector<int> &g, const std::vector<int64_t> &st, std::vector<int32_t> &out) {
                out.clear();
                for (size_t k = 0; k < g.size(); ++k) {
                    const uint64_t d = (uint64_t)n.dims[g[k]];
                    const uint64_t magic = ((uint64_t(1) << 40) + d - 1) / d;
                    out.push_back((int32_t)d);
                    out.push_back((int32_t)(uint32_t)(magic & 0xffffffffu));
                    out.push_back((int32_t)(uint32_t)(magic >> 32));
                    out.push_back((int32_t)st[k]);
                }
            };
            digits(s.t_gm, cm, s.c_digits_m);
            digits(s.t_gn, cn, s.c_digits_n);
            choose_tile(s, 64 * s.f_nw);
            // matrix-core mode (TM = 0): 16x16 blocks, one wave each, when
            // the blocks are mostly filled and the accumulator is the
            // compute type (not an FP64 final sum over FP32 data)
            const bool acc_is_compute =
                !s.final_step || n.compute == HTN_F64 || n.final_sum == HTN_SUM_PLAIN;
            if (n.allow_mfma && acc_is_compute && s.tM >= 16 && s.tN >= 16 && s.tK >= 4) {
                s.TM = 0;
                s.TN = 0;
            }
        }
        if (s.mfma) {
            // pack A -> [batch][M][K], B -> [batch][N][K]: unary permutes
            auto pack = [&](const std::vector<int> &src, const std::vector<int64_t> &st, const std::vector<int> &mid,
                            StepPlan::Pack &pk) {
                std::vector<int> order = s.g_batch;
                order.insert(order.end(), mid.begin(), mid.end());
                order.insert(order.end(), s.g_k.begin(), s.g_k.end());
                std::vector<int64_t> so, zero(order.size(), 0);
                for (int l : order) so.push_back(stride_in(src, st, l));
                group_tables(n, order, so, zero, P.tables, pk.n_ohi, pk.n_olo, pk.t_ohi, pk.t_olo);
                int64_t a, b;
                group_tables(n, {}, {}, {}, P.tables, a, b, pk.t_one, pk.t_one);
                pk.n = pk.n_ohi * pk.n_olo;
                pk.identity = false;
            };
            pack(s.a_labels, sta, s.g_m, s.pack_a);
            pack(s.b_labels, stb, s.g_n, s.pack_b);
            auto in_order = [&](int v, const std::vector<int> &mid) {
                if (P.values[v].input) return false;
                const StepPlan &prod = P.steps[P.values[v].producer];
                if (prod.mfma || prod.final_step || (prod.absorbed && n.compute == HTN_BF16)) return false;
                std::vector<int> o = s.g_batch;
                o.insert(o.end(), mid.begin(), mid.end());
                o.insert(o.end(), s.g_k.begin(), s.g_k.end());
                return P.values[v].labels == o;
            };
            s.pack_a.identity = in_order(s.a, s.g_m);
            s.pack_b.identity = in_order(s.b, s.g_n);
            if (n.compute == HTN_BF16) {
                if (s.pack_a.identity) P.steps[P.values[s.a].producer].out_bf16 = true;
                if (s.pack_b.identity) P.steps[P.values[s.b].producer].out_bf16 = true;
            }
        }
        s.n_out = s.n_ohi * s.n_olo;
        s.n_sum = s.n_shi * s.n_slo;
        // fused kernel: lanes per output (the whole-workgroup mode needs the
        // step to own the workgroup: it synchronises all of it)
        const int fth = 64 * s.f_nw;
        if (s.n_out >= fth) {
            s.r_fused = 1;
        } else if (s.n_out <= 2 && s.n_sum >= 512 && fth > 64 && fth == n.fused_threads) {
            s.r_fused = fth;  // whole block per output
        } else {
            int r = std::min<int64_t>(64, pow2floor(fth / s.n_out));
            r = std::min(r, pow2ceil(s.n_sum));
            s.r_fused = std::max(1, r);
        }
        // per-step kernel: enough threads to fill the chip
        int rg = 1;
        while (rg < 64 && s.n_out * rg < 131072 && (int64_t)rg * 4 <= s.n_sum) rg *= 2;
        s.r_global = rg;
        // few outputs with long sums: split each sum over several lane
        // groups (at least 32 terms per lane) until ~2^16 lanes run
        int64_t sp = 1;
        const int64_t lanes = s.n_out * rg;
        if (lanes < 65536 && s.n_sum >= 64 * (int64_t)rg) {
            sp = std::min<int64_t>((65536 + lanes - 1) / lanes, s.n_sum / (32 * (int64_t)rg));
            sp = std::max<int64_t>(1, std::min<int64_t>(sp, 4096));
        }
        s.split_global = (int)sp;
    }

    // Loads of inputs with folded coefficient tensors, in first-use order.
    std::vector<int> load_of(P.values.size(), -1);
    auto scale_tables = [&](const Value &v, LoadPlan &lp) {
        auto stv = strides_of(n, v.labels);
        for (int sc : v.scales) {
            auto sts = strides_of(n, n.labels[sc]);
            std::vector<int64_t> sa, zero(v.labels.size(), 0);
            for (int l : v.labels) sa.push_back(stride_in(n.labels[sc], sts, l));
            ScaleRef r;
            r.tensor = sc;
            int64_t n_hi;
            group_tables(n, v.labels, sa, zero, P.tables, n_hi, r.n_lo, r.t_hi, r.t_lo);
            lp.scales.push_back(r);
        }
    };
    for (int k : P.kernel_steps) {
        const StepPlan &s = P.steps[k];
        for (int id : {s.a, s.b}) {
            if (id < 0 || !P.values[id].input || load_of[id] >= 0) continue;
            LoadPlan lp;
            lp.value = id;
            lp.base = P.values[id].base;
            lp.size = P.values[id].size;
            scale_tables(P.values[id], lp);
            const auto &vl = P.values[id].labels;
            const auto &bl = n.labels[lp.base];
            if (vl != bl) {
                auto stb = strides_of(n, bl);
                std::vector<int64_t> sa, zero(vl.size(), 0);
                for (int l : vl) sa.push_back(stride_in(bl, stb, l));
                int64_t n_hi;
                group_tables(n, vl, sa, zero, P.tables, n_hi, lp.src_nlo, lp.src_thi, lp.src_tlo);
            }
            load_of[id] = (int)P.loads.size();
            P.loads.push_back(lp);
        }
    }

    // Fold chains for the per-step executor: a step contracting a large
    // value X (>= kFoldMinSize elements) with a small input matrix M (read
    // raw from its original tensor, so M may carry no folded scales)
    // over one label l of X, M's other label l' taking l's place, is a
    // fold; a fold whose X is the result of another fold continues that
    // one's chain.  A chain runs as one launch at its first step (its
    // intermediate results are never stored), so that each large tensor is
    // read and written once instead of once per matrix.
    P.chains.clear();
    {
        constexpr int64_t kFoldMinSize = 65536, kFoldMaxMatrix = 4096, kFoldMaxExtent = 64;
        auto fold_big = [&](const StepPlan &s) -> int {  // X's SSA id, or -1
            if (s.mfma || s.b < 0 || s.final_step || s.split_global > 1 || s.sum_labels.size() != 1) return -1;
            for (int pick = 0; pick < 2; ++pick) {
                const int m = pick ? s.a : s.b, x = pick ? s.b : s.a;
                const Value &M = P.values[m], &X = P.values[x];
                if (!M.input || !M.scales.empty() || M.labels.size() != 2 ||
                    M.size > kFoldMaxMatrix || X.size < kFoldMinSize)
                    continue;
                const int l = s.sum_labels[0];
                const int lp = M.labels[0] == l ? M.labels[1] : (M.labels[1] == l ? M.labels[0] : -1);
                if (lp < 0 || !contains(X.labels, l) || contains(X.labels, lp)) continue;
                if (n.dims[l] > kFoldMaxExtent || n.dims[lp] > kFoldMaxExtent) continue;
                std::vector<int> want;
                for (int y : X.labels) want.push_back(y == l ? lp : y);
                std::vector<int> got = s.c_labels;
                std::sort(want.begin(), want.end());
                std::sort(got.begin(), got.end());
                if (want == got) return x;
            }
            return -1;
        };
        std::vector<int> big(P.steps.size(), -1);
        for (int k : P.kernel_steps) big[k] = fold_big(P.steps[k]);
        for (int k : P.kernel_steps) {
            if (big[k] < 0) continue;
            const int pr = P.values[big[k]].producer;
            if (!P.values[big[k]].input && pr >= 0 && big[pr] >= 0 && P.steps[pr].chain >= 0) {
                StepPlan &s = P.steps[k];
                s.chain = P.steps[pr].chain;
                s.chain_pos = (int)P.chains[s.chain].size();
                P.chains[s.chain].push_back(k);
            } else {
                P.steps[k].chain = (int)P.chains.size();
                P.steps[k].chain_pos = 0;
                P.chains.push_back({k});
            }
        }
        // chains the fold kernel cannot take run step by step
        std::vector<std::vector<int>> kept;
        for (auto &ch : P.chains) {
            const bool ok = fold_layout(n, P, ch).ok;
            for (int k : ch) {
                P.steps[k].chain = ok ? (int)kept.size() : -1;
                if (!ok) P.steps[k].chain_pos = -1;
            }
            if (ok) kept.push_back(ch);
        }
        P.chains = std::move(kept);
        // groups of chains launched together (Plan::chain_lead): a chain
        // whose large tensor is a network input joins the open group when
        // every step since the group's first is a step of its chains
        P.chain_x_raw.assign(P.chains.size(), 0);
        for (size_t c = 0; c < P.chains.size(); ++c) P.chain_x_raw[c] = fold_layout(n, P, P.chains[c]).x_raw ? 1 : 0;
        P.chain_lead.assign(P.chains.size(), -1);
        int open = -1;
        for (int k : P.kernel_steps) {
            const StepPlan &s = P.steps[k];
            if (s.chain >= 0 && s.chain_pos > 0 && open >= 0 && P.chain_lead[s.chain] == open) continue;
            if (s.chain >= 0 && s.chain_pos == 0) {
                const int x = P.values[s.a].size >= P.values[s.b].size ? s.a : s.b;
                if (open >= 0 && P.values[x].input) {
                    P.chain_lead[s.chain] = open;
                } else {
                    P.chain_lead[s.chain] = s.chain;
                    open = s.chain;
                }
                continue;
            }
            open = -1;
        }
    }

    // Per-step executor workspace: scaled inputs are written up front by
    // one launch; each kernel step then allocates its result and releases
    // its operands.
    {
        const int64_t es = dtype_size(inter_dtype(n.compute));
        FirstFit ff;
        P.ws_off.assign(P.values.size(), -1);
        // (inputs a fold chain reads in place get no copy here: its large
        // tensor when unscaled, and its matrices, always read raw; the
        // queue and the fused kernel keep their own copies)
        std::vector<char> in_place(P.values.size(), 0);
        for (size_t c = 0; c < P.chains.size(); ++c) {
            const StepPlan &h = P.steps[P.chains[c][0]];
            int prev = P.values[h.a].size >= P.values[h.b].size ? h.a : h.b;
            if (P.chain_x_raw[c]) in_place[prev] = 1;
            for (int k : P.chains[c]) {
                const StepPlan &s = P.steps[k];
                in_place[s.a == prev ? s.b : s.a] = 1;  // the matrix (an input)
                prev = s.c;
            }
        }
        for (auto &lp : P.loads)
            if (lp.needs_copy() && !in_place[lp.value]) P.ws_off[lp.value] = ff.alloc(lp.size * es, 256);
        const int64_t pes = n.compute == HTN_BF16 ? 2 : es;  // packed operand element size
        for (int k : P.kernel_steps) {
            StepPlan &s = P.steps[k];
            if (s.chain >= 0) {
                // a group of fold chains writes the last result of each
                // chain at the group's first step (every result allocated
                // before any operand of the group is released: the chains
                // run side by side); their other results are never stored
                if (s.chain_pos == 0 && P.chain_lead[s.chain] == s.chain) {
                    std::vector<int> group;
                    for (int c = 0; c < (int)P.chains.size(); ++c)
                        if (P.chain_lead[c] == s.chain) group.push_back(c);
                    for (int c : group) {
                        const StepPlan &last = P.steps[P.chains[c].back()];
                        P.ws_off[last.c] = ff.alloc(P.values[last.c].size * es, 256);
                    }
                    for (int c : group) {
                        const StepPlan &h = P.steps[P.chains[c][0]];
                        for (int id : {h.a, h.b})
                            if (id >= 0 && P.ws_off[id] >= 0) ff.release(P.ws_off[id]);
                    }
                } else if (s.chain_pos > 0) {
                    for (int id : {s.a, s.b})
                        if (id >= 0 && P.ws_off[id] >= 0 && P.values[id].input) ff.release(P.ws_off[id]);
                }
                continue;
            }
            if (!s.final_step) P.ws_off[s.c] = ff.alloc(P.values[s.c].size * es, 256);
            if (s.mfma) {
                s.ws_pa = s.pack_a.identity ? -1 : ff.alloc(s.pack_a.n * pes, 256);
                s.ws_pb = s.pack_b.identity ? -1 : ff.alloc(s.pack_b.n * pes, 256);
                // too few 128x128 output tiles to fill the chip: split K
                // (ranges of >= 128) into parallel partial products
                const int64_t tiles = ((s.gm + 127) / 128) * ((s.gn + 127) / 128) * s.gb;
                int64_t ks = 1;
                if (tiles < 256 && s.gk >= 256) {
                    ks = std::min<int64_t>((512 + tiles - 1) / tiles, s.gk / 128);
                    ks = std::min<int64_t>(ks, (int64_t(256) << 20) / std::max<int64_t>(1, s.gb * s.gm * s.gn * 8));
                    ks = std::max<int64_t>(1, ks);
                }
                s.ksplit = (int)ks;
                if (ks > 1) {
                    s.ws_kpart = ff.alloc(ks * s.gb * s.gm * s.gn * 8, 256);
                    ff.release(s.ws_kpart);
                }
                ff.release(s.ws_pa);
                ff.release(s.ws_pb);
            } else if (s.split_global > 1) {
                s.ws_part = ff.alloc(s.n_out * s.split_global * 16, 256);
                ff.release(s.ws_part);
            }
            for (int id : {s.a, s.b})
                if (id >= 0 && P.ws_off[id] >= 0) ff.release(P.ws_off[id]);
        }
        P.ws_bytes = std::max<int64_t>(ff.peak, 256);
    }

    // Fused executor.  Inputs are first materialised (permuted into their
    // planned layout, coefficient tensors applied) by one prep launch into
    // the front of the network's workspace; the fused kernel then only moves
    // contiguous 16-byte chunks (OP_COPY) and computes.  Device image
    // (int32 words): [0] program words, [1] LDS bytes, [2] op count,
    // [3] LDS word offset of table slot 0, [4] words per slot, [5] LDS byte
    // offset of the 256-byte reduction scratch, [6] image word offset of the
    // step tables, [7] image word offset of the load descriptors; ops from
    // word 8; then step tables; then load descriptors (digit form, read by
    // the prep kernel).  Phase 0 copies the tables and LDS-resident operands
    // of step 0; phase k runs step k and copies those of step k+1 (the
    // kernel issues these copies before the step's arithmetic); a barrier
    // ends each phase.  Value locations: >= 0 LDS element offset; <= -2
    // workspace element offset -loc-2; -1 the network's output / none.
    {
        const int64_t es = dtype_size(inter_dtype(n.compute));
        const auto &ks = P.kernel_steps;
        // step tables: one block per phase (the concatenated tables of its
        // table-driven steps, each padded to 16 bytes); a step's table
        // offsets (rel) are relative to its phase's block
        const auto &phs = P.fused_phases;
        std::vector<int32_t> gtab;
        std::vector<int64_t> tab_off(phs.size()), tab_words(phs.size());
        std::vector<std::vector<int32_t>> rel(ks.size());
        int64_t slot_words = 4;
        for (size_t ph = 0; ph < phs.size(); ++ph) {
            tab_off[ph] = (int64_t)gtab.size();
            for (int q : phs[ph]) {
                const StepPlan &s = P.steps[ks[q]];
                auto put_pairs = [&](int64_t pair_off, int64_t count) {
                    if ((gtab.size() - tab_off[ph]) % 2) gtab.push_back(0);
                    const int32_t o = (int32_t)((gtab.size() - tab_off[ph]) / 2);
                    for (int64_t e = 0; e < 2 * count; ++e) gtab.push_back(P.tables[2 * pair_off + e]);
                    return o;
                };
                if (s.tile) {
                    rel[q] = {0, 0, 0, 0};  // offsets computed from digits: no tables
                } else {
                    rel[q] = {put_pairs(s.t_ohi, s.n_ohi), put_pairs(s.t_olo, s.n_olo), put_pairs(s.t_shi, s.n_shi),
                              put_pairs(s.t_slo, s.n_slo)};
                }
                while (gtab.size() % 4) gtab.push_back(0);
            }
            tab_words[ph] = (int64_t)gtab.size() - tab_off[ph];
            slot_words = std::max(slot_words, tab_words[ph]);
        }
        slot_words = (slot_words + 3) / 4 * 4;

        // load descriptors (digit form) for the prep kernel
        bool loads_fit = true;
        std::vector<int32_t> ldesc;
        std::vector<int64_t> ld_off(P.loads.size(), -1);
        P.fused_in_ptr_slots.clear();
        for (size_t li = 0; li < P.loads.size(); ++li) {
            const LoadPlan &lp = P.loads[li];
            const auto &vl = P.values[lp.value].labels;
            const auto &bl = n.labels[lp.base];
            auto stb = strides_of(n, bl);
            const int rk = (int)vl.size(), ns = (int)lp.scales.size();
            if (rk > 16 || ns > kMaxScales) loads_fit = false;
            ld_off[li] = (int64_t)ldesc.size();
            // [base ptr (2), dst element offset in workspace (2), size, rank, ns, scale ptrs (2 each),
            //  per label: extent, magic (2), source stride, scale strides]
            P.fused_in_ptr_slots.push_back({(int64_t)ldesc.size(), lp.base});
            ldesc.insert(ldesc.end(), {0, 0, 0, 0, (int32_t)lp.size, rk, ns});
            for (size_t q = 0; q < lp.scales.size(); ++q) {
                P.fused_in_ptr_slots.push_back({(int64_t)ldesc.size(), lp.scales[q].tensor});
                ldesc.push_back(0);
                ldesc.push_back(0);
            }
            std::vector<std::vector<int64_t>> sst;
            for (auto &sc : lp.scales) sst.push_back(strides_of(n, n.labels[sc.tensor]));
            if (lp.size >= (int64_t(1) << 24)) loads_fit = false;  // magic division range
            for (int k = 0; k < rk; ++k) {
                const int l = vl[k];
                if (n.dims[l] >= 65536) loads_fit = false;
                // floor(e / d) = (e * magic) >> 40 for e < 2^24, d < 2^16
                const uint64_t magic = ((uint64_t(1) << 40) + (uint64_t)n.dims[l] - 1) / (uint64_t)n.dims[l];
                ldesc.push_back((int32_t)n.dims[l]);
                ldesc.push_back((int32_t)(uint32_t)(magic & 0xffffffffu));
                ldesc.push_back((int32_t)(uint32_t)(magic >> 32));
                ldesc.push_back((int32_t)stride_in(bl, stb, l));
                for (int q = 0; q < ns; ++q)
                    ldesc.push_back((int32_t)stride_in(n.labels[lp.scales[q].tensor], sst[q], l));
            }
        }

        // workspace: materialised inputs first, spill scratch after
        FirstFit glb_ff;
        std::vector<int64_t> in_off(P.values.size(), -1);
        for (size_t li = 0; li < P.loads.size(); ++li) {
            const LoadPlan &lp = P.loads[li];
            in_off[lp.value] = glb_ff.alloc(lp.size, 32);
            ldesc[ld_off[li] + 2] = (int32_t)(in_off[lp.value] & 0xffffffff);
            ldesc[ld_off[li] + 3] = (int32_t)(in_off[lp.value] >> 32);
        }
        const int64_t inputs_end = glb_ff.peak;

        struct OpRec {
            int kind;
            int step = -1, value = -1, q = -1;
            std::vector<int32_t> w;
        };
        std::vector<OpRec> seq;
        auto copies_of_phase = [&](size_t ph) {
            OpRec t;
            t.kind = OP_COPY;
            t.q = (int)ph;
            // [kind 0: image words, src chunk, chunks, dst chunk]
            t.w = {OP_COPY, 0, (int32_t)(tab_off[ph] / 4), (int32_t)(tab_words[ph] / 4), 0};
            if (tab_words[ph] > 0) seq.push_back(t);
            for (int q : phs[ph]) {
                const StepPlan &s = P.steps[ks[q]];
                for (int id : {s.a, s.b})
                    if (id >= 0 && P.values[id].input) {
                        OpRec r;
                        r.kind = OP_COPY;
                        r.value = id;
                        r.w = {OP_COPY, 1, 0, 0, 0};
                        seq.push_back(r);
                    }
            }
        };
        if (!phs.empty()) copies_of_phase(0);
        seq.push_back(OpRec{OP_SYNC, -1, -1, -1, {OP_SYNC}});
        for (size_t ph = 0; ph < phs.size(); ++ph) {
            for (int q : phs[ph]) {
                const StepPlan &s = P.steps[ks[q]];
                OpRec r;
                r.step = ks[q];
                r.q = q;
                const int32_t slot = (int32_t)(ph % 2);
                if (s.tile) {
                    r.kind = OP_TSTEP;
                    // [a, b, c, M, N, K, TM, TN, GX, final, nm, nn, w0, nw, digits of M (4 each), digits of N]
                    r.w = {OP_TSTEP, 0, 0, 0, (int32_t)s.tM, (int32_t)s.tN, (int32_t)s.tK, s.TM, s.TN, s.GX,
                           s.final_step ? 1 : 0, (int32_t)(s.c_digits_m.size() / 4),
                           (int32_t)(s.c_digits_n.size() / 4), s.f_w0, s.f_nw};
                    r.w.insert(r.w.end(), s.c_digits_m.begin(), s.c_digits_m.end());
                    r.w.insert(r.w.end(), s.c_digits_n.begin(), s.c_digits_n.end());
                } else {
                    r.kind = OP_STEP;
                    // [a, b, c, n_ohi, n_olo, n_shi, n_slo, t_ohi, t_olo, t_shi, t_slo, R, final, slot, w0, nw]
                    r.w = {OP_STEP, 0, 0, 0, (int32_t)s.n_ohi, (int32_t)s.n_olo, (int32_t)s.n_shi, (int32_t)s.n_slo,
                           rel[q][0], rel[q][1], rel[q][2], rel[q][3], s.r_fused, s.final_step ? 1 : 0, slot,
                           s.f_w0, s.f_nw};
                }
                seq.push_back(r);
            }
            if (ph + 1 < phs.size()) copies_of_phase(ph + 1);
            seq.push_back(OpRec{OP_SYNC, -1, -1, -1, {OP_SYNC}});
        }
        int64_t prog_words = 8 + 1;
        for (auto &r : seq) prog_words += (int64_t)r.w.size();
        prog_words = (prog_words + 3) / 4 * 4;
        const int64_t slot0 = prog_words;
        const int64_t scratch_byte = (slot0 + 2 * slot_words) * 4;
        const int64_t values_byte = scratch_byte + 256;
        const int64_t vbase = (values_byte + es - 1) / es;
        const int64_t budget = std::max<int64_t>(0, n.fused_lds_budget / es - vbase);
        const int64_t ealign = 16 / es;  // 16-byte aligned LDS values

        FirstFit lds_ff;
        glb_ff.peak = inputs_end;
        std::vector<int64_t> loc(P.values.size(), INT64_MIN);
        auto place = [&](int64_t size) -> int64_t {
            const int64_t old_peak = lds_ff.peak;
            const int64_t off = lds_ff.alloc((size + ealign - 1) / ealign * ealign, 16);
            if (off + size <= budget) return vbase + off;
            lds_ff.release(off);
            lds_ff.peak = old_peak;
            return -1;
        };
        auto place_or_spill = [&](int64_t size) -> int64_t {
            const int64_t l = place(size);
            if (l >= 0) return l;
            return -(glb_ff.alloc(size, 32) + 2);
        };
        auto unplace = [&](int64_t l) {
            if (l >= 0)
                lds_ff.release(l - vbase);
            else if (l <= -2 && -l - 2 >= inputs_end)
                glb_ff.release(-l - 2);
        };
        // keep spill scratch above the inputs area
        glb_ff.used[0] = inputs_end;
        int n_ops = 0;
        std::vector<int> pending;
        int phase = 0, last_step = -1;
        bool lds_only = true;
        for (auto &r : seq) {
            if (r.kind == OP_COPY && r.value >= 0) {
                const int64_t sz = P.values[r.value].size;
                const int64_t l = place(sz);
                if (l >= 0) {
                    loc[r.value] = l;
                    const int64_t bytes = (sz * es + 15) / 16 * 16;
                    r.w[2] = (int32_t)(in_off[r.value] * es / 16);
                    r.w[3] = (int32_t)(bytes / 16);
                    r.w[4] = (int32_t)(l * es / 16);
                } else {
                    loc[r.value] = -(in_off[r.value] + 2);  // read in place
                    r.w[3] = 0;
                }
                if (last_step >= 0) P.steps[last_step].f_copy_chunks += r.w[3];
            } else if (r.kind == OP_COPY) {
                r.w[4] = (int32_t)((slot0 + (r.q % 2) * slot_words) / 4);
                if (last_step >= 0) P.steps[last_step].f_copy_chunks += r.w[3];
            } else if (r.kind == OP_STEP || r.kind == OP_TSTEP) {
                StepPlan &s = P.steps[r.step];
                int64_t cl = -1;
                if (!s.final_step) cl = loc[s.c] = place_or_spill(P.values[s.c].size);
                r.w[1] = (int32_t)loc[s.a];
                r.w[2] = s.b >= 0 ? (int32_t)loc[s.b] : -1;
                r.w[3] = (int32_t)cl;
                pending.push_back(s.a);
                pending.push_back(s.b);
                if (loc[s.a] < 0 || (s.b >= 0 && loc[s.b] < 0) || (!s.final_step && cl < 0)) lds_only = false;
                s.f_phase = phase;
                s.f_spill = (loc[s.a] < 0 ? 1 : 0) | (s.b >= 0 && loc[s.b] < 0 ? 2 : 0) |
                            (!s.final_step && cl < 0 ? 4 : 0);
                s.f_copy_chunks = 0;
                last_step = r.step;
            } else if (r.kind == OP_SYNC) {
                for (int id : pending)
                    if (id >= 0) unplace(loc[id]);
                pending.clear();
                ++phase;
                last_step = -1;
            }
            ++n_ops;
        }
        std::vector<int32_t> prog = {0, 0, n_ops, (int32_t)slot0, (int32_t)slot_words, (int32_t)scratch_byte, 0, 0};
        // within a phase the copies (which land after its steps, into
        // regions no step of the phase touches) come first, so the kernel
        // issues their loads before decoding the steps
        {
            std::vector<int32_t> steps_of_phase;
            for (auto &r : seq) {
                if (r.kind == OP_COPY && r.w[3] == 0) continue;
                if (r.kind == OP_STEP || r.kind == OP_TSTEP) {
                    steps_of_phase.insert(steps_of_phase.end(), r.w.begin(), r.w.end());
                    continue;
                }
                if (r.kind == OP_SYNC) {
                    prog.insert(prog.end(), steps_of_phase.begin(), steps_of_phase.end());
                    steps_of_phase.clear();
                }
                prog.insert(prog.end(), r.w.begin(), r.w.end());
            }
            prog.insert(prog.end(), steps_of_phase.begin(), steps_of_phase.end());
        }
        prog.push_back(OP_END);
        prog.resize(prog_words, 0);
        prog[0] = (int32_t)prog_words;
        prog[6] = (int32_t)prog.size();
        prog.insert(prog.end(), gtab.begin(), gtab.end());
        prog[7] = (int32_t)prog.size();
        for (auto &ps : P.fused_in_ptr_slots) ps.first += prog[7];
        for (size_t li = 0; li < P.loads.size(); ++li) P.loads[li].desc_word = prog[7] + ld_off[li];
        prog.insert(prog.end(), ldesc.begin(), ldesc.end());
        P.fused_lds_bytes = (vbase + lds_ff.peak) * es;
        // 16-byte chunk copies may read up to 15 bytes past a value's end
        P.fused_scratch_bytes = (glb_ff.peak * es + 255) / 256 * 256;
        P.fused_input_bytes = inputs_end * es;
        prog[1] = (int32_t)P.fused_lds_bytes;
        P.program = std::move(prog);
        P.ptr_slots = P.fused_in_ptr_slots;
        P.fused_pure = glb_ff.peak <= inputs_end;
        P.fused_lds_only = lds_only;
        bool has_mfma = false;
        for (const auto &st : P.steps) has_mfma |= st.mfma != 0;
        // The fused kernel needs its program and table slots in LDS.  Dense
        // matrix-core steps run best on the whole GPU: AUTO then uses the
        // per-step executor.
        P.fused_possible = loads_fit && values_byte <= n.fused_lds_budget;
        P.fused_ok = P.fused_possible && !has_mfma && (P.fused_pure || P.mults <= n.fused_max_mults);
        // In a batch, throughput favours the fused kernel unless the network
        // is large enough to occupy the GPU by itself.
        P.fused_batch_ok = P.fused_possible && (P.fused_ok || P.mults <= n.batch_fused_max_mults);
    }
    if (P.tables.empty()) P.tables.assign(2, 0);
    n.plan = std::move(P);
    n.plan_version++;
}

// ------------------------------------------------------------------ json

static void json_ints(std::ostringstream &o, const std::vector<int> &v) {
    o << "[";
    for (size_t k = 0; k < v.size(); ++k) o << (k ? "," : "") << v[k];
    o << "]";
}

double path_peak(const Net &n, const std::vector<int64_t> &dims) {
    const int N = n.n_t;
    std::vector<int> ref(dims.size(), 0);
    std::vector<char> is_out(dims.size(), 0);
    for (int l : n.out_labels) is_out[l] = 1;
    std::vector<std::vector<int>> lab(N + n.path.size());
    for (int i = 0; i < N; ++i) {
        lab[i] = n.labels[i];
        std::sort(lab[i].begin(), lab[i].end());
        for (int l : lab[i]) ref[l]++;
    }
    // inputs and inputs scaled by absorbed ones are loads, not intermediates
    std::vector<char> input(N + n.path.size(), 0);
    for (int i = 0; i < N; ++i) input[i] = 1;
    double peak = 0.0;
    for (size_t t = 0; t < n.path.size(); ++t) {
        const int i = n.path[t].first, j = n.path[t].second;
        const auto &a = lab[i], &b = lab[j];
        std::vector<int> u = sorted_union(a, b), kept;
        for (int l : a) ref[l]--;
        for (int l : b) ref[l]--;
        double sz = 1.0;
        bool sums = false;
        for (int l : u)
            if (is_out[l] || ref[l] > 0) {
                kept.push_back(l);
                sz *= (double)dims[l];
            } else if (dims[l] > 1) {
                sums = true;
            }
        for (int l : kept) ref[l]++;
        const bool absorption = input[i] && input[j] && !sums &&
                                (std::includes(a.begin(), a.end(), b.begin(), b.end()) ||
                                 std::includes(b.begin(), b.end(), a.begin(), a.end()));
        input[N + t] = absorption;
        if (!absorption) peak = std::max(peak, sz);
        lab[N + t] = kept;
    }
    return peak;
}

std::vector<int64_t> sliced_dims(const Net &n) {
    std::vector<int64_t> d = n.dims;
    for (int l : n.sliced) d[l] = 1;
    return d;
}

// Slicing (for a path whose largest intermediate exceeds the cap): fix
// summed labels one at a time, each time the label that leaves the smallest
// largest intermediate (fewer slices, then the lower id, on ties), until
// the path fits.  Every slice is the network with those labels fixed; the
// slices' results sum to the network's value.
void plan_net(Net &n) {
    if (!n.slice_mode || path_peak(n, n.dims) <= (double)n.max_intermediate) {
        build_plan(n);
        n.sliced.clear();
        n.n_slices = 1;
        return;
    }
    constexpr int64_t kMaxSlices = 65536;
    std::vector<char> is_out(n.dims.size(), 0), used(n.dims.size(), 0);
    for (int l : n.out_labels) is_out[l] = 1;
    for (const auto &ls : n.labels)
        for (int l : ls) used[l] = 1;
    std::vector<int64_t> dims = n.dims;
    std::vector<int> sliced;
    int64_t slices = 1;
    double peak = path_peak(n, dims);
    while (peak > (double)n.max_intermediate) {
        int best = -1;
        double best_peak = 0.0;
        for (int l = 0; l < (int)dims.size(); ++l) {
            if (is_out[l] || !used[l] || dims[l] <= 1) continue;
            if (slices * dims[l] > kMaxSlices) continue;
            const int64_t keep = dims[l];
            dims[l] = 1;
            const double pk = path_peak(n, dims);
            dims[l] = keep;
            if (best < 0 || pk < best_peak || (pk == best_peak && dims[l] < dims[best])) {
                best = l;
                best_peak = pk;
            }
        }
        if (best < 0 || best_peak >= peak)
            throw make_err(HTN_E_OOM, "no slicing of at most " + std::to_string(kMaxSlices) +
                                          " slices brings the largest intermediate under the cap " +
                                          std::to_string(n.max_intermediate));
        slices *= dims[best];
        dims[best] = 1;
        sliced.push_back(best);
        peak = best_peak;
    }
    Net t = structure_copy(n);
    t.dims = dims;
    for (int i = 0; i < t.n_t; ++i) {
        int64_t sz = 1;
        for (int l : t.labels[i]) sz *= t.dims[l];
        t.sizes[i] = sz;
    }
    t.path = n.path;
    build_plan(t);
    n.plan = std::move(t.plan);
    n.sliced = sliced;
    n.n_slices = slices;
    n.plan_version++;
}

// Fold chains with their kernel layouts (see FoldLayout), as JSON.
static std::string chains_json(const Net &n) {
    std::ostringstream o;
    auto arr = [&](const char *name, const auto &v) {
        o << "\"" << name << "\":[";
        for (size_t k = 0; k < v.size(); ++k) o << (k ? "," : "") << v[k];
        o << "]";
    };
    o << "[";
    for (size_t c = 0; c < n.plan.chains.size(); ++c) {
        const FoldLayout F = fold_layout(n, n.plan, n.plan.chains[c]);
        o << (c ? "," : "") << "{";
        arr("steps", n.plan.chains[c]);
        o << ",\"lead\":" << n.plan.chain_lead[c] << ",\"x_raw\":" << (F.x_raw ? 1 : 0) << ",\"ws_x\":" << n.plan.ws_off[F.x] << ",\"ws_y\":" << n.plan.ws_off[F.y];
        o << ",\"x\":" << F.x << ",\"y\":" << F.y << ",\"tf\":" << F.tf << ",\"d_max\":" << F.d_max
          << ",\"n_outer\":" << F.n_outer << ",";
        arr("ext0", F.ext0);
        o << ",";
        arr("ext1", F.ext1);
        o << ",";
        arr("s_src", F.s_src);
        o << ",";
        arr("s_dst", F.s_dst);
        o << ",";
        arr("fold_ax", F.fold_ax);
        o << ",";
        arr("fold_ext", F.fold_ext);
        o << ",";
        arr("m_tensor", F.m_tensor);
        o << ",";
        arr("m_in", F.m_in);
        o << ",";
        arr("m_out", F.m_out);
        o << ",";
        arr("o_ext", F.o_ext);
        o << ",";
        arr("o_src", F.o_src);
        o << ",";
        arr("o_dst", F.o_dst);
        o << "}";
    }
    o << "]";
    return o.str();
}

std::string plan_json(const Net &n) {
    const Plan &P = n.plan;
    std::ostringstream o;
    o.precision(17);
    o << "{\"n_tensors\":" << n.n_t << ",\"mults\":" << P.mults << ",\"peak\":" << P.peak
      << ",\"fused_possible\":" << (P.fused_possible ? "true" : "false")
      << ",\"elem_bytes\":" << dtype_size(inter_dtype(n.compute))
      << ",\"n_absorbed\":" << P.n_absorbed << ",\"fused_ok\":" << (P.fused_ok ? "true" : "false")
      << ",\"fused_batch_ok\":" << (P.fused_batch_ok ? "true" : "false")
      << ",\"fused_pure\":" << (P.fused_pure ? "true" : "false")
      << ",\"fused_lds_only\":" << (P.fused_lds_only ? "true" : "false") << ",\"fused_lds_bytes\":" << P.fused_lds_bytes
      << ",\"fused_scratch_bytes\":" << P.fused_scratch_bytes << ",\"ws_bytes\":" << P.ws_bytes
      << ",\"final_value\":" << P.final_value << ",\"n_table_entries\":" << P.tables.size() / 2
      << ",\"chains\":" << chains_json(n)
      << ",\"steps\":[";
    for (size_t k = 0; k < P.steps.size(); ++k) {
        const StepPlan &s = P.steps[k];
        o << (k ? "," : "") << "{\"a\":" << s.a << ",\"b\":" << s.b << ",\"c\":" << s.c << ",\"a_labels\":";
        json_ints(o, s.a_labels);
        o << ",\"b_labels\":";
        json_ints(o, s.b_labels);
        o << ",\"c_labels\":";
        json_ints(o, s.c_labels);
        o << ",\"sum_labels\":";
        json_ints(o, s.sum_labels);
        o << ",\"mults\":" << s.mults << ",\"absorbed\":" << (s.absorbed ? "true" : "false")
          << ",\"final\":" << (s.final_step ? "true" : "false") << ",\"synthetic\":" << (s.synthetic ? "true" : "false")
          << ",\"n_out\":" << s.n_out << ",\"n_sum\":" << s.n_sum << ",\"r_fused\":" << s.r_fused
          << ",\"r_global\":" << s.r_global << ",\"split\":" << s.split_global << ",\"ksplit\":" << s.ksplit << ",\"chain\":" << s.chain << ",\"chain_pos\":" << s.chain_pos << ",\"f_phase\":" << s.f_phase << ",\"geom\":[" << s.n_ohi << "," << s.n_olo << "," << s.n_shi << ","
          << s.n_slo << "," << s.t_ohi << "," << s.t_olo << "," << s.t_shi << "," << s.t_slo << "],\"pack_a\":["
          << s.pack_a.n_ohi << "," << s.pack_a.n_olo << "," << s.pack_a.t_ohi << "," << s.pack_a.t_olo << "],\"pack_b\":["
          << s.pack_b.n_ohi << "," << s.pack_b.n_olo << "," << s.pack_b.t_ohi << "," << s.pack_b.t_olo
          << "],\"pack_id\":[" << (s.pack_a.identity ? 1 : 0) << "," << (s.pack_b.identity ? 1 : 0)
          << "],\"t_cm\":" << s.t_cm << ",\"t_cn\":" << s.t_cn << ",\"mfma\":" << s.mfma << ",\"gemm\":[" << s.gb << "," << s.gm
          << "," << s.gn << "," << s.gk << "],\"tile\":" << s.tile << ",\"tmnk\":[" << s.tM << "," << s.tN << ","
          << s.tK << "],\"tcfg\":[" << s.TM << "," << s.TN << "," << s.GX << "]}";
    }
    o << "],\"values\":[";
    for (size_t v = 0; v < P.values.size(); ++v) {
        o << (v ? "," : "") << "{\"labels\":";
        json_ints(o, P.values[v].labels);
        o << ",\"input\":" << (P.values[v].input ? "true" : "false") << ",\"base\":" << P.values[v].base << "}";
    }
    o << "],\"program\":";
    {
        // pointer slots hold the tensor id in the low word here
        std::vector<int> pw(P.program.begin(), P.program.end());
        for (auto &ps : P.ptr_slots) pw[ps.first] = ps.second;
        json_ints(o, pw);
    }
    o << ",\"loads\":[";
    for (size_t k = 0; k < P.loads.size(); ++k) {
        const LoadPlan &lp = P.loads[k];
        o << (k ? "," : "") << "{\"value\":" << lp.value << ",\"base\":" << lp.base << ",\"size\":" << lp.size
          << ",\"src\":[" << lp.src_thi << "," << lp.src_tlo << "," << lp.src_nlo << "],\"scales\":[";
        for (size_t q = 0; q < lp.scales.size(); ++q)
            o << (q ? "," : "") << "[" << lp.scales[q].tensor << "," << lp.scales[q].t_hi << "," << lp.scales[q].t_lo
              << "," << lp.scales[q].n_lo << "]";
        o << "]}";
    }
    o << "]}";
    return o.str();
}

}  // namespace htn
