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

// FLOP-greedy: among live pairs that share a label, contract the one with
// the fewest multiplications (product of the extents of the union of the
// two label sets); ties: smaller result, then lower (i, j).  When no pair
// shares a label the two smallest live tensors are joined (outer product).
std::vector<std::pair<int, int>> greedy_path(const Net &n) {
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
    std::vector<std::vector<int>> holders(L);
    while (n_alive > 1) {
        for (auto &h : holders) h.clear();
        for (int i = 0; i < next; ++i)
            if (alive[i])
                for (int l : lab[i]) holders[l].push_back(i);
        bool found = false;
        double bc = 0, bs = 0;
        int bi = -1, bj = -1;
        std::vector<int> bkept;
        auto consider = [&](int i, int j, bool shared_only) {
            (void)shared_only;
            std::vector<int> u = sorted_union(lab[i], lab[j]);
            double cost = prod_dims(n, u);
            std::vector<int> kept;
            for (int l : u) {
                int r = ref[l] - (int)contains(lab[i], l) - (int)contains(lab[j], l);
                if (is_out[l] || r > 0) kept.push_back(l);
            }
            double os = prod_dims(n, kept);
            bool better = !found || cost < bc || (cost == bc && (os < bs || (os == bs && (i < bi || (i == bi && j < bj)))));
            if (better) {
                found = true;
                bc = cost;
                bs = os;
                bi = i;
                bj = j;
                bkept = kept;
            }
        };
        for (int l = 0; l < L; ++l) {
            const auto &h = holders[l];
            for (size_t x = 0; x < h.size(); ++x)
                for (size_t y = x + 1; y < h.size(); ++y) consider(std::min(h[x], h[y]), std::max(h[x], h[y]), true);
        }
        if (!found) {
            // disconnected: join the two smallest live tensors
            std::vector<std::pair<double, int>> sz;
            for (int i = 0; i < next; ++i)
                if (alive[i]) sz.push_back({prod_dims(n, lab[i]), i});
            std::sort(sz.begin(), sz.end());
            int i = std::min(sz[0].second, sz[1].second), j = std::max(sz[0].second, sz[1].second);
            consider(i, j, false);
        }
        path.push_back({bi, bj});
        for (int l : lab[bi]) ref[l]--;
        for (int l : lab[bj]) ref[l]--;
        alive[bi] = alive[bj] = 0;
        lab[next] = bkept;
        for (int l : bkept) ref[l]++;
        alive[next] = 1;
        ++next;
        --n_alive;
    }
    return path;
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

enum { OP_END = 0, OP_LOAD = 1, OP_STEP = 2, OP_SYNC = 3 };

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
        // Absorption: both operands are (possibly already scaled) inputs, one
        // label set contains the other and nothing is summed, so the result
        // is the larger input scaled entry-wise by the smaller one.
        int tgt = -1, sml = -1;
        if (A.input && B.input && sums.empty()) {
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
            };
            pack(s.a_labels, sta, s.g_m, s.pack_a);
            pack(s.b_labels, stb, s.g_n, s.pack_b);
        }
        s.n_out = s.n_ohi * s.n_olo;
        s.n_sum = s.n_shi * s.n_slo;
        // fused kernel: lanes per output
        if (s.n_out >= kBlock) {
            s.r_fused = 1;
        } else if (s.n_out <= 2 && s.n_sum >= 512) {
            s.r_fused = kBlock;  // whole block per output
        } else {
            int r = std::min<int64_t>(64, pow2floor(kBlock / s.n_out));
            r = std::min(r, pow2ceil(s.n_sum));
            s.r_fused = std::max(1, r);
        }
        // per-step kernel: enough threads to fill the chip
        int rg = 1;
        while (rg < 64 && s.n_out * rg < 131072 && (int64_t)rg * 4 <= s.n_sum) rg *= 2;
        s.r_global = rg;
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
            load_of[id] = (int)P.loads.size();
            P.loads.push_back(lp);
        }
    }

    // Per-step executor workspace: scaled inputs are written up front by
    // one launch; each kernel step then allocates its result and releases
    // its operands.
    {
        const int64_t es = dtype_size(inter_dtype(n.compute));
        FirstFit ff;
        P.ws_off.assign(P.values.size(), -1);
        for (auto &lp : P.loads)
            if (!lp.scales.empty()) P.ws_off[lp.value] = ff.alloc(lp.size * es, 256);
        const int64_t pes = n.compute == HTN_BF16 ? 2 : es;  // packed operand element size
        for (int k : P.kernel_steps) {
            StepPlan &s = P.steps[k];
            if (!s.final_step) P.ws_off[s.c] = ff.alloc(P.values[s.c].size * es, 256);
            if (s.mfma) {
                s.ws_pa = ff.alloc(s.pack_a.n * pes, 256);
                s.ws_pb = ff.alloc(s.pack_b.n * pes, 256);
                ff.release(s.ws_pa);
                ff.release(s.ws_pb);
            }
            for (int id : {s.a, s.b})
                if (id >= 0 && P.ws_off[id] >= 0) ff.release(P.ws_off[id]);
        }
        P.ws_bytes = std::max<int64_t>(ff.peak, 256);
    }

    // Fused executor program.  Phase 0 loads the operands of kernel step 0;
    // phase k runs step k and loads the inputs of step k+1; a barrier ends
    // every phase.  Offsets are in elements of the intermediate type.  A
    // value goes to LDS when it fits the budget (after a 256-byte reduction
    // scratch), otherwise to the network's global scratch.  Locations are
    // encoded as loc >= 0: LDS offset; loc <= -2: scratch offset -loc-2;
    // -1: the network's output (final step) / no operand.
    {
        const int64_t es = dtype_size(inter_dtype(n.compute));
        const int64_t scratch = 256 / es;
        const int64_t budget = std::max<int64_t>(0, n.fused_lds_budget / es - scratch);
        FirstFit lds_ff, glb_ff;
        std::vector<int64_t> loc(P.values.size(), INT64_MIN);
        auto place = [&](int64_t size) -> int64_t {
            const int64_t old_peak = lds_ff.peak;
            const int64_t off = lds_ff.alloc(size, 4);
            if (off + size <= budget) return scratch + off;
            lds_ff.release(off);
            lds_ff.peak = old_peak;
            return -(glb_ff.alloc(size, 64) + 2);
        };
        auto unplace = [&](int64_t l) {
            if (l >= 0)
                lds_ff.release(l - scratch);
            else if (l <= -2)
                glb_ff.release(-l - 2);
        };
        std::vector<int32_t> prog = {0, 0, 0};
        int n_ops = 0;
        auto emit_loads = [&](const StepPlan &s) {
            for (int id : {s.a, s.b}) {
                if (id < 0 || !P.values[id].input) continue;
                const LoadPlan &lp = P.loads[load_of[id]];
                loc[id] = place(lp.size);
                prog.push_back(OP_LOAD);
                prog.push_back(lp.base);
                prog.push_back((int32_t)loc[id]);
                prog.push_back((int32_t)lp.size);
                prog.push_back((int32_t)lp.scales.size());
                for (auto &r : lp.scales) {
                    prog.push_back(r.tensor);
                    prog.push_back((int32_t)r.t_hi);
                    prog.push_back((int32_t)r.t_lo);
                    prog.push_back((int32_t)r.n_lo);
                }
                ++n_ops;
            }
        };
        const auto &ks = P.kernel_steps;
        if (!ks.empty()) emit_loads(P.steps[ks[0]]);
        prog.push_back(OP_SYNC);
        ++n_ops;
        for (size_t q = 0; q < ks.size(); ++q) {
            const StepPlan &s = P.steps[ks[q]];
            int64_t cl = -1;
            if (!s.final_step) cl = loc[s.c] = place(P.values[s.c].size);
            prog.push_back(OP_STEP);
            prog.push_back((int32_t)loc[s.a]);
            prog.push_back(s.b >= 0 ? (int32_t)loc[s.b] : -1);
            prog.push_back((int32_t)cl);
            for (int64_t x : {s.n_ohi, s.n_olo, s.n_shi, s.n_slo, s.t_ohi, s.t_olo, s.t_shi, s.t_slo})
                prog.push_back((int32_t)x);
            prog.push_back(s.r_fused);
            prog.push_back(s.final_step ? 1 : 0);
            ++n_ops;
            if (q + 1 < ks.size()) emit_loads(P.steps[ks[q + 1]]);
            prog.push_back(OP_SYNC);
            ++n_ops;
            for (int id : {s.a, s.b})
                if (id >= 0) unplace(loc[id]);
        }
        prog.push_back(OP_END);
        prog[0] = (int32_t)prog.size();
        P.fused_lds_bytes = (scratch + lds_ff.peak) * es;
        P.fused_scratch_bytes = glb_ff.peak * es;
        prog[1] = (int32_t)P.fused_lds_bytes;
        prog[2] = n_ops;
        P.program = std::move(prog);
        P.fused_pure = P.fused_scratch_bytes == 0;
        P.fused_ok = P.fused_pure || P.mults <= n.fused_max_mults;
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

std::string plan_json(const Net &n) {
    const Plan &P = n.plan;
    std::ostringstream o;
    o.precision(17);
    o << "{\"n_tensors\":" << n.n_t << ",\"mults\":" << P.mults << ",\"peak\":" << P.peak
      << ",\"n_absorbed\":" << P.n_absorbed << ",\"fused_ok\":" << (P.fused_ok ? "true" : "false")
      << ",\"fused_pure\":" << (P.fused_pure ? "true" : "false") << ",\"fused_lds_bytes\":" << P.fused_lds_bytes
      << ",\"fused_scratch_bytes\":" << P.fused_scratch_bytes << ",\"ws_bytes\":" << P.ws_bytes
      << ",\"final_value\":" << P.final_value << ",\"n_table_entries\":" << P.tables.size() / 2
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
          << ",\"r_global\":" << s.r_global << ",\"mfma\":" << s.mfma << ",\"gemm\":[" << s.gb << "," << s.gm
          << "," << s.gn << "," << s.gk << "]}";
    }
    o << "],\"loads\":[";
    for (size_t k = 0; k < P.loads.size(); ++k) {
        const LoadPlan &lp = P.loads[k];
        o << (k ? "," : "") << "{\"value\":" << lp.value << ",\"base\":" << lp.base << ",\"size\":" << lp.size
          << ",\"scales\":[";
        for (size_t q = 0; q < lp.scales.size(); ++q) o << (q ? "," : "") << lp.scales[q].tensor;
        o << "]}";
    }
    o << "]}";
    return o.str();
}

}  // namespace htn
