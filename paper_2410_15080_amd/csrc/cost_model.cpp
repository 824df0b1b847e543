// Learned path selection: step features and candidate scoring by the MLP
// cost model.
//
// The paper picks a contraction order by minimising a FLOP objective with
// a hyper-optimised search (Sec. 4.2; Sec. 6.1, Step 3).  Here every
// candidate order (FLOP-greedy plus Boltzmann-sampled greedy orders) is
// planned, each of its kernel steps is described by a feature row, and the
// model's predicted step times are combined (a fused phase costs its slowest
// step, phases and per-step launches add up); the fastest predicted
// candidate among those within twice the fewest multiplications wins,
// FLOP-greedy on ties (or the first such candidate when FLOP-greedy itself
// lies outside that range).
#include <algorithm>
#include <cmath>
#include <limits>

#include "htn_core.hpp"

namespace htn {

namespace {
float lg(double v) { return (float)(std::log2(std::max(v, 1.0)) / 8.0); }

bool runs_fused(const Net &n) {
    if (n.exec == HTN_EXEC_STEPS) return false;
    if (n.exec == HTN_EXEC_FUSED) return n.plan.fused_possible;
    return n.plan.fused_batch_ok;
}
}  // namespace

void step_features(const Net &n, std::vector<float> &rows) {
    const Plan &P = n.plan;
    const bool fused = runs_fused(n);
    const int threads = n.fused_threads;
    std::vector<int> sharing;  // steps per fused phase
    for (int si : P.kernel_steps) {
        const int f = std::max(0, P.steps[si].f_phase);
        if ((int)sharing.size() <= f) sharing.resize(f + 1, 0);
        sharing[f]++;
    }
    for (int si : P.kernel_steps) {
        const StepPlan &s = P.steps[si];
        float f[kFeatures] = {0};
        f[0] = lg(1.0 + s.mults);
        f[1] = lg((double)s.n_out);
        f[2] = lg((double)s.n_sum);
        f[3] = lg((double)P.values[s.a].size);
        f[4] = s.b >= 0 ? lg((double)P.values[s.b].size) : 0.0f;
        const bool tile = fused && s.tile;
        // matrix cores: a per-step GEMM, or a fused tiled step in MFMA mode
        const bool mfma = (!fused && s.mfma) || (tile && s.TM == 0);
        if (tile) {
            f[5] = lg((double)s.tM);
            f[6] = lg((double)s.tN);
            f[7] = lg((double)s.tK);
            f[8] = lg((double)std::max(1, s.TM * s.TN));
        }
        const int R = fused ? s.r_fused : s.r_global;
        if (!tile && !mfma) f[9] = lg((double)R);
        f[10] = tile ? 1.0f : 0.0f;
        if (!tile && !mfma) {
            if (R <= 1)
                f[11] = 1.0f;
            else if (fused && R >= threads)
                f[13] = 1.0f;
            else
                f[12] = 1.0f;
        }
        f[14] = mfma ? 1.0f : 0.0f;
        f[15] = s.b < 0 ? 1.0f : 0.0f;
        f[16] = s.final_step ? 1.0f : 0.0f;
        if (fused) {
            f[17] = (s.f_spill & 1) ? 1.0f : 0.0f;
            f[18] = (s.f_spill & 2) ? 1.0f : 0.0f;
            f[19] = (s.f_spill & 4) ? 1.0f : 0.0f;
            f[20] = lg(1.0 + (double)s.f_copy_chunks);
        }
        f[21] = fused ? 1.0f : 0.0f;
        f[22] = n.compute == HTN_F64 ? 1.0f : 0.0f;
        f[23] = (float)dtype_size(inter_dtype(n.compute)) / 8.0f;
        if (fused) {
            f[24] = lg(64.0 * s.f_nw);
            f[25] = (float)sharing[s.f_phase >= 0 ? s.f_phase : 0] / 8.0f;
        } else {
            f[24] = lg(256.0);
        }
        rows.insert(rows.end(), f, f + kFeatures);
    }
}

std::vector<std::pair<int, int>> learned_path(const Net &n) {
    if (!n.model) return greedy_path(n);
    auto cands = candidate_paths(n, n.path_samples, n.path_seed);  // cands[0]: FLOP-greedy
    Net t = structure_copy(n);
    std::vector<float> rows;
    std::vector<int> owner;  // candidate of each row
    std::vector<int> group;  // fused phase of each row (-1: per-step executor)
    std::vector<char> ok(cands.size(), 0);
    std::vector<double> mults(cands.size(), 0.0);
    double min_mults = std::numeric_limits<double>::infinity();
    for (size_t c = 0; c < cands.size(); ++c) {
        t.path = cands[c];
        try {
            build_plan(t);
        } catch (const Error &e) {
            if (c == 0) throw;  // FLOP-greedy must plan
            continue;           // e.g. above the intermediate cap
        }
        ok[c] = 1;
        mults[c] = t.plan.mults;
        min_mults = std::min(min_mults, mults[c]);
        const size_t before = rows.size();
        step_features(t, rows);
        owner.insert(owner.end(), (rows.size() - before) / kFeatures, (int)c);
        const bool fused = runs_fused(t);
        for (int si : t.plan.kernel_steps) group.push_back(fused ? t.plan.steps[si].f_phase : -1);
    }
    const std::vector<float> y = model_predict(n.model, rows);
    // steps sharing a fused phase run side by side: the phase costs its
    // slowest step (a candidate's rows are contiguous)
    std::vector<double> total(cands.size(), 0.0);
    std::vector<double> phase;
    for (size_t r = 0; r < owner.size();) {
        size_t e = r;
        phase.clear();
        for (; e < owner.size() && owner[e] == owner[r]; ++e) {
            const double d = std::exp((double)y[e]);
            if (group[e] < 0) {
                total[owner[r]] += d;
                continue;
            }
            if ((int)phase.size() <= group[e]) phase.resize(group[e] + 1, 0.0);
            phase[group[e]] = std::max(phase[group[e]], d);
        }
        for (double d : phase) total[owner[r]] += d;
        r = e;
    }
    // trust region: the model ranks candidates within kTrust times the
    // fewest multiplications among them (it is trained on paths near the
    // FLOP optimum and does not extrapolate to far costlier ones)
    constexpr double kTrust = 2.0;
    size_t best = 0;
    for (size_t c = 1; c < cands.size(); ++c)
        if (ok[c] && mults[c] <= kTrust * min_mults && std::isfinite(total[c]) &&
            (mults[best] > kTrust * min_mults || total[c] < total[best]))
            best = c;
    return cands[best];
}

}  // namespace htn
