// Device bodies shared by the per-step kernels (kernels.hip) and the
// persistent work queue (queue.hip), so that a step gives the same result
// bit for bit whichever of the two runs it.
#pragma once

#include "kern_common.hpp"

namespace htn {
namespace kern {

// Block `blk` of the pairwise step C[o] = sum_s A[.]*B[.] (k_step's grid:
// R lanes per output, outputs in block order; with split sums, `split`
// lane groups per output write (sum, compensation) partials).
template <typename TA, typename TB, typename TC, typename ACC, bool UNARY, bool COMP>
__device__ __forceinline__ void step_block(const TA *__restrict__ A, const TB *__restrict__ B, TC *__restrict__ C,
                                           const int2 *__restrict__ tab, const StepArgs &s, int64_t blk) {
    const int64_t gt = blk * kBlk + threadIdx.x;
    const int64_t grp = gt >> s.log2R;
    const int64_t o = s.split > 1 ? grp / s.split : grp;
    const int jc = (int)(grp - o * s.split);  // chunk of the summed range (split > 1)
    const int sub = (int)(gt & (s.R - 1));
    const bool active = o < s.n_out;
    ACC acc = 0, cmp = 0;
    if (active && s.split > 1) {
        const int oh = (int)(o / s.n_olo);
        const int ol = (int)(o - (int64_t)oh * s.n_olo);
        const int2 x = tab[s.t_ohi + oh], y = tab[s.t_olo + ol];
        const TA *a0 = A + (x.x + y.x);
        const TB *b0 = B;
        if constexpr (!UNARY) b0 = B + (x.y + y.y);
        const int2 *th = tab + s.t_shi;
        const int2 *tl = tab + s.t_slo;
        const int64_t n_sum = (int64_t)s.n_shi * s.n_slo;
        int64_t e = (int64_t)jc * s.chunk + sub;
        const int64_t e_end = min(n_sum, (int64_t)(jc + 1) * s.chunk);
        int sh = (int)(e / s.n_slo);
        int sl = (int)(e - (int64_t)sh * s.n_slo);
        const int dq = s.R / s.n_slo, dr = s.R - dq * s.n_slo;
        for (; e < e_end; e += s.R) {
            const int2 h = th[sh], l = tl[sl];
            ACC p = Ld<ACC, TA>::get(a0 + h.x + l.x);
            if constexpr (!UNARY) p *= Ld<ACC, TB>::get(b0 + h.y + l.y);
            accum<COMP>(acc, cmp, p);
            sh += dq;
            sl += dr;
            if (sl >= s.n_slo) {
                sl -= s.n_slo;
                ++sh;
            }
        }
    } else if (active) {
        const int oh = (int)(o / s.n_olo);
        const int ol = (int)(o - (int64_t)oh * s.n_olo);
        const int2 x = tab[s.t_ohi + oh], y = tab[s.t_olo + ol];
        const TA *a0 = A + (x.x + y.x);
        const TB *b0 = B;
        if constexpr (!UNARY) b0 = B + (x.y + y.y);
        const int2 *th = tab + s.t_shi;
        const int2 *tl = tab + s.t_slo;
        if (s.R == 1) {
            for (int sh = 0; sh < s.n_shi; ++sh) {
                const int2 h = th[sh];
                const TA *a1 = a0 + h.x;
                const TB *b1 = b0;
                if constexpr (!UNARY) b1 = b0 + h.y;
                for (int sl = 0; sl < s.n_slo; ++sl) {
                    const int2 l = tl[sl];
                    ACC p = Ld<ACC, TA>::get(a1 + l.x);
                    if constexpr (!UNARY) p *= Ld<ACC, TB>::get(b1 + l.y);
                    accum<COMP>(acc, cmp, p);
                }
            }
        } else {
            const int dq = s.R / s.n_slo, dr = s.R - dq * s.n_slo;
            int sh = sub / s.n_slo;
            int sl = sub - sh * s.n_slo;
            while (sh < s.n_shi) {
                const int2 h = th[sh], l = tl[sl];
                ACC p = Ld<ACC, TA>::get(a0 + h.x + l.x);
                if constexpr (!UNARY) p *= Ld<ACC, TB>::get(b0 + h.y + l.y);
                accum<COMP>(acc, cmp, p);
                sh += dq;
                sl += dr;
                if (sl >= s.n_slo) {
                    sl -= s.n_slo;
                    ++sh;
                }
            }
        }
    }
    lane_reduce<COMP>(acc, cmp, s.R);
    if (active && sub == 0) {
        if (s.split > 1) {
            double *q = s.part + 2 * (o * s.split + jc);
            q[0] = (double)acc;
            q[1] = COMP ? (double)cmp : 0.0;
        } else {
            C[o] = st_cvt<TC>(COMP ? acc + cmp : acc);
        }
    }
}

// Second pass of a split sum for output o, run by one wave (lane = lane
// index): lanes stride over the `split` partial (sum, compensation) pairs,
// then a fixed shuffle tree combines them.
template <typename TC, bool COMP>
__device__ __forceinline__ void split_finish_one(const double *__restrict__ part, TC *__restrict__ C, int split,
                                                 int64_t o, int lane) {
    double sum = 0.0, cmp = 0.0;
    for (int j = lane; j < split; j += 64) {
        const double *q = part + 2 * (o * split + j);
        combine<COMP>(sum, cmp, q[0], q[1]);
    }
    lane_reduce<COMP>(sum, cmp, 64);
    if (lane == 0) C[o] = st_cvt<TC>(COMP ? sum + cmp : sum);
}

// Element e of a scaled-input materialisation: the input entry (through the
// source gather table when the layout changes) times each folded
// coefficient tensor's entry, in the intermediate type.
template <typename TIN, typename TI>
__device__ __forceinline__ TI prep_value(const PrepDesc &q, const int2 *__restrict__ tab, int e) {
    const TIN *src = (const TIN *)q.src;
    int se = e;
    if (q.snlo > 0) {
        const int eh = e / q.snlo;
        se = tab[q.sthi + eh].x + tab[q.stlo + (e - eh * q.snlo)].x;
    }
    TI v = Ld<TI, TIN>::get(src + se);
    for (int k = 0; k < q.ns; ++k) {
        const int eh = e / q.nlo[k];
        const int el = e - eh * q.nlo[k];
        v *= Ld<TI, TIN>::get((const TIN *)q.sp[k] + tab[q.thi[k] + eh].x + tab[q.tlo[k] + el].x);
    }
    return v;
}

}  // namespace kern
}  // namespace htn
