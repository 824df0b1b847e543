// The fused whole-network kernel (k_fused) and its step routines.  One
// workgroup contracts an entire network: a program image (built by the
// planner) is copied into LDS and interpreted; operands and intermediates
// stay in LDS where they fit (else in the network's workspace); each
// pairwise step is a register-tiled product or a table-driven reduction;
// the last step writes the result.  One launch serves a batch of networks
// (one workgroup each).  Each workgroup size is instantiated in its own
// translation unit (fused_b*.hip).
#pragma once

#include <type_traits>

#include "kern_common.hpp"

namespace htn {
namespace kern {

// ----------------------------------------------------------------- k_fused

// One step inside the fused kernel.  A, B point into LDS; C into LDS or, for
// the final step, global memory.
// Sum over the summed index space (n_shi x n_slo, two-level tables) of one
// output, visiting s = start, start + stride, ... in (sh, sl) form with
// stride = dq * n_slo + dr (dr < n_slo).  Plain sums keep four independent
// partial sums, so four table reads and four operand reads are in flight
// together; compensated sums stay sequential.
template <typename T, typename ACC, bool COMP, bool UNARY>
__device__ __forceinline__ void strided_sum(const T *a0, const T *b0, const int2 *tsh, const int2 *tsl, int sh, int sl,
                                            int dq, int dr, int n_shi, int n_slo, ACC &s, ACC &c) {
    if constexpr (!COMP) {
        ACC s1 = 0, s2 = 0, s3 = 0;
        while (sh < n_shi) {
            int hv[4], lv[4];
            hv[0] = sh;
            lv[0] = sl;
#pragma unroll
            for (int u = 1; u < 4; ++u) {
                hv[u] = hv[u - 1] + dq;
                lv[u] = lv[u - 1] + dr;
                if (lv[u] >= n_slo) {
                    lv[u] -= n_slo;
                    ++hv[u];
                }
            }
            sh = hv[3] + dq;
            sl = lv[3] + dr;
            if (sl >= n_slo) {
                sl -= n_slo;
                ++sh;
            }
            ACC pv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool ok = hv[u] < n_shi;
                const int2 h = tsh[ok ? hv[u] : 0], l = tsl[lv[u]];
                ACC q = (ACC)a0[h.x + l.x];
                if constexpr (!UNARY) q *= (ACC)b0[h.y + l.y];
                pv[u] = ok ? q : ACC(0);
            }
            s += pv[0];
            s1 += pv[1];
            s2 += pv[2];
            s3 += pv[3];
        }
        s += (s1 + s2) + s3;
    } else {
        while (sh < n_shi) {
            const int2 h = tsh[sh], l = tsl[sl];
            ACC q = (ACC)a0[h.x + l.x];
            if constexpr (!UNARY) q *= (ACC)b0[h.y + l.y];
            accum<COMP>(s, c, q);
            sh += dq;
            sl += dr;
            if (sl >= n_slo) {
                sl -= n_slo;
                ++sh;
            }
        }
    }
}

template <int BLK, typename T, typename ACC, bool COMP, bool UNARY, typename TOUT>
// Threads tid = 0..nthr-1 of the step's waves run it; R == nthr (the whole
// workgroup per output) is planned only when the step owns the workgroup
// (nthr == BLK), since it synchronises every wave.
__device__ __forceinline__ void fstep(const T *A, const T *B, TOUT *C, const int2 *__restrict__ tab,
                                      const int32_t *g, int R, ACC *scratch, const int tid, const int nthr) {
    const int n_ohi = g[0], n_olo = g[1], n_shi = g[2], n_slo = g[3];
    const int2 *toh = tab + g[4];
    const int2 *tol = tab + g[5];
    const int2 *tsh = tab + g[6];
    const int2 *tsl = tab + g[7];
    const int n_out = n_ohi * n_olo;
    if (R == BLK && nthr == BLK) {
        // whole workgroup per output (tiny outputs, long sums)
        const int dq = BLK / n_slo, dr = BLK - dq * n_slo;
        const int sh0 = tid / n_slo, sl0 = tid - sh0 * n_slo;
        for (int o = 0; o < n_out; ++o) {
            const int oh = o / n_olo, ol = o - oh * n_olo;  // wave-uniform
            const int2 x = toh[oh], y = tol[ol];
            const T *a0 = A + (x.x + y.x);
            const T *b0 = B;
            if constexpr (!UNARY) b0 = B + (x.y + y.y);
            ACC s = 0, c = 0;
            strided_sum<T, ACC, COMP, UNARY>(a0, b0, tsh, tsl, sh0, sl0, dq, dr, n_shi, n_slo, s, c);
            lane_reduce<COMP>(s, c, 64);
            if ((tid & 63) == 0) {
                scratch[2 * (tid >> 6)] = s;
                scratch[2 * (tid >> 6) + 1] = c;
            }
            __syncthreads();
            if (tid == 0) {
                ACC ts = scratch[0], tc = scratch[1];
                for (int w = 1; w < BLK / 64; ++w) combine<COMP>(ts, tc, scratch[2 * w], scratch[2 * w + 1]);
                C[o] = st_cvt<TOUT>(COMP ? ts + tc : ts);
            }
            __syncthreads();
        }
        return;
    }
    int log2R = 0;
    while ((1 << log2R) < R) ++log2R;
    const int groups = nthr >> log2R;
    const int gi = tid >> log2R, sub = tid & (R - 1);
    const int dq = R / n_slo, dr = R - dq * n_slo;
    // output o = oh * n_olo + ol, advanced by `groups` per pass without a
    // division (one per thread up front)
    const int oq = groups / n_olo, orr = groups - oq * n_olo;
    int oh = gi / n_olo, ol = gi - oh * n_olo;
    const int sh0 = sub / n_slo, sl0 = sub - sh0 * n_slo;
    for (int o0 = 0; o0 < n_out; o0 += groups) {
        const int o = o0 + gi;
        const bool active = o < n_out;
        ACC s = 0, c = 0;
        if (active) {
            const int2 x = toh[oh], y = tol[ol];
            const T *a0 = A + (x.x + y.x);
            const T *b0 = B;
            if constexpr (!UNARY) b0 = B + (x.y + y.y);
            if (R == 1) {
                ACC s1 = 0, s2 = 0, s3 = 0;
                for (int sh = 0; sh < n_shi; ++sh) {
                    const int2 h = tsh[sh];
                    const T *a1 = a0 + h.x;
                    const T *b1 = b0;
                    if constexpr (!UNARY) b1 = b0 + h.y;
                    int sl = 0;
                    if constexpr (!COMP) {
                        // four independent partial sums (ILP)
                        for (; sl + 4 <= n_slo; sl += 4) {
                            const int2 l0 = tsl[sl], l1 = tsl[sl + 1], l2 = tsl[sl + 2], l3 = tsl[sl + 3];
                            ACC p0 = (ACC)a1[l0.x], p1 = (ACC)a1[l1.x], p2 = (ACC)a1[l2.x], p3 = (ACC)a1[l3.x];
                            if constexpr (!UNARY) {
                                p0 *= (ACC)b1[l0.y];
                                p1 *= (ACC)b1[l1.y];
                                p2 *= (ACC)b1[l2.y];
                                p3 *= (ACC)b1[l3.y];
                            }
                            s += p0;
                            s1 += p1;
                            s2 += p2;
                            s3 += p3;
                        }
                    }
                    for (; sl < n_slo; ++sl) {
                        const int2 l = tsl[sl];
                        ACC p = (ACC)a1[l.x];
                        if constexpr (!UNARY) p *= (ACC)b1[l.y];
                        accum<COMP>(s, c, p);
                    }
                }
                s += (s1 + s2) + s3;
            } else {
                strided_sum<T, ACC, COMP, UNARY>(a0, b0, tsh, tsl, sh0, sl0, dq, dr, n_shi, n_slo, s, c);
            }
        }
        lane_reduce<COMP>(s, c, R);
        if (active && sub == 0) C[o] = st_cvt<TOUT>(COMP ? s + c : s);
        oh += oq;
        ol += orr;
        if (ol >= n_olo) {
            ol -= n_olo;
            ++oh;
        }
    }
}

// Register-tiled step: C[tcm[m] + tcn[n]] = sum_k A[k*M + m] * B[k*N + n].
// Thread (tx, ty) of a GX x (kBlk/GX) grid owns outputs m = m0 + tx + GX*i,
// n = n0 + ty + GY*j (i < TM, j < TN).  Across a wave, A reads are
// consecutive or broadcast, B reads broadcast or consecutive.
// Offset of index x of a label group from its digit descriptors (per label,
// last fastest: extent, magic (2 words), stride).
__device__ __forceinline__ int digit_offset(uint32_t x, const int32_t *dg, int nl) {
    int off = 0;
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        if (k < nl) {
            const int32_t *q = dg + 4 * k;
            const uint64_t magic = ((uint64_t)(uint32_t)q[2] << 32) | (uint32_t)q[1];
            const uint32_t quo = (uint32_t)(((uint64_t)x * magic) >> 40);
            off += (int)(x - quo * (uint32_t)q[0]) * q[3];
            x = quo;
        }
    }
    return off;
}

template <int BLK, typename T, typename ACC, int TM, int TN, typename TOUT>
__device__ __forceinline__ void tstep(const T *A, const T *B, TOUT *C, const int32_t *dgm, int nm, const int32_t *dgn,
                                      int nn_l, int M, int N, int K, int GX, const int tid, const int nthr) {
    int lgx = 0;
    while ((1 << lgx) < GX) ++lgx;
    const int GY = nthr >> lgx;
    const int tx = tid & (GX - 1), ty = tid >> lgx;
    const int SM = GX * TM, SN = GY * TN;
    for (int m0 = 0; m0 < M; m0 += SM) {
        if (m0 + tx >= M) break;
        for (int n0 = 0; n0 < N; n0 += SN) {
            if (n0 + ty >= N) break;
            int mi[TM], nj[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int m = m0 + tx + GX * i;
                mi[i] = m < M ? m : M - 1;
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int nn = n0 + ty + GY * j;
                nj[j] = nn < N ? nn : N - 1;
            }
            // U independent partial sums over k hide LDS latency (ILP)
            constexpr int U = TM * TN >= 16 ? 1 : (TM * TN >= 8 ? 2 : (TM * TN >= 4 ? 4 : 8));
            ACC acc[U][TM][TN];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[u][i][j] = 0;
            const T *a = A;
            const T *b = B;
            int k = 0;
            for (; k + U <= K; k += U) {
                T av[U][TM], bv[U][TN];
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int i = 0; i < TM; ++i) av[u][i] = a[u * M + mi[i]];
#pragma unroll
                    for (int j = 0; j < TN; ++j) bv[u][j] = b[u * N + nj[j]];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) acc[u][i][j] += (ACC)av[u][i] * (ACC)bv[u][j];
                a += U * M;
                b += U * N;
            }
            for (; k < K; ++k) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[0][i][j] += (ACC)a[mi[i]] * (ACC)b[nj[j]];
                a += M;
                b += N;
            }
#pragma unroll
            for (int u = 1; u < U; ++u)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[0][i][j] += acc[u][i][j];
            int cn[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) cn[j] = digit_offset((uint32_t)nj[j], dgn, nn_l);
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int m = m0 + tx + GX * i;
                if (m < M) {
                    const int cm = digit_offset((uint32_t)m, dgm, nm);
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        const int nn = n0 + ty + GY * j;
                        if (nn < N) C[cm + cn[j]] = st_cvt<TOUT>(acc[0][i][j]);
                    }
                }
            }
        }
    }
}

// Matrix-core tiled step (same contract as tstep): 16x16 output blocks,
// one wave per block, K in slices of 4 through the FP64 or FP32 16x16x4
// MFMA with accumulation in the compute type.  Lane l supplies
// A(m = 16 bm + l % 16, k = k0 + l / 16) and B(n = 16 bn + l % 16, same k)
// (zero outside the matrices) and receives column l % 16 of the block in
// rows FMfma<T>::row(l, r), r = 0..3.
template <typename T>
struct FMfma;
template <>
struct FMfma<double> {
    typedef double acc __attribute__((ext_vector_type(4)));
    __device__ __forceinline__ static acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct FMfma<float> {
    typedef float acc __attribute__((ext_vector_type(4)));
    __device__ __forceinline__ static acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <int BLK, typename T, typename TOUT>
__device__ __forceinline__ void mstep(const T *A, const T *B, TOUT *C, const int32_t *dgm, int nm, const int32_t *dgn,
                                      int nn_l, int M, int N, int K, const int tid, const int nthr) {
    typedef FMfma<T> Op;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nbm = (M + 15) >> 4, nbn = (N + 15) >> 4;
    for (int blk = wave; blk < nbm * nbn; blk += nthr >> 6) {
        const int bm = blk / nbn, bn = blk - bm * nbn;
        const int m = bm * 16 + li, n = bn * 16 + li;
        const bool mok = m < M, nok = n < N;
        const T *a = A + (mok ? m : 0);
        const T *b = B + (nok ? n : 0);
        typename Op::acc acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
        int k0 = 0;
        for (; k0 + 8 <= K; k0 += 8) {
            const int k = k0 + lk;
            T a0 = a[k * M], b0 = b[k * N], a1 = a[(k + 4) * M], b1 = b[(k + 4) * N];
            a0 = mok ? a0 : T(0);
            a1 = mok ? a1 : T(0);
            b0 = nok ? b0 : T(0);
            b1 = nok ? b1 : T(0);
            acc0 = Op::mma(a0, b0, acc0);
            acc1 = Op::mma(a1, b1, acc1);
        }
        for (; k0 < K; k0 += 4) {
            const int k = k0 + lk;
            const bool kok = k < K;
            T a0 = a[(kok ? k : 0) * M], b0 = b[(kok ? k : 0) * N];
            a0 = (mok && kok) ? a0 : T(0);
            b0 = (nok && kok) ? b0 : T(0);
            acc0 = Op::mma(a0, b0, acc0);
        }
        if (nok) {
            const int cn = digit_offset((uint32_t)n, dgn, nn_l);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int mm = bm * 16 + Op::row(lane, r);
                if (mm < M) C[digit_offset((uint32_t)mm, dgm, nm) + cn] = st_cvt<TOUT>(acc0[r] + acc1[r]);
            }
        }
    }
}

template <int BLK, typename T, typename ACC, typename TOUT>
__device__ __forceinline__ void tstep_sel(const T *A, const T *B, TOUT *C, const int32_t *tcm, int nm,
                                          const int32_t *tcn, int nn_l, int M, int N, int K, int TM, int TN, int GX,
                                          const int tid, const int nthr) {
    if constexpr (std::is_same<T, ACC>::value) {
        if (TM == 0) {  // matrix-core mode
            mstep<BLK, T, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, tid, nthr);
            return;
        }
    }
    switch (TM * 8 + TN) {
        case 9: tstep<BLK, T, ACC, 1, 1, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
        case 10: tstep<BLK, T, ACC, 1, 2, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
        case 12: tstep<BLK, T, ACC, 1, 4, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
        case 17: tstep<BLK, T, ACC, 2, 1, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
        case 18: tstep<BLK, T, ACC, 2, 2, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
        case 20: tstep<BLK, T, ACC, 2, 4, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
        case 33: tstep<BLK, T, ACC, 4, 1, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
        case 34: tstep<BLK, T, ACC, 4, 2, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
        default: tstep<BLK, T, ACC, 4, 4, TOUT>(A, B, C, tcm, nm, tcn, nn_l, M, N, K, GX, tid, nthr); break;
    }
}

// OP_TSTEP: [a, b, c, M, N, K, TM, TN, GX, final, nm, nn, w0, nw, digits of M, digits of N]
// (TM = 0: matrix-core mode, planned only where the accumulator is the
// compute type)
template <int BLK, typename T, int FM, bool PURE>
__device__ __forceinline__ void tstep_dispatch(const int32_t *p, T *sm, T *scr, void *out, const int tid,
                                               const int nthr) {
    const int la = p[1], lb = p[2], lc = p[3];
    const int M = p[4], N = p[5], K = p[6];
    const int TM = p[7], TN = p[8], GX = p[9];
    const bool fin = p[10] != 0;
    const int nm = p[11], nn_l = p[12];
    const int32_t *tcm = p + 15;
    const int32_t *tcn = p + 15 + 4 * nm;
    typedef typename std::conditional<FM == FM_INTER, T, double>::type TO;
    if (PURE || (la >= 0 && lb >= 0 && (fin || lc >= 0))) {
        if (!fin)
            tstep_sel<BLK, T, T, T>(sm + la, sm + lb, sm + lc, tcm, nm, tcn, nn_l, M, N, K, TM, TN, GX, tid, nthr);
        else
            tstep_sel<BLK, T, TO, TO>(sm + la, sm + lb, (TO *)out, tcm, nm, tcn, nn_l, M, N, K, TM, TN, GX, tid,
                                      nthr);
    } else if constexpr (!PURE) {
        const T *A = la >= 0 ? sm + la : scr + (-la - 2);
        const T *B = lb >= 0 ? sm + lb : scr + (-lb - 2);
        if (!fin)
            tstep_sel<BLK, T, T, T>(A, B, lc >= 0 ? sm + lc : scr + (-lc - 2), tcm, nm, tcn, nn_l, M, N, K, TM, TN,
                                    GX, tid, nthr);
        else
            tstep_sel<BLK, T, TO, TO>(A, B, (TO *)out, tcm, nm, tcn, nn_l, M, N, K, TM, TN, GX, tid, nthr);
    }
}

// Contiguous 16-byte-chunk copies of one phase.  The copies that follow a
// step are issued into registers before the step's arithmetic and written
// to LDS after it, so their global latency overlaps the computation.
constexpr int kPrefetch = 4;  // staged chunks per thread
// Global-memory view of a copy source: the image and the workspace both
// live in device memory, so the loads are plain global loads (no flat
// address-space dispatch) and stay independent of LDS traffic.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_uint4;

struct CopyOp {
    const g_uint4 *src;
    int dst;  // 16-byte chunk index in LDS
    int n;
};

__device__ __forceinline__ CopyOp decode_copy(const int32_t *p, const int32_t *image, const unsigned char *ws) {
    // [kind, src chunk, chunks, dst chunk]; kind 0: image words, 1: workspace
    CopyOp c;
    const u32x4 *s = p[1] == 0 ? (const u32x4 *)(image) + p[2] : (const u32x4 *)ws + p[2];
    c.src = (const g_uint4 *)s;
    c.dst = p[4];
    c.n = p[3];
    return c;
}

// Copy n 16-byte chunks from global memory to LDS, four independent loads
// in flight per thread.
template <int BLK>
__device__ __forceinline__ void copy_chunks(const g_uint4 *src, u32x4 *dst, int n) {
    for (int c0 = threadIdx.x; c0 < n; c0 += 4 * BLK) {
        u32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c0 + u * BLK < n) v[u] = src[c0 + u * BLK];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c0 + u * BLK < n) dst[c0 + u * BLK] = v[u];
    }
}

// Copies the chunks [from, ...) of a phase's copy ops [ops, ops_end) (their
// chunks numbered consecutively in op order) with kFlatLoads independent
// loads in flight per thread: the phase then waits about one memory
// latency for all of them, not one per op.
constexpr int kFlatLoads = 8;
template <int BLK>
__device__ __forceinline__ void copy_ops_flat(const int32_t *ops, const int32_t *ops_end, int from,
                                              const int32_t *image, const unsigned char *ws, u32x4 *lds4) {
    if (ops == ops_end) return;
    const int32_t *r = ops;
    CopyOp cur = decode_copy(r, image, ws);
    int cur_start = 0;
    for (int base = from;; base += kFlatLoads * BLK) {
        u32x4 v[kFlatLoads];
        int dst[kFlatLoads];
#pragma unroll
        for (int u = 0; u < kFlatLoads; ++u) {
            const int c = base + (int)threadIdx.x + u * BLK;
            while (r != ops_end && c >= cur_start + cur.n) {  // this thread's chunks only grow
                cur_start += cur.n;
                r += 5;
                if (r != ops_end) cur = decode_copy(r, image, ws);
            }
            dst[u] = -1;
            if (r != ops_end) {
                v[u] = cur.src[c - cur_start];
                dst[u] = cur.dst + (c - cur_start);
            }
        }
#pragma unroll
        for (int u = 0; u < kFlatLoads; ++u)
            if (dst[u] >= 0) lds4[dst[u]] = v[u];
        if (r == ops_end) break;
    }
}

// The fused kernel.  A workgroup copies its network's program into LDS and
// interprets it: COPY moves tables or materialised inputs into LDS,
// STEP / TSTEP contract two values, SYNC ends a phase.
// The interpreter for one network.  PURE: every operand and result lives
// in LDS (no workspace-operand paths, so a smaller body with less register
// pressure).
template <int BLK, typename T, typename TIN, int FM, bool PURE>
__device__ __forceinline__ void fused_body(const FusedDesc &d, const int net, void *const *__restrict__ outs,
                                                     int64_t *__restrict__ stamps, void *out1,
                                                     int64_t *__restrict__ phase_ticks, int max_phases, int64_t t0) {
    extern __shared__ __align__(16) unsigned char smem[];
    int phase = 0;
    int32_t *img = reinterpret_cast<int32_t *>(smem);
    // program words (a multiple of four) as 16-byte chunks
    copy_chunks<BLK>((const g_uint4 *)d.prog, (u32x4 *)smem, d.prog[0] / 4);
    if (d.n_fprep > 0) {
        // materialise the network's inputs into its workspace, one wave per
        // entry, then make the writes visible to the workgroup's reads
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int j = wave; j < d.n_fprep; j += BLK / 64) fprep_entry<T, TIN>(d.fprep[j], lane);
        __threadfence();
    }
    __syncthreads();
    int32_t *slots = img + img[3];
    const int slot_words = img[4];
    unsigned char *red = smem + img[5];  // reduction scratch (256 bytes)
    const int32_t *gimg = d.prog + img[6];
    T *sm = reinterpret_cast<T *>(smem);
    T *scr = (T *)d.scratch;
    void *out = out1 ? out1 : outs[net];
    const int32_t *p = img + 8;
    for (;;) {
        const int op = p[0];
        if (op == OP_END) break;
        if (op == OP_SYNC) {
            __syncthreads();
            if (phase_ticks && threadIdx.x == 0 && phase < max_phases)
                phase_ticks[(int64_t)net * max_phases + phase] = (int64_t)wall_clock64();
            ++phase;
            p += 1;
            continue;
        }
        // A phase: the copies for the next phase (tables and operands; they
        // land after this phase's steps, in regions no step of the phase
        // touches), then the step ops (independent steps, each run by its
        // own waves [w0, w0 + nw); none in the first phase, which only loads
        // operands).  The copies come first so that their loads are issued
        // before the steps are decoded: each thread stages up to kPrefetch
        // chunks in registers while the steps run.
        auto step_length = [](const int32_t *r) { return r[0] == OP_TSTEP ? 15 + 4 * (r[11] + r[12]) : 17; };
        const int32_t *const copies0 = p;
        const int32_t *q = p;
        CopyOp cps[4];
        int starts[5] = {0, 0, 0, 0, 0};
        int nc = 0, tot = 0;
        while (nc < 4 && q[0] == OP_COPY) {
            cps[nc] = decode_copy(q, gimg, (const unsigned char *)d.scratch);
            starts[nc] = tot;
            tot += cps[nc].n;
            ++nc;
            q += 5;
        }
        starts[nc] = tot;
        u32x4 stg0, stg1, stg2, stg3;
        int dst0 = -1, dst1 = -1, dst2 = -1, dst3 = -1;
        {
            const g_uint4 *src[kPrefetch];
            int dst[kPrefetch];
#pragma unroll
            for (int j = 0; j < kPrefetch; ++j) {
                const int c = threadIdx.x + j * BLK;
                src[j] = cps[0].src;
                dst[j] = -1;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < nc && c >= starts[k] && c < starts[k + 1]) {
                        src[j] = cps[k].src + (c - starts[k]);
                        dst[j] = cps[k].dst + (c - starts[k]);
                    }
            }
            if (dst[0] >= 0) stg0 = *src[0];
            if (dst[1] >= 0) stg1 = *src[1];
            if (dst[2] >= 0) stg2 = *src[2];
            if (dst[3] >= 0) stg3 = *src[3];
            dst0 = dst[0];
            dst1 = dst[1];
            dst2 = dst[2];
            dst3 = dst[3];
        }
        const int32_t *const staged_end = q;  // copy ops [copies0, staged_end) are staged
        while (q[0] == OP_COPY) q += 5;        // more than four copy ops: copied after the steps
        const int32_t *const copies_end = q;
        const int32_t *const steps0 = q;
        while (q[0] == OP_STEP || q[0] == OP_TSTEP) q += step_length(q);
        const int32_t *const steps_end = q;
        const int wave = threadIdx.x >> 6;
        for (const int32_t *op_w = steps0; op_w != steps_end; op_w += step_length(op_w)) {
            const int w0 = op_w[0] == OP_TSTEP ? op_w[13] : op_w[15];
            const int nw = op_w[0] == OP_TSTEP ? op_w[14] : op_w[16];
            if (wave < w0 || wave >= w0 + nw) continue;  // wave-uniform
            const int tid = threadIdx.x - 64 * w0, nthr = 64 * nw;
            if (op_w[0] == OP_TSTEP) {
                tstep_dispatch<BLK, T, FM, PURE>(op_w, sm, scr, out, tid, nthr);
                continue;
            }
            // OP_STEP: [a, b, c, n_ohi, n_olo, n_shi, n_slo, t_ohi, t_olo, t_shi, t_slo, R, final, slot, w0, nw]
            const int2 *itab2 = reinterpret_cast<const int2 *>(slots + op_w[14] * slot_words);
            const int la = op_w[1], lb = op_w[2], lc = op_w[3];
            const bool unary = lb == -1;
            const bool fin = op_w[13] != 0;
            const int R = op_w[12];
            typedef typename std::conditional<FM == FM_INTER, T, double>::type TO;
            constexpr bool CMP = (FM == FM_COMP);
            if (PURE || (la >= 0 && (unary || lb >= 0) && (fin || lc >= 0))) {
                const T *A = sm + la;
                const T *B = unary ? nullptr : sm + lb;
                if (!fin) {
                    if (unary)
                        fstep<BLK, T, T, false, true, T>(A, B, sm + lc, itab2, op_w + 4, R, (T *)red, tid, nthr);
                    else
                        fstep<BLK, T, T, false, false, T>(A, B, sm + lc, itab2, op_w + 4, R, (T *)red, tid, nthr);
                } else {
                    if (unary)
                        fstep<BLK, T, TO, CMP, true, TO>(A, B, (TO *)out, itab2, op_w + 4, R, (TO *)red, tid, nthr);
                    else
                        fstep<BLK, T, TO, CMP, false, TO>(A, B, (TO *)out, itab2, op_w + 4, R, (TO *)red, tid, nthr);
                }
            } else if constexpr (!PURE) {
                const T *A = la >= 0 ? sm + la : scr + (-la - 2);
                const T *B = unary ? nullptr : (lb >= 0 ? sm + lb : scr + (-lb - 2));
                if (!fin) {
                    T *C = lc >= 0 ? sm + lc : scr + (-lc - 2);
                    if (unary)
                        fstep<BLK, T, T, false, true, T>(A, B, C, itab2, op_w + 4, R, (T *)red, tid, nthr);
                    else
                        fstep<BLK, T, T, false, false, T>(A, B, C, itab2, op_w + 4, R, (T *)red, tid, nthr);
                } else {
                    if (unary)
                        fstep<BLK, T, TO, CMP, true, TO>(A, B, (TO *)out, itab2, op_w + 4, R, (TO *)red, tid, nthr);
                    else
                        fstep<BLK, T, TO, CMP, false, TO>(A, B, (TO *)out, itab2, op_w + 4, R, (TO *)red, tid, nthr);
                }
            }
        }
        // land the staged chunks, copy any remainder directly
        u32x4 *lds4 = (u32x4 *)smem;
        if (dst0 >= 0) lds4[dst0] = stg0;
        if (dst1 >= 0) lds4[dst1] = stg1;
        if (dst2 >= 0) lds4[dst2] = stg2;
        if (dst3 >= 0) lds4[dst3] = stg3;
        // then every chunk beyond the staged ones, all loads in flight
        if (tot > kPrefetch * BLK || copies_end != staged_end)
            copy_ops_flat<BLK>(copies0, copies_end, min(tot, kPrefetch * BLK), gimg, (const unsigned char *)d.scratch,
                               lds4);
        p = steps_end;
    }
    if (stamps && threadIdx.x == 0) {
        stamps[2 * net] = t0;
        stamps[2 * net + 1] = (int64_t)wall_clock64();
    }
}

template <int BLK, typename T, typename TIN, int FM>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(2))) void k_fused(const FusedDesc *__restrict__ nets, const int32_t *__restrict__ order,
                                               void *const *__restrict__ outs, int64_t *__restrict__ stamps,
                                               void *out1, int64_t *__restrict__ phase_ticks, int max_phases) {
    const int net = order ? order[blockIdx.x] : (int)blockIdx.x;
    const int64_t t0 = stamps ? (int64_t)wall_clock64() : 0;
    const FusedDesc d = nets[net];
    if (d.lds_only)
        fused_body<BLK, T, TIN, FM, true>(d, net, outs, stamps, out1, phase_ticks, max_phases, t0);
    else
        fused_body<BLK, T, TIN, FM, false>(d, net, outs, stamps, out1, phase_ticks, max_phases, t0);
}

template <int BLK, typename T, typename TIN, int FM>
static hipError_t go_fused(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps,
                           void *out1, int64_t *phase_ticks, int max_phases, int n_blocks, int lds_bytes,
                           hipStream_t st) {
    static int configured = -1;
    if (lds_bytes > configured) {
        hipError_t e = hipFuncSetAttribute((const void *)k_fused<BLK, T, TIN, FM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        configured = lds_bytes;
    }
    hipLaunchKernelGGL((k_fused<BLK, T, TIN, FM>), dim3(n_blocks), dim3(BLK), lds_bytes, st, nets, order, outs,
                       stamps, out1, phase_ticks, max_phases);
    return hipGetLastError();
}

template <int BLK>
hipError_t launch_fused_blk(const FusedDesc *nets, const int32_t *order, void *const *outs, int64_t *stamps,
                            void *out1, int64_t *phase_ticks, int max_phases, int n_blocks, int lds_bytes, int compute,
                            int fm, hipStream_t st) {
#define HTN_GO(T, TIN, F) go_fused<BLK, T, TIN, F>(nets, order, outs, stamps, out1, phase_ticks, max_phases, n_blocks, lds_bytes, st)
    if (compute == 0) return fm == FM_COMP ? HTN_GO(double, double, FM_COMP) : HTN_GO(double, double, FM_INTER);
    if (compute == 1) {
        if (fm == FM_COMP) return HTN_GO(float, float, FM_COMP);
        if (fm == FM_F64) return HTN_GO(float, float, FM_F64);
        return HTN_GO(float, float, FM_INTER);
    }
    if (compute == 2) {
        if (fm == FM_COMP) return HTN_GO(float, bf16_t, FM_COMP);
        if (fm == FM_F64) return HTN_GO(float, bf16_t, FM_F64);
        return HTN_GO(float, bf16_t, FM_INTER);
    }
#undef HTN_GO
    return hipErrorInvalidValue;
}

}  // namespace kern
}  // namespace htn
