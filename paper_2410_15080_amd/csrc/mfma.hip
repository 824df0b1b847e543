// Matrix-core (MFMA) GEMM for pairwise steps that are dense matrix products.
//
// Fragment layouts (checked on gfx950 with an in-bounds probe): A and B
// lanes hold row/column lane%16 and K slice lane/16; the 16x16 result
// block holds column lane%16 in every register, with rows 4*(lane/16)+r for
// the FP32-accumulating instructions and lane/16+4*r for the FP64 one.
//
//   C[b][m][n] = sum_k A[b][m][k] * B[b][n][k]
//
// Operands are packed K-contiguous by the step's pack kernels, so every
// lane's MFMA fragment is a contiguous LDS read.  Workgroup tile 128x128,
// four wave64s each owning a 64x64 sub-tile (4x4 MFMA 16x16 blocks), or
// 64x128 with 32x64 sub-tiles where FP64 accumulators sit beside the FP32
// ones; K staged through double-buffered LDS.  Per input type:
//   double : v_mfma_f64_16x16x4_f64,  FP64 accumulation
//   float  : v_mfma_f32_16x16x4_f32,  FP32 accumulation per K-chunk
//   bf16   : v_mfma_f32_16x16x32_bf16, FP32 accumulation per K-chunk
// With FP32 accumulation, every `kchunk` elements of K the partial products
// are added into FP64 accumulators (the signed QPD sum is combined in FP64).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "kernels.hpp"
#include "mfma_dev.hpp"

namespace htn {
namespace kern {

// Output tiles t = ((b * ksplit + kz) * tiles_m + tm) * tiles_n + tn: batch
// entry b, K range kz (of length kper, a multiple of BK), tile row tm and
// column tn; the output of range kz goes to C + (kz * batch + b) * sC.
// Each workgroup takes tiles blockIdx.x, blockIdx.x + gridDim.x, ...: the
// first K slice of its next tile is loaded while the current tile's last
// slice is multiplied and its results are stored, so the store of one tile
// and the loads of the next overlap.
// Each wave owns WI x 4 blocks of 16x16 (the workgroup tile is 32 WI x 128):
// WI = 4 where the accumulators are the instruction's own; WI = 2 where FP64
// accumulators are kept beside FP32 ones, so that two waves per SIMD still
// fit in the register file.
template <typename T, typename TOUT, bool COMBINE64, int WI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm(const T *__restrict__ A0, const T *__restrict__ B0,
                                             TOUT *__restrict__ C0, int M, int N, int K, int64_t sA, int64_t sB,
                                             int64_t sC, int kchunk, int ksplit, int kper, int batch, int tiles_m,
                                             int tiles_n, int n_tiles) {
    typedef MfmaOp<T> Op;
    constexpr int BK = Op::BK;
    constexpr int LD = BK + Op::PAD;
    constexpr int TBM = 32 * WI;
    __shared__ __align__(16) T As[2][TBM * LD];
    __shared__ __align__(16) T Bs[2][GBN * LD];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * (16 * WI), wn = (wave & 1) * 64;
    const int lr = lane & 15, lk = (lane >> 4) * Op::KPL;
    struct Tile {
        const T *A, *B;
        TOUT *C;
        int m0, n0, kbeg, kend;
    };
    auto tile_of = [&](int t) {
        Tile u;
        const int tn = t % tiles_n;
        const int r = t / tiles_n;
        const int tm = r % tiles_m;
        const int z = r / tiles_m;
        const int bz = z / ksplit, kz = z - bz * ksplit;
        u.kbeg = kz * kper;
        u.kend = min(K, u.kbeg + kper);
        u.A = A0 + bz * sA;
        u.B = B0 + bz * sB;
        u.C = C0 + ((int64_t)kz * batch + bz) * sC;
        u.m0 = tm * TBM;
        u.n0 = tn * GBN;
        return u;
    };

    TileLoader<T, TBM> la;
    TileLoader<T, GBN> lb;
    int t = blockIdx.x;
    Tile cur = tile_of(t);
    la.load(cur.A, M, K, cur.kend, cur.m0, cur.kbeg);
    lb.load(cur.B, N, K, cur.kend, cur.n0, cur.kbeg);
    for (;;) {
        la.store(As[0]);
        lb.store(Bs[0]);
        __syncthreads();
        typename Op::acc acc[WI][4];
        d4_t acc64[COMBINE64 ? WI : 1][4];
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = typename Op::acc{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < (COMBINE64 ? WI : 1); ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc64[i][j] = d4_t{0, 0, 0, 0};
        const int nk = (cur.kend - cur.kbeg + BK - 1) / BK;
        const int t_next = t + gridDim.x;
        Tile nxt = cur;
        if (t_next < n_tiles) nxt = tile_of(t_next);
        int since = 0;
        for (int kt = 0; kt < nk; ++kt) {
            const int cb = kt & 1;
            if (kt + 1 < nk) {
                la.load(cur.A, M, K, cur.kend, cur.m0, cur.kbeg + (kt + 1) * BK);
                lb.load(cur.B, N, K, cur.kend, cur.n0, cur.kbeg + (kt + 1) * BK);
            } else if (t_next < n_tiles) {
                la.load(nxt.A, M, K, nxt.kend, nxt.m0, nxt.kbeg);
                lb.load(nxt.B, N, K, nxt.kend, nxt.n0, nxt.kbeg);
            }
            const T *as = As[cb];
            const T *bs = Bs[cb];
#pragma unroll
            for (int kk = 0; kk < BK; kk += Op::KI) {
                typename Op::frag fa[WI], fb[4];
#pragma unroll
                for (int i = 0; i < WI; ++i) fa[i] = Op::ld(as + (wm + 16 * i + lr) * LD + kk + lk);
#pragma unroll
                for (int j = 0; j < 4; ++j) fb[j] = Op::ld(bs + (wn + 16 * j + lr) * LD + kk + lk);
#pragma unroll
                for (int i = 0; i < WI; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = Op::mma(fa[i], fb[j], acc[i][j]);
            }
            if constexpr (COMBINE64) {
                since += BK;
                if (since >= kchunk || kt + 1 == nk) {
#pragma unroll
                    for (int i = 0; i < WI; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                acc64[i][j][r] += (double)acc[i][j][r];
                                acc[i][j][r] = 0;
                            }
                    since = 0;
                }
            }
            if (kt + 1 < nk) {
                la.store(As[cb ^ 1]);
                lb.store(Bs[cb ^ 1]);
            }
            __syncthreads();
        }
        if (nk == 0 && t_next < n_tiles) {  // (empty K range: nothing loaded above)
            la.load(nxt.A, M, K, nxt.kend, nxt.m0, nxt.kbeg);
            lb.load(nxt.B, N, K, nxt.kend, nxt.n0, nxt.kbeg);
        }
        // D block: column lane%16; the row of register r depends on the
        // instruction (Op::row).  Streaming (nontemporal) stores: the
        // result is written once and not read back by this launch, and
        // where the output dominates the traffic (BF16 inputs, FP64 output)
        // they cut the GEMM's time by a fifth against plain stores.
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gm = cur.m0 + wm + 16 * i + Op::row(lane, r);
                    const int gn = cur.n0 + wn + 16 * j + (lane & 15);
                    if (gm < M && gn < N) {
                        TOUT v;
                        if constexpr (COMBINE64)
                            v = (TOUT)acc64[COMBINE64 ? i : 0][j][r];
                        else
                            v = (TOUT)acc[i][j][r];
                        __builtin_nontemporal_store(v, cur.C + (int64_t)gm * N + gn);
                    }
                }
        if (t_next >= n_tiles) break;
        t = t_next;
        cur = nxt;
    }
}

// Sum of the K-range partial products, in range order.
template <typename TOUT>
__global__ __launch_bounds__(256) void k_ksum(const TOUT *__restrict__ part, TOUT *__restrict__ C, int64_t total,
                                             int ksplit) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        TOUT a = part[i];
        for (int kz = 1; kz < ksplit; ++kz) a += part[(int64_t)kz * total + i];
        C[i] = a;
    }
}

static int compute_units() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        return 256;
    return n;
}

template <typename T, typename TOUT, bool C64>
static hipError_t go_gemm(const void *A, const void *B, void *C, int M, int N, int K, int batch, int kchunk,
                          int ksplit, void *part, hipStream_t st) {
    const int64_t sA = (int64_t)M * K, sB = (int64_t)N * K, sC = (int64_t)M * N;
    int kper = 0;
    gemm_ksplit(K, ksplit, kper);
    constexpr int WI = C64 ? 2 : 4;
    const int tiles_n = (N + GBN - 1) / GBN, tiles_m = (M + 32 * WI - 1) / (32 * WI);
    const int64_t n_tiles = (int64_t)tiles_n * tiles_m * batch * ksplit;
    if (n_tiles > INT32_MAX) return hipErrorInvalidValue;
    // two resident workgroups per CU (registers and LDS allow two), each
    // walking over its share of the tiles
    static const int cus = compute_units();
    const int grid = (int)std::min<int64_t>(n_tiles, 2 * (int64_t)cus);
    TOUT *dst = ksplit > 1 ? (TOUT *)part : (TOUT *)C;
    hipLaunchKernelGGL((k_gemm<T, TOUT, C64, WI>), dim3(grid), dim3(256), 0, st, (const T *)A, (const T *)B, dst, M,
                       N, K, sA, sB, sC, kchunk, ksplit, kper, batch, tiles_m, tiles_n, (int)n_tiles);
    if (ksplit > 1) {
        const int64_t total = (int64_t)batch * sC;
        const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL((k_ksum<TOUT>), dim3((unsigned)blocks), dim3(256), 0, st, (const TOUT *)part, (TOUT *)C,
                           total, ksplit);
    }
    return hipGetLastError();
}

hipError_t launch_gemm(const void *A, const void *B, void *C, int tin, int tout, int M, int N, int K, int batch,
                       int kchunk, int ksplit, void *part, hipStream_t st) {
    if (ksplit < 1 || (ksplit > 1 && !part)) return hipErrorInvalidValue;
    if (tin == 0 && tout == 0) return go_gemm<double, double, false>(A, B, C, M, N, K, batch, kchunk, ksplit, part, st);
    if (tin == 1 && tout == 0) return go_gemm<float, double, true>(A, B, C, M, N, K, batch, kchunk, ksplit, part, st);
    if (tin == 1 && tout == 1) return go_gemm<float, float, false>(A, B, C, M, N, K, batch, kchunk, ksplit, part, st);
    if (tin == 2 && tout == 0) return go_gemm<bf16_t, double, true>(A, B, C, M, N, K, batch, kchunk, ksplit, part, st);
    if (tin == 2 && tout == 1) return go_gemm<bf16_t, float, false>(A, B, C, M, N, K, batch, kchunk, ksplit, part, st);
    return hipErrorInvalidValue;
}

}  // namespace kern
}  // namespace htn
