// Matrix-core building blocks shared by the GEMM kernel (mfma.hip) and the
// persistent work queue (queue.hip): instruction wrappers per input type,
// the register-staged tile loader, and one output tile computed start to
// end (the queue's unit of GEMM work; the same K order and FP64 chunk
// combine as the GEMM kernel, so both give the same result).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace htn {
namespace kern {

typedef uint16_t bf16_t;
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int GBN = 128;

template <typename T>
struct MfmaOp;

template <>
struct MfmaOp<double> {
    typedef double frag;
    typedef d4_t acc;
    static constexpr int KI = 4;   // K per instruction
    static constexpr int KPL = 1;  // K values per lane
    static constexpr int BK = 16;
    static constexpr int PAD = 1;
    // output block: lane holds rows lane/16 + 4*r (interleaved)
    __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
    __device__ __forceinline__ static acc mma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static frag ld(const double *p) { return *p; }
};

template <>
struct MfmaOp<float> {
    typedef float frag;
    typedef f4_t acc;
    static constexpr int KI = 4;
    static constexpr int KPL = 1;
    static constexpr int BK = 32;
    static constexpr int PAD = 1;
    // output block: lane holds rows 4*(lane/16) + r (blocked)
    __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ __forceinline__ static acc mma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static frag ld(const float *p) { return *p; }
};

template <>
struct MfmaOp<bf16_t> {
    typedef bf8_t frag;
    typedef f4_t acc;
    static constexpr int KI = 32;
    static constexpr int KPL = 8;
    static constexpr int BK = 64;
    static constexpr int PAD = 8;
    __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ __forceinline__ static acc mma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static frag ld(const bf16_t *p) { return *(const bf8_t *)p; }
};

// Load a ROWS x BK tile (rows r0.., K-columns k0..) of a [rows][K] operand
// into registers: 16 bytes per load, zero outside the matrix.
template <typename T, int ROWS>
struct TileLoader {
    static constexpr int BK = MfmaOp<T>::BK;
    static constexpr int EPV = 16 / sizeof(T);               // elements per 16B vector
    static constexpr int VPR = BK / EPV;                      // vectors per row
    static constexpr int NV = ROWS * VPR / 256;               // vectors per thread
    static_assert(NV * 256 == ROWS * VPR, "tile rows must fill the workgroup's loads");
    uint4 v[NV];
    // rows of length K (the row stride); columns at or beyond klim read 0
    __device__ __forceinline__ void load(const T *__restrict__ src, int rows, int K, int klim, int r0, int k0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int idx = threadIdx.x + i * 256;
            const int r = idx / VPR, c = (idx % VPR) * EPV;
            const int gr = r0 + r, gk = k0 + c;
            if (gr < rows && gk + EPV <= klim && ((K % EPV) == 0)) {
                v[i] = *(const uint4 *)(src + (int64_t)gr * K + gk);
            } else {
                T tmp[EPV];
#pragma unroll
                for (int e = 0; e < EPV; ++e) {
                    const bool ok = gr < rows && gk + e < klim;
                    tmp[e] = ok ? src[(int64_t)gr * K + gk + e] : T(0);
                }
                v[i] = *(const uint4 *)tmp;
            }
        }
    }
    __device__ __forceinline__ void store(T *lds) const {
        constexpr int LD = BK + MfmaOp<T>::PAD;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int idx = threadIdx.x + i * 256;
            const int r = idx / VPR, c = (idx % VPR) * EPV;
            const T *tv = (const T *)&v[i];
#pragma unroll
            for (int e = 0; e < EPV; ++e) lds[r * LD + c + e] = tv[e];
        }
    }
};

// One output tile of C[b][m][n] = sum_k A[b][m][k] B[b][n][k]: tile index t
// as in the GEMM kernel ((b * ksplit + kz) * tiles_m + tm) * tiles_n + tn.
// lds: 16-byte aligned, gemm_lds_bytes<T, WI, NBUF>() bytes.  NBUF = 2:
// the next K slice is staged into the other LDS buffer while the current
// one is multiplied; NBUF = 1: one buffer (half the LDS), the next slice
// waits in registers until the current one is consumed.  Neither the tile
// shape (WI) nor the buffering changes any output's K order.
template <typename T, int WI, int NBUF = 2>
__host__ __device__ constexpr int gemm_lds_bytes() {
    return NBUF * (32 * WI + GBN) * (MfmaOp<T>::BK + MfmaOp<T>::PAD) * (int)sizeof(T);
}

template <typename T, typename TOUT, bool COMBINE64, int WI, int NBUF = 2>
__device__ void gemm_tile(const T *__restrict__ A0, const T *__restrict__ B0, TOUT *__restrict__ C0, int M, int N,
                          int K, int kchunk, int ksplit, int kper, int batch, int tiles_m, int tiles_n, int t,
                          unsigned char *lds) {
    typedef MfmaOp<T> Op;
    constexpr int BK = Op::BK;
    constexpr int LD = BK + Op::PAD;
    constexpr int TBM = 32 * WI;
    T *const As = (T *)lds;                     // NBUF buffers of TBM x LD
    T *const Bs = (T *)lds + NBUF * TBM * LD;   // NBUF buffers of GBN x LD
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * (16 * WI), wn = (wave & 1) * 64;
    const int lr = lane & 15, lk = (lane >> 4) * Op::KPL;
    const int tn = t % tiles_n;
    const int r = t / tiles_n;
    const int tm = r % tiles_m;
    const int z = r / tiles_m;
    const int bz = z / ksplit, kz = z - bz * ksplit;
    const int kbeg = kz * kper, kend = min(K, kbeg + kper);
    const T *A = A0 + (int64_t)bz * M * K;
    const T *B = B0 + (int64_t)bz * N * K;
    TOUT *C = C0 + ((int64_t)kz * batch + bz) * ((int64_t)M * N);
    const int m0 = tm * TBM, n0 = tn * GBN;
    TileLoader<T, TBM> la;
    TileLoader<T, GBN> lb;
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
    const int nk = (kend - kbeg + BK - 1) / BK;
    if (nk > 0) {
        la.load(A, M, K, kend, m0, kbeg);
        lb.load(B, N, K, kend, n0, kbeg);
        la.store(As);
        lb.store(Bs);
    }
    __syncthreads();
    int since = 0;
    for (int kt = 0; kt < nk; ++kt) {
        const int cb = NBUF == 2 ? (kt & 1) : 0;
        if (kt + 1 < nk) {
            la.load(A, M, K, kend, m0, kbeg + (kt + 1) * BK);
            lb.load(B, N, K, kend, n0, kbeg + (kt + 1) * BK);
        }
        const T *as = As + cb * (TBM * LD);
        const T *bs = Bs + cb * (GBN * LD);
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
                        for (int q = 0; q < 4; ++q) {
                            acc64[i][j][q] += (double)acc[i][j][q];
                            acc[i][j][q] = 0;
                        }
                since = 0;
            }
        }
        if constexpr (NBUF == 2) {
            if (kt + 1 < nk) {
                la.store(As + (cb ^ 1) * (TBM * LD));
                lb.store(Bs + (cb ^ 1) * (GBN * LD));
            }
        } else {
            __syncthreads();  // every wave is done with the buffer
            if (kt + 1 < nk) {
                la.store(As);
                lb.store(Bs);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gm = m0 + wm + 16 * i + Op::row(lane, q);
                const int gn = n0 + wn + 16 * j + (lane & 15);
                if (gm < M && gn < N) {
                    if constexpr (COMBINE64)
                        C[(int64_t)gm * N + gn] = (TOUT)acc64[COMBINE64 ? i : 0][j][q];
                    else
                        C[(int64_t)gm * N + gn] = (TOUT)acc[i][j][q];
                }
            }
}

// K range of each split part (a multiple of 64) and the number of parts.
__host__ __device__ inline void gemm_ksplit(int K, int &ksplit, int &kper) {
    kper = ksplit > 1 ? ((K + ksplit - 1) / ksplit + 63) / 64 * 64 : K;
    if (ksplit > 1) ksplit = (K + kper - 1) / kper;
}

}  // namespace kern
}  // namespace htn
