// QT evaluator (Sec. 6.2): exact statevector simulation of subcircuit
// instances on the GPU, one workgroup per instance, and the assembly of
// quantum-tensor entries as signed sums of instance results.
//
// Qubit q of an n-qubit instance is bit n-1-q of the amplitude index
// (qubit 0 slowest, as a row-major (2,)*n array).  A state of up to
// kSvLdsQubits qubits lives in LDS, a larger one in its instance's slice of
// a global buffer.  Ops are applied in place, one per barrier-separated
// pass: a single-qubit unitary updates amplitude pairs, CZ / RZZ /
// projections scale amplitudes, CX swaps pairs.  The result of a Pauli
// observable O = (x)_q P_q with projectors on the kept qubits,
//     out[x] = Re sum_{s: kept bits of s = x} conj(psi[s ^ m]) c(s) psi[s],
// uses O|s> = c(s) |s ^ m>: m flips the X and Y qubits, and
// c(s) = i^{#Y} (-1)^{popcount(s & (Z|Y qubits))}.  Each output's terms are
// summed in a fixed order (deterministic results).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kern_common.hpp"
#include "kernels.hpp"

namespace htn {
namespace kern {

namespace {

constexpr int kSvThreads = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// index j of the 2^(n-1) pairs with bit p cleared -> amplitude index
__device__ __forceinline__ int64_t insert_zero(int64_t j, int p) {
    return ((j >> p) << (p + 1)) | (j & ((int64_t(1) << p) - 1));
}

__global__ __launch_bounds__(kSvThreads) void k_sv_eval(const SvInst *__restrict__ insts,
                                                        const SvOp *__restrict__ ops, double2 *__restrict__ gstate,
                                                        double *__restrict__ outs) {
    extern __shared__ double2 lds_state[];
    __shared__ double red[kSvThreads / 64];
    __shared__ int pos_kept[kSvMaxQubits], pos_rest[kSvMaxQubits];
    const SvInst &I = insts[blockIdx.x];
    const int n = I.n, tid = threadIdx.x;
    const int64_t N = int64_t(1) << n;
    double2 *psi = I.state_off < 0 ? lds_state : gstate + I.state_off;
    // product state
    for (int64_t s = tid; s < N; s += kSvThreads) {
        double2 a = make_double2(1.0, 0.0);
        for (int q = 0; q < n; ++q) {
            const int b = (int)((s >> (n - 1 - q)) & 1);
            a = cmul(a, make_double2(I.init[q][2 * b], I.init[q][2 * b + 1]));
        }
        psi[s] = a;
    }
    // bit positions of the kept qubits (in output order) and of the others
    // (ascending)
    if (tid < I.n_kept) pos_kept[tid] = n - 1 - I.kept[tid];
    if (tid == 0) {
        int r = 0;
        for (int q = n - 1; q >= 0; --q) {
            bool kept = false;
            for (int k = 0; k < I.n_kept; ++k) kept = kept || I.kept[k] == q;
            if (!kept) pos_rest[r++] = n - 1 - q;
        }
    }
    __syncthreads();
    for (int k = 0; k < I.n_ops; ++k) {
        const SvOp &op = ops[I.op_off + k];
        if (op.kind == SV_U1) {
            const int p = n - 1 - op.q0;
            const double2 u00 = make_double2(op.m[0], op.m[1]), u01 = make_double2(op.m[2], op.m[3]);
            const double2 u10 = make_double2(op.m[4], op.m[5]), u11 = make_double2(op.m[6], op.m[7]);
            for (int64_t j = tid; j < N / 2; j += kSvThreads) {
                const int64_t i0 = insert_zero(j, p), i1 = i0 | (int64_t(1) << p);
                const double2 a = psi[i0], b = psi[i1];
                const double2 x = cmul(u00, a), y = cmul(u01, b), z = cmul(u10, a), w = cmul(u11, b);
                psi[i0] = make_double2(x.x + y.x, x.y + y.y);
                psi[i1] = make_double2(z.x + w.x, z.y + w.y);
            }
        } else if (op.kind == SV_CZ) {
            const int64_t mask = (int64_t(1) << (n - 1 - op.q0)) | (int64_t(1) << (n - 1 - op.q1));
            for (int64_t s = tid; s < N; s += kSvThreads)
                if ((s & mask) == mask) psi[s] = make_double2(-psi[s].x, -psi[s].y);
        } else if (op.kind == SV_CX) {
            const int pc = n - 1 - op.q0, pt = n - 1 - op.q1;
            for (int64_t j = tid; j < N / 2; j += kSvThreads) {
                const int64_t i0 = insert_zero(j, pt), i1 = i0 | (int64_t(1) << pt);
                if ((i0 >> pc) & 1) {
                    const double2 a = psi[i0];
                    psi[i0] = psi[i1];
                    psi[i1] = a;
                }
            }
        } else if (op.kind == SV_RZZ) {
            const int pa = n - 1 - op.q0, pb = n - 1 - op.q1;
            const double c = cos(0.5 * op.m[0]), sn = sin(0.5 * op.m[0]);
            const double2 even = make_double2(c, -sn), odd = make_double2(c, sn);
            for (int64_t s = tid; s < N; s += kSvThreads)
                psi[s] = cmul(psi[s], (((s >> pa) ^ (s >> pb)) & 1) ? odd : even);
        } else {  // SV_PROJ
            const int p = n - 1 - op.q0;
            const int64_t keep = op.q1;
            for (int64_t s = tid; s < N; s += kSvThreads)
                if (((s >> p) & 1) != keep) psi[s] = make_double2(0.0, 0.0);
        }
        __syncthreads();
    }
    // measurement
    const int64_t xm = I.xmask, zy = I.zymask;
    const int ny4 = I.n_y & 3;
    const int k = I.n_kept, m = n - k;
    const int64_t n_out = int64_t(1) << k, n_rest = int64_t(1) << m;
    auto term = [&](int64_t x, int64_t r) -> double {
        int64_t s = 0;
        for (int j = 0; j < k; ++j) s |= ((x >> (k - 1 - j)) & 1) << pos_kept[j];
        for (int j = 0; j < m; ++j) s |= ((r >> j) & 1) << pos_rest[j];
        const double2 a = psi[s ^ xm], b = psi[s];
        const double P = a.x * b.x + a.y * b.y, Q = a.x * b.y - a.y * b.x;
        double v = ny4 == 0 ? P : (ny4 == 1 ? -Q : (ny4 == 2 ? -P : Q));
        return (__popcll((unsigned long long)(s & zy)) & 1) ? -v : v;
    };
    if (m <= 6) {
        // few terms per output: one thread per output
        for (int64_t x = tid; x < n_out; x += kSvThreads) {
            double acc = 0.0;
            for (int64_t r = 0; r < n_rest; ++r) acc += term(x, r);
            outs[I.out_off + x] = acc;
        }
    } else {
        for (int64_t x = 0; x < n_out; ++x) {
            double acc = 0.0;
            for (int64_t r = tid; r < n_rest; r += kSvThreads) acc += term(x, r);
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double t = 0.0;
                for (int w = 0; w < kSvThreads / 64; ++w) t += red[w];
                outs[I.out_off + x] = t;
            }
            __syncthreads();
        }
    }
}

// entries[e] = sum over e's terms t (in order) of coef[t] * outs[term_out[t]]
__global__ __launch_bounds__(256) void k_qt_assemble(const int64_t *__restrict__ start,
                                                     const int64_t *__restrict__ term_out,
                                                     const double *__restrict__ coef, int64_t n_entries,
                                                     const double *__restrict__ outs, double *__restrict__ entries) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_entries; e += (int64_t)gridDim.x * 256) {
        double acc = 0.0;
        for (int64_t t = start[e]; t < start[e + 1]; ++t) acc += coef[t] * outs[term_out[t]];
        entries[e] = acc;
    }
}

}  // namespace

hipError_t launch_sv_eval(const SvInst *insts, int n_insts, const SvOp *ops, double2 *gstate, double *outs,
                          hipStream_t st) {
    if (n_insts <= 0) return hipSuccess;
    constexpr int lds = (1 << kSvLdsQubits) * (int)sizeof(double2);
    static bool configured = false;
    if (!configured) {
        hipError_t e = hipFuncSetAttribute((const void *)k_sv_eval, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        configured = true;
    }
    hipLaunchKernelGGL(k_sv_eval, dim3((unsigned)n_insts), dim3(kSvThreads), lds, st, insts, ops, gstate, outs);
    return hipGetLastError();
}

hipError_t launch_qt_assemble(const int64_t *start, const int64_t *term_out, const double *coef, int64_t n_entries,
                              const double *outs, double *entries, hipStream_t st) {
    if (n_entries <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n_entries + 255) / 256, 4096);
    hipLaunchKernelGGL(k_qt_assemble, dim3((unsigned)blocks), dim3(256), 0, st, start, term_out, coef, n_entries,
                       outs, entries);
    return hipGetLastError();
}

}  // namespace kern
}  // namespace htn
