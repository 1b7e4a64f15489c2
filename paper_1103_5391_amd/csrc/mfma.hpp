// MFMA arithmetic traits shared by the block-product kernels (gfx950): operand fragment types,
// packed-operator loads, conversion of FP64 data values to the MFMA input type, and the
// multiply-accumulate of one K chunk.
//
// Inside one MFMA the K index each lane group supplies is free as long as A and B agree, so
// lane group g takes the KPL consecutive indices k = KPL g + t of a chunk.  The operator
// factors are packed in exactly that order (see internal.hpp), so lane (g, r) reads its part
// of a chunk as one contiguous piece.
#pragma once

#include "internal.hpp"

namespace dmrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Global-memory loads (pointers from descriptor tables would otherwise become flat loads).
template <typename T>
__device__ __forceinline__ T ldg(const T* p, int64_t i) {
    return ((const __attribute__((address_space(1))) T*)p)[i];
}
template <typename V>
__device__ __forceinline__ V ldgv(const void* p) {
    return *((const __attribute__((address_space(1))) V*)p);
}

// ---------------------------------------------------------------------------------------
// arithmetic traits
// ---------------------------------------------------------------------------------------
struct PF64 {
    static constexpr int CK = 16, KPL = 4, PER = 1;   // PER: packed pieces per value
    using op_t = double;          // packed operator element
    using ws_t = double;          // workspace element
    using acc_t = d4;
    using frag_t = d4;            // one lane's operand values of one chunk
    __device__ static frag_t from(const double (&v)[KPL]) { return (d4){v[0], v[1], v[2], v[3]}; }
    __device__ static frag_t load_op(const op_t* p) { return ldgv<d4>(p); }
    __device__ static acc_t mma(const frag_t& a, const frag_t& b, acc_t c) {
#pragma unroll
        for (int t = 0; t < 4; ++t) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], c, 0, 0, 0);
        return c;
    }
    __device__ static int row(int g, int v) { return g + 4 * v; }   // result lane layout
};

struct PF32 {
    static constexpr int CK = 16, KPL = 4, PER = 1;
    using op_t = float;
    using ws_t = float;
    using acc_t = f4;
    using frag_t = f4;
    __device__ static frag_t from(const double (&v)[KPL]) {
        return (f4){(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    }
    __device__ static frag_t load_op(const op_t* p) { return ldgv<f4>(p); }
    __device__ static acc_t mma(const frag_t& a, const frag_t& b, acc_t c) {
#pragma unroll
        for (int t = 0; t < 4; ++t) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[t], c, 0, 0, 0);
        return c;
    }
    __device__ static int row(int g, int v) { return 4 * g + v; }
};

// Split bf16 operands: NP pieces per value; the products of total order below NP (pieces
// i + j < NP) are accumulated, smallest orders last.
template <int NP>
struct PSplit {
    static constexpr int CK = 32, KPL = 8, PER = NP;
    using op_t = __bf16;          // packed as KPL values of piece 0, then piece 1, ... per lane
    using ws_t = float;
    using acc_t = f4;
    struct frag_t {
        bf8 p[NP];
    };
    __device__ static frag_t from(const double (&v)[KPL]) {
        frag_t f;
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
            float rest = (float)v[t];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const __bf16 h = (__bf16)rest;
                f.p[q][t] = h;
                rest -= (float)h;
            }
        }
        return f;
    }
    __device__ static frag_t load_op(const op_t* p) {
        frag_t f;
#pragma unroll
        for (int q = 0; q < NP; ++q) f.p[q] = ldgv<bf8>(p + q * KPL);
        return f;
    }
    __device__ static acc_t mma(const frag_t& a, const frag_t& b, acc_t c) {
#pragma unroll
        for (int o = 0; o < NP; ++o)
#pragma unroll
            for (int i = 0; i <= o; ++i)
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[i], b.p[o - i], c, 0, 0, 0);
        return c;
    }
    __device__ static int row(int g, int v) { return 4 * g + v; }
};
using PBF3 = PSplit<2>;
using PBF6 = PSplit<3>;

// Elements of one packed panel chunk per lane (all pieces of a split value) and per chunk.
template <class P>
constexpr int lane_elems() {
    return P::KPL * P::PER;
}
template <class P>
constexpr int chunk_elems() {
    return kPanel * 4 * lane_elems<P>();
}

template <class P>
__device__ __forceinline__ void zero(typename P::acc_t& a) {
#pragma unroll
    for (int v = 0; v < 4; ++v) a[v] = 0;
}

// KPL consecutive data values v[t] = src[base + t] (workspace, zero-padded chunks)
template <class P, typename T>
__device__ __forceinline__ void load_run(const T* src, int64_t base, double (&v)[P::KPL]) {
#pragma unroll
    for (int t = 0; t < P::KPL; ++t) v[t] = (double)ldg(src, base + t);
}
// KPL values src[base + min(k0 + t, K - 1) * stride] (input vector, clamped)
template <class P>
__device__ __forceinline__ void load_clamped(const double* src, int64_t base, int k0, int K,
                                             int64_t stride, double (&v)[P::KPL]) {
#pragma unroll
    for (int t = 0; t < P::KPL; ++t) v[t] = ldg(src, base + (int64_t)min(k0 + t, K - 1) * stride);
}

}  // namespace dmrg
