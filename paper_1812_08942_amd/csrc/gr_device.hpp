// Device helpers shared by the HIP sources: 16-byte row chunks of test
// vectors (float32 or bfloat16 storage) and the fixed-shape chunk sums.
#pragma once

#include "gr_internal.hpp"

namespace gr {

// ------------------------------------------------------------- chunk I/O
// A chunk is 16 bytes of a row: E = 4 float32 or 8 bfloat16 values.
template <int DT> struct Chunk;
template <> struct Chunk<GR_F32> {
    static constexpr int E = 4;
    __device__ static inline void load(const void* X, int64_t row, int K, int q, float* v) {
        float4 t = *reinterpret_cast<const float4*>((const float*)X + row * K + q * 4);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
    __device__ static inline void store(void* X, int64_t row, int K, int q, const float* v) {
        float4 t = make_float4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<float4*>((float*)X + row * K + q * 4) = t;
    }
};
template <> struct Chunk<GR_BF16> {
    static constexpr int E = 8;
    __device__ static inline void load(const void* X, int64_t row, int K, int q, float* v) {
        uint4 t = *reinterpret_cast<const uint4*>((const uint16_t*)X + row * K + q * 8);
        uint32_t u[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 * i] = __uint_as_float(u[i] << 16);
            v[2 * i + 1] = __uint_as_float(u[i] & 0xffff0000u);
        }
    }
    __device__ static inline void store(void* X, int64_t row, int K, int q, const float* v) {
        uint32_t u[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            u[i] = (uint32_t)f32_to_bf16(v[2 * i]) | ((uint32_t)f32_to_bf16(v[2 * i + 1]) << 16);
        *reinterpret_cast<uint4*>((uint16_t*)X + row * K + q * 8) = make_uint4(u[0], u[1], u[2], u[3]);
    }
};

// Sum of the Q partial sums of a row-group, fixed xor tree over q.
template <int Q>
__device__ inline float qsum(float v) {
#pragma unroll
    for (int off = 1; off < Q; off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <int E>
__device__ inline float chunk_dot(const float* a, const float* b) {
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < E; ++i) s = __fmaf_rn(a[i], b[i], s);
    return s;
}

}  // namespace gr
