// Buffer-instruction access to the state for the fused sweeps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbcg {

// State buffers are read and written with buffer instructions: the byte
// offset of a pair splits into a per-thread part (the node's column), fixed
// over a sweep, and a part uniform over the wave (the plane or row of the
// sweep, direction i) that travels in a scalar register, so a population
// costs no address arithmetic.  The host keeps a state buffer below 4 GiB; the resource's
// size also bounds every access (an offset past it reads 0 and drops a
// write).
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit dword buffer (gfx9 family)
constexpr int kNonTemporal = 2;         // cache-policy bit of a streaming store

template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_rsrc(const S *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(p), (short)0, int(bytes), kRsrcWord3);
}

template <typename P2>
__device__ __forceinline__ P2 load_pair(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(P2) == 8)
        return __builtin_bit_cast(P2, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0));
    else
        return __builtin_bit_cast(P2, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
}

template <typename P2>
__device__ __forceinline__ void store_pair(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, P2 v) {
    constexpr int pol = kNonTemporal;  // the new state is not read again in this step
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(P2) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, int(voff), int(soff), pol);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, int(voff), int(soff), pol);
}

// Wait until every vector memory operation of the wave has completed
// (s_waitcnt vmcnt(0); the export and LDS/scalar counters are left alone).
__device__ __forceinline__ void wait_memory() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// A value the caller knows to be the same in every lane (the plane or row of
// a sweep), marked so for the compiler: buffer offsets derived from it then
// stay in scalar registers.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

}  // namespace lbcg
