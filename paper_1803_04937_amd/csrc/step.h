// Shared pieces of the stream-collide kernels (step_tg.hip, step_aa.hip):
// memory hints, the residency cap and the dispatch of stochastic rounding.
#pragma once

#include "dispatch.h"
#include "launch.h"

namespace lbm {

// Memory hints of the stream-collide kernels for direction q (x component
// cx): with NT (the streaming cache policy) as set by LBM_NT_FWD_LOADS and
// LBM_NT_FWD_STORES, none otherwise.
template <bool NT>
__host__ __device__ constexpr bool fwd_load_hint(int cx) { return NT && hint_of(LBM_NT_FWD_LOADS, cx); }
template <bool NT>
__host__ __device__ constexpr bool fwd_store_hint(int cx) { return NT && hint_of(LBM_NT_FWD_STORES, cx); }

// Dynamic LDS reserved per stream-collide block (residency cap).
static constexpr unsigned step_lds_bytes(int qn, int dtype, bool gen) {
    return qn == 27 ? LBM_STEP27_LDS_BYTES
           : dtype == LBM_F32 || dtype == LBM_F32_SHIFTED ? LBM_STEP_LDS_BYTES_4B
           : gen && dtype != LBM_F64 ? LBM_STEP_LDS_BYTES_GEN16
                                     : LBM_STEP_LDS_BYTES;
}

}  // namespace lbm

// Stochastic rounding exists for the 16-bit formats only.
#define LBM_DISPATCH_SR(BODY)                                                       \
    if constexpr (DT == LBM_F16_SHIFTED || DT == LBM_BF16_SHIFTED) {                \
        if (sr) { constexpr bool SR = true; BODY; }                                 \
        else { constexpr bool SR = false; BODY; }                                   \
    } else { constexpr bool SR = false; BODY; }
