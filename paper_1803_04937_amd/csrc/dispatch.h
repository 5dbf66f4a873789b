// Run-time to compile-time dispatch of the kernel templates.  Each macro
// opens one scope per case with a constexpr of the case's value and expands
// BODY there; the enclosing function returns hipErrorInvalidValue for an
// unknown storage type.
#pragma once

#define LBM_DISPATCH_DT(dtype, BODY)                                  \
    switch (dtype) {                                                  \
    case LBM_F64: { constexpr int DT = LBM_F64; BODY; } break;                 \
    case LBM_F32: { constexpr int DT = LBM_F32; BODY; } break;                 \
    case LBM_F32_SHIFTED: { constexpr int DT = LBM_F32_SHIFTED; BODY; } break; \
    case LBM_F16_SHIFTED: { constexpr int DT = LBM_F16_SHIFTED; BODY; } break; \
    case LBM_BF16_SHIFTED: { constexpr int DT = LBM_BF16_SHIFTED; BODY; } break; \
    default: return hipErrorInvalidValue;                             \
    }

// D3Q27 has one equilibrium (the standard form, Sec. 3.1).
#define LBM_DISPATCH_EQ(eq, BODY)                                                              \
    if (qn == 27) { constexpr int QN = 27; constexpr int EQ = LBM_EQ_STANDARD; BODY; }         \
    else if (eq == LBM_EQ_IMPROVED) { constexpr int QN = 19; constexpr int EQ = LBM_EQ_IMPROVED; BODY; } \
    else if (eq == LBM_EQ_IMPROVED3) { constexpr int QN = 19; constexpr int EQ = LBM_EQ_IMPROVED3; BODY; } \
    else { constexpr int QN = 19; constexpr int EQ = LBM_EQ_STANDARD; BODY; }

// MRT exists for D3Q19 only.
#define LBM_DISPATCH_MRT(BODY)                                          \
    if constexpr (QN == 19) {                                           \
        if (mrt) { constexpr bool MRT = true; BODY; }                   \
        else { constexpr bool MRT = false; BODY; }                      \
    } else { constexpr bool MRT = false; BODY; }

#define LBM_DISPATCH_Q(BODY)                              \
    if (qn == 27) { constexpr int QN = 27; BODY; }        \
    else { constexpr int QN = 19; BODY; }

#define LBM_DISPATCH_GEN(gen, BODY)                      \
    if (gen) { constexpr bool GEN = true; BODY; }        \
    else { constexpr bool GEN = false; BODY; }

// Non-temporal hints on (streaming) or off (cache-resident lattices).
#define LBM_DISPATCH_NT(BODY)                             \
    if (nt) { constexpr bool NT = true; BODY; }           \
    else { constexpr bool NT = false; BODY; }

// Boundary handling of the two-grid stream-collide kernel (kGen*).
#define LBM_DISPATCH_GEN3(gen, BODY)                                         \
    if (gen == kGenOpen) { constexpr int GEN = kGenOpen; BODY; }             \
    else if (gen == kGenWalls) { constexpr int GEN = kGenWalls; BODY; }      \
    else if (gen == kGenWallsPlanar) { constexpr int GEN = kGenWallsPlanar; BODY; } \
    else if (gen == kGenOpenPlanar) { constexpr int GEN = kGenOpenPlanar; BODY; } \
    else { constexpr int GEN = kGenPeriodic; BODY; }

// Collision operator of the stream-collide kernels (kCo*); MRT and KBC exist
// for D3Q19 only.
#define LBM_DISPATCH_CO(BODY)                                               \
    if constexpr (QN == 19) {                                               \
        if (co == kCoMrt) { constexpr int CO = kCoMrt; BODY; }              \
        else if (co == kCoKbc) { constexpr int CO = kCoKbc; BODY; }         \
        else { constexpr int CO = kCoPair; BODY; }                          \
    } else { constexpr int CO = kCoPair; BODY; }
