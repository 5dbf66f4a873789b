// Device-side building blocks of the D3Q19 / D3Q27 stream-collide library
// (gfx950).
//
// Lattices: D3Q19 and D3Q27 (Sec. 2.3), direction order fixed by
// include/lbm.h (D3Q27 = the 19 D3Q19 directions followed by the 8 corners).
// Arithmetic is done in "shifted" variables d_q = f_q - w_q: moments,
// equilibrium and collision are written in d, which keeps FP32 accurate for
// the small deviations of f from the rest state and lets the 16-bit storage
// formats hold s (f - w) directly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "lbm.h"

namespace lbm {

constexpr int kQMax = 27;     // D3Q27
constexpr int kBlock = 256;   // threads per block for every cell kernel

// ---------------------------------------------------------------------------
// Velocity sets (Sec. 2.3).  Opposite pairs are (2k-1, 2k), k = 1..9 for
// D3Q19 and k = 1..13 for D3Q27.
// ---------------------------------------------------------------------------
struct Vec3i {
    int x, y, z;
};
constexpr Vec3i kC[kQMax] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},
    {1, -1, -1},
};
__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
// D3Q19 weights: 1/3, 1/18, 1/36.
__host__ __device__ constexpr double weight(int q) {
    return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
// Weights of the QN-direction stencil; D3Q27: 8/27, 2/27, 1/54, 1/216.
__host__ __device__ constexpr double wq(int qn, int q) {
    return qn == 19 ? weight(q)
                    : (q == 0 ? 8.0 / 27.0
                              : (q <= 6 ? 2.0 / 27.0 : (q <= 18 ? 1.0 / 54.0 : 1.0 / 216.0)));
}

// Directions that shift along x, for kernels that write them x-shifted:
// rank[q] numbers the directions with c_x != 0 (-1 for the others), and
// q0[q] is the direction (0, c_y, c_z) that keeps q's row shift.
struct XTab {
    int n;
    int rank[kQMax];
    int q0[kQMax];
};
constexpr XTab make_xtab(int qn) {
    XTab t{};
    for (int q = 0; q < qn; ++q) {
        t.rank[q] = kC[q].x != 0 ? t.n++ : -1;
        for (int p = 0; p < qn; ++p)
            if (kC[p].x == 0 && kC[p].y == kC[q].y && kC[p].z == kC[q].z) t.q0[q] = p;
    }
    return t;
}
constexpr XTab kXTab19 = make_xtab(19), kXTab27 = make_xtab(27);
static_assert(kXTab19.n == 10 && kXTab27.n == 18, "x-shifted direction count");

// ---------------------------------------------------------------------------
// Streaming memory access.  Every PDF and adjoint value is read once and
// written once per step, so accesses may carry the non-temporal hint (NT).
// The hint is a template parameter: a run-time choice between a hinted and a
// plain access of the same address is merged by the optimiser into one plain
// access (the hint is lost before the direction loops are unrolled), so each
// instantiation below performs one kind of access only.  Where the hint
// depends on the direction, callers branch between two instantiations on a
// condition that unrolling makes constant.
// ---------------------------------------------------------------------------
// Hint modes per kernel role (build-time tuning): 0 none, 1 only the
// directions with c_x = 0 (aligned in memory), 2 all; the adjoint takes
// 0 or 2.  Measured on MI355X at 256^3: forward loads 1 is best (all loads
// hinted evict lines that the x-neighbours' waves still read; none leaves
// the stream-collide output's lines competing with the next kernel), the
// adjoint is best with every access hinted (aligned-only stores cost the
// following forward step 12 %).  With the cached policy (NT = false) the
// stream-collide kernels take no hint at all.
#ifndef LBM_NT_FWD_LOADS
#define LBM_NT_FWD_LOADS 1
#endif
#ifndef LBM_NT_FWD_STORES
#define LBM_NT_FWD_STORES 2
#endif
#ifndef LBM_NT_ADJ_LOADS
#define LBM_NT_ADJ_LOADS 2
#endif
#ifndef LBM_NT_ADJ_STORES
#define LBM_NT_ADJ_STORES 2
#endif
__host__ __device__ constexpr bool hint_of(int mode, int cx) { return mode == 2 || (mode == 1 && cx == 0); }
// The hint pays only when the data does not fit the 256 MB last-level cache:
// the stream-collide and adjoint kernels take NT = false (every access
// cached) when one step touches at most kCacheResidentBytes, which that
// cache then serves between steps (forward +10 % at 96^3 FP32 and 128^3
// FP16, adjoint +2 % at 96^3; streaming wins clearly from about 320 MB up).
constexpr size_t kCacheResidentBytes = size_t(240) << 20;
// Occupancy (build-time tuning).  LBM_STEP_LDS_BYTES > 0 reserves that much
// dynamic LDS per stream-collide block, which caps the resident blocks per
// CU at floor(160 KiB / bytes) (one 256-thread block = one wave per SIMD).
// Measured on MI355X at 256^3 in the plane-blocked layout, two-grid pull:
//   blocks per CU       8      6      5      4
//   FP32 (TB/s)       6.07   6.25   6.33   6.32
//   shifted FP32      6.29   6.36   6.42   6.42
//   FP16 shifted      6.04   6.21   5.88   5.86
//   BF16 shifted      6.06   6.25   5.98   5.97
//   FP64              6.09   6.09   6.09   6.09  (registers allow 4)
// so 4-byte storage takes 5 blocks (32 KiB) and the others 6 (26.5 KiB);
// the AA steps do not change.
// LBM_ADJ_WAVES_PER_EU > 0 asks the compiler to fit the adjoint kernel into
// that many waves per SIMD, LBM_ADJ_LDS_BYTES caps its resident blocks like
// LBM_STEP_LDS_BYTES.  The FP32 adjoint's registers allow 4 blocks per CU,
// which is best (3: 7 % slower, 2: 32 % slower), so neither is set.
#ifndef LBM_STEP_LDS_BYTES
#define LBM_STEP_LDS_BYTES 27136
#endif
#ifndef LBM_STEP_LDS_BYTES_4B
#define LBM_STEP_LDS_BYTES_4B 32768
#endif
// 16-bit storage on lattices with walls or a mask: these kernels wait for a
// link word before their pulls, and more waves hide that latency.  Uncapped
// (8 blocks) the 768 x 192 x 192 FP16 tube runs its steps 7.5 % faster than
// with 6 (side by side), while the periodic 16-bit kernels keep 6.
#ifndef LBM_STEP_LDS_BYTES_GEN16
#define LBM_STEP_LDS_BYTES_GEN16 0
#endif
// D3Q27 stream-collide: its 84 VGPRs allow 5 blocks per CU.  With the
// planar launch 4 is best (FP32 1.5 % and FP16 1 % faster than 5, measured
// side by side); 3 lost up to 30 % before.
#ifndef LBM_STEP27_LDS_BYTES
#define LBM_STEP27_LDS_BYTES 40960
#endif
#ifndef LBM_ADJ_WAVES_PER_EU
#define LBM_ADJ_WAVES_PER_EU 0
#endif
#ifndef LBM_ADJ_LDS_BYTES
#define LBM_ADJ_LDS_BYTES 0
#endif
#if LBM_ADJ_WAVES_PER_EU > 0
#define LBM_ADJ_OCCUPANCY __attribute__((amdgpu_waves_per_eu(LBM_ADJ_WAVES_PER_EU)))
#else
#define LBM_ADJ_OCCUPANCY
#endif

template <bool NT, typename T>
__device__ __forceinline__ T ld(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st(T *p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
// 16-bit storage goes through its bit pattern.
template <bool NT>
__device__ __forceinline__ _Float16 ld(const _Float16 *p) {
    return __builtin_bit_cast(_Float16, ld<NT>((const uint16_t *)p));
}
template <bool NT>
__device__ __forceinline__ void st(_Float16 *p, _Float16 v) {
    st<NT>((uint16_t *)p, __builtin_bit_cast(uint16_t, v));
}
template <bool NT>
__device__ __forceinline__ __bf16 ld(const __bf16 *p) {
    return __builtin_bit_cast(__bf16, ld<NT>((const uint16_t *)p));
}
template <bool NT>
__device__ __forceinline__ void st(__bf16 *p, __bf16 v) {
    st<NT>((uint16_t *)p, __builtin_bit_cast(uint16_t, v));
}

// ---------------------------------------------------------------------------
// Storage formats.  load() returns d = f - w in the compute type R; store()
// takes d.  s / inv_s are the 16-bit scale and its inverse (powers of two).
// ---------------------------------------------------------------------------
template <int DT>
struct Store;

// Store<DT>: load returns d = f - w (R precision), store takes d; NT selects
// the non-temporal hint.  load_f / store_f move raw f (FP64 and FP32 only).
template <>
struct Store<LBM_F64> {
    using T = double;
    using R = double;
    template <bool NT = true>
    static __device__ __forceinline__ R load(const T *p, int64_t i, R w, R) {
        return ld<NT>(p + i) - w;
    }
    template <bool NT = true>
    static __device__ __forceinline__ void store(T *p, int64_t i, R d, R w, R) {
        st<NT>(p + i, (T)(d + w));
    }
    static __device__ __forceinline__ double load_f(const T *p, int64_t i, double, double) {
        return ld<true>(p + i);
    }
    static __device__ __forceinline__ void store_f(T *p, int64_t i, double f, double, double) {
        st<true>(p + i, f);
    }
};
template <>
struct Store<LBM_F32> {
    using T = float;
    using R = float;
    template <bool NT = true>
    static __device__ __forceinline__ R load(const T *p, int64_t i, R w, R) {
        return ld<NT>(p + i) - w;
    }
    template <bool NT = true>
    static __device__ __forceinline__ void store(T *p, int64_t i, R d, R w, R) {
        st<NT>(p + i, (T)(d + w));
    }
    static __device__ __forceinline__ double load_f(const T *p, int64_t i, double, double) {
        return ld<true>(p + i);
    }
    static __device__ __forceinline__ void store_f(T *p, int64_t i, double f, double, double) {
        st<true>(p + i, (float)f);
    }
};
template <>
struct Store<LBM_F32_SHIFTED> {
    using T = float;
    using R = float;
    template <bool NT = true>
    static __device__ __forceinline__ R load(const T *p, int64_t i, R, R) {
        return ld<NT>(p + i);
    }
    template <bool NT = true>
    static __device__ __forceinline__ void store(T *p, int64_t i, R d, R, R) {
        st<NT>(p + i, d);
    }
};
template <>
struct Store<LBM_F16_SHIFTED> {
    using T = _Float16;
    using R = float;
    template <bool NT = true>
    static __device__ __forceinline__ R load(const T *p, int64_t i, R, R inv_s) {
        return static_cast<float>(ld<NT>(p + i)) * inv_s;
    }
    template <bool NT = true>
    static __device__ __forceinline__ void store(T *p, int64_t i, R d, R, R s) {
        st<NT>(p + i, static_cast<_Float16>(d * s));  // round to nearest even
    }
};
template <>
struct Store<LBM_BF16_SHIFTED> {
    using T = __bf16;
    using R = float;
    template <bool NT = true>
    static __device__ __forceinline__ R load(const T *p, int64_t i, R, R inv_s) {
        return static_cast<float>(ld<NT>(p + i)) * inv_s;
    }
    template <bool NT = true>
    static __device__ __forceinline__ void store(T *p, int64_t i, R d, R, R s) {
        st<NT>(p + i, static_cast<__bf16>(d * s));  // round to nearest even
    }
};

// Compile-time loop over directions: f(std::integral_constant<int, q>) for
// q = 0 .. N-1, so that per-direction template arguments (memory hints) are
// constants.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// Stochastic rounding of the 16-bit formats.  The random bits of the value
// f*_q(x) written by step t are a function of (seed, t, x, q) alone: the same
// logical population gets the same bits in the two-grid and the AA pattern,
// and every run is reproducible.  The cell hash mixes (seed, t, x) with the
// 32-bit finaliser of MurmurHash3 (Appleby), a bijection with full avalanche.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// Key of step t under a seed (host side, once per launch).
inline uint32_t step_key(uint32_t seed, int64_t t) {
    return mix32(seed ^ mix32((uint32_t)t ^ mix32((uint32_t)((uint64_t)t >> 32) + 0x9e3779b9u)));
}

// 16 random bits per direction of one cell, drawn in direction order from
// the cell hash: the rest direction takes its high half; each opposite pair
// (q = 2p+1, 2p+2) advances a xorshift32 generator (Marsaglia 2003, shifts
// 13, 17, 5) once and takes the low and the high half of the new state.
// Only shifts and xors, so the per-cell cost is one hash.
struct SrBits {
    uint32_t r;
    __device__ __forceinline__ uint32_t next(int q) {
        if (q & 1) {
            r ^= r << 13;
            r ^= r >> 17;
            r ^= r << 5;
            return r & 0xffffu;
        }
        return r >> 16;
    }
};

// Round v to the format that keeps the top 23 - DROP bits of the FP32
// mantissa: add DROP uniform random bits below the kept ones and truncate
// toward zero.  The result is the lower or the upper neighbour with
// probabilities proportional to the distance from the other, so its
// expectation is v.  (FP16: DROP = 13 for |v| >= 2^-14, the normal range.)
template <int DROP>
__device__ __forceinline__ float sr_truncate(float v, uint32_t r) {
    constexpr uint32_t mask = (1u << DROP) - 1u;
    const uint32_t b = (__float_as_uint(v) + (r & mask)) & ~mask;
    return __uint_as_float(b);
}

template <int DT, bool NT = true>
__device__ __forceinline__ void store_sr(typename Store<DT>::T *p, int64_t i, float d, float s,
                                         uint32_t r) {
    if constexpr (DT == LBM_F16_SHIFTED)
        st<NT>(p + i, static_cast<_Float16>(sr_truncate<13>(d * s, r)));
    else if constexpr (DT == LBM_BF16_SHIFTED)
        st<NT>(p + i, static_cast<__bf16>(sr_truncate<16>(d * s, r)));
}

// Canonical (FP64) access: f = w + d.  The raw formats override these with
// exact copies.
template <int DT>
__device__ __forceinline__ double load_canonical(const typename Store<DT>::T *p, int64_t i,
                                                 double w, double inv_s) {
    if constexpr (DT == LBM_F64 || DT == LBM_F32) {
        return Store<DT>::load_f(p, i, w, inv_s);
    } else {
        using R = typename Store<DT>::R;
        return w + (double)Store<DT>::load(p, i, (R)w, (R)inv_s);
    }
}
template <int DT>
__device__ __forceinline__ void store_canonical(typename Store<DT>::T *p, int64_t i, double f,
                                                double w, double s) {
    if constexpr (DT == LBM_F64 || DT == LBM_F32) {
        Store<DT>::store_f(p, i, f, w, s);
    } else {
        using R = typename Store<DT>::R;
        Store<DT>::store(p, i, (R)(f - w), (R)w, (R)s);
    }
}

// ---------------------------------------------------------------------------
// Unsigned 32-bit division by a run-time constant (round-up multiplier):
// n / d = (umulhi(n, m) + n) >> l, l = ceil(log2 d), valid for all n < 2^32.
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, m, l;
};
inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.l = l;
    f.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
    return f;
}
__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
#ifdef __HIP_DEVICE_COMPILE__
    uint32_t hi = __umulhi(n, f.m);
#else
    uint32_t hi = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
    return (uint32_t)(((uint64_t)hi + n) >> f.l);
}

// ---------------------------------------------------------------------------
// Geometry shared by all cell kernels.
// ---------------------------------------------------------------------------
// PDF and adjoint buffers are plane-blocked: the Q direction arrays of each
// z-plane are contiguous, element (q, cell) at (z Q + q) qstride + y nx + x,
// i.e. q qstride + pos(cell) with pos(cell) = cell + z zskip.
struct Geom {
    uint32_t ncells, nx, ny, nz, nxy;
    FastDiv div_nx, div_ny, div_nxy;
    int32_t per[3];       // periodic flags
    int64_t qstride;      // elements between consecutive q arrays of one plane
    int64_t zskip;        // Q qstride - nxy
    // Per-cell link words, built by the library from the walls and the solid
    // mask when there is a mask (nullptr: no solid cell; kernels then derive
    // the words of the walls in registers, see make_hood_links):
    // bit q (q < Q) is set when the pull source x - c_q is inside the domain
    // and fluid, bit kSolidBit when the cell itself is solid.  A kernel reads
    // one coalesced word per cell instead of looking up the mask at each
    // neighbour, which would put a dependent mask load in front of every
    // pull and made masked lattices 2.4-4.5 times slower.
    const uint32_t *links;
    // Open x faces (kernels with GEN == kGenOpen): inflow velocity at the
    // inlet cells, device double [3][nz][ny] (caller-owned).
    const double *inlet;
    // Lattices with a mask: the 256-cell blocks that hold at least one fluid
    // cell, ascending (caller-owned, after the link words), and their count;
    // nullptr when every block does.  The stream-collide kernels with walls
    // or a mask, and the adjoint when it leaves solid cells unwritten, run one
    // workgroup per listed block only.
    const uint32_t *active;
    uint32_t nactive;
};

// Slot of this workgroup in a one-dimensional launch.  The dispatcher hands
// workgroup i to XCD i mod 8; the slots are taken in groups of 4 consecutive
// blocks per XCD (workgroups 32 m + 8 t + k take slots 32 m + 4 k + t), so
// that most neighbouring blocks, whose pulls share the cache lines at their
// edges, meet in the same L2 while the whole grid still sweeps memory as one
// front.  The last n mod 32 workgroups keep their own index.
__device__ __forceinline__ uint32_t xcd_slot() {
    const uint32_t b = blockIdx.x;
    if (b >= (gridDim.x & ~31u)) return b;
    const uint32_t w = b & 31u;
    return (b & ~31u) + 4u * (w & 7u) + (w >> 3);
}

// Cell block of a workgroup at a slot of a launch over the active list (or
// over every block when there is none).
__device__ __forceinline__ uint32_t gen_block(const Geom &g, uint32_t slot) {
    return g.active ? g.active[slot] : slot;
}
__device__ __forceinline__ uint32_t gen_block(const Geom &g) { return gen_block(g, xcd_slot()); }
constexpr int kSolidBit = 31;

// Boundary handling of the stream-collide kernels (template parameter GEN):
// fully periodic without a mask (planar launch), walls and / or a mask, and
// walls / mask with an open inlet face at x = -1/2 and outlet face at
// x = nx - 1/2.
constexpr int kGenPeriodic = 0, kGenWalls = 1, kGenOpen = 2;
// kGenWallsPlanar: walls and / or a mask on a lattice whose planes hold a
// whole number of 256-cell blocks, so that each block lies in one z-plane,
// and whose state spans less than 4 GiB: the two-grid step then addresses
// every pull and every bounce-back slot as a 32-bit byte offset from the
// state's base, the plane term uniform over the block.
constexpr int kGenWallsPlanar = 3;
// kGenOpenPlanar: the same with open x faces.
constexpr int kGenOpenPlanar = 4;

// Collision operators of the stream-collide kernels (template parameter CO):
// SRT / TRT in pair form, MRT (Sec. 3.2), KBC (Sec. 3.3).
constexpr int kCoPair = 0, kCoMrt = 1, kCoKbc = 2;
constexpr uint32_t kAllLinks = ~(1u << kSolidBit);   // fluid, every neighbour fluid

__device__ __forceinline__ bool link_solid(uint32_t w) { return (w >> kSolidBit) & 1u; }

// Buffer position of cell idx (add q * qstride for direction q).
__device__ __forceinline__ int64_t cell_pos(uint32_t idx, const Geom &g) {
    return (int64_t)idx + (int64_t)fdiv(idx, g.div_nxy) * g.zskip;
}

// Planar launch of a periodic lattice without a mask: blockIdx.y is z and
// blockIdx.x runs over 256-cell segments of the plane, so z and every plane
// base pointer are uniform over a block, and each access is addressed as a
// scalar base plus a 32-bit in-plane byte offset (the host uses it when
// nz <= kMaxPlanes and a plane's bytes fit 32 bits).  This takes about
// three vector instructions per access off the general 64-bit addressing.
constexpr uint32_t kMaxPlanes = 65535;
struct PlaneHood {
    uint32_t p;            // in-plane index y nx + x
    int32_t ox[3], oy[3];  // in-plane offsets of x - 1, x, x + 1 and y - 1, y, y + 1
    uint32_t zp[3];        // planes z - 1, z, z + 1; uniform
};

__device__ __forceinline__ PlaneHood make_plane_hood(uint32_t p, uint32_t z, const Geom &g) {
    PlaneHood h;
    h.p = p;
    const uint32_t y = fdiv(p, g.div_nx), x = p - y * g.nx;
    const int32_t nx = (int32_t)g.nx, ny = (int32_t)g.ny;
    h.ox[0] = x == 0 ? nx - 1 : -1;
    h.ox[1] = 0;
    h.ox[2] = x == g.nx - 1 ? -(nx - 1) : 1;
    h.oy[0] = y == 0 ? (ny - 1) * nx : -nx;
    h.oy[1] = 0;
    h.oy[2] = y == g.ny - 1 ? -(ny - 1) * nx : nx;
    h.zp[0] = z == 0 ? g.nz - 1 : z - 1;
    h.zp[1] = z;
    h.zp[2] = z == g.nz - 1 ? 0 : z + 1;
    return h;
}

// Link word of an in-plane cell from the walls alone (no mask): bit q when
// x - c_q lies inside the domain.
template <int QN>
__device__ __forceinline__ uint32_t plane_wall_links(uint32_t p, uint32_t z, const Geom &g) {
    const uint32_t y = fdiv(p, g.div_nx), x = p - y * g.nx;
    const bool vx[3] = {x != 0 || g.per[0], true, x != g.nx - 1 || g.per[0]};
    const bool vy[3] = {y != 0 || g.per[1], true, y != g.ny - 1 || g.per[1]};
    const bool vz[3] = {z != 0 || g.per[2], true, z != g.nz - 1 || g.per[2]};
    uint32_t w = 0;
#pragma unroll
    for (int q = 0; q < QN; ++q)
        if (vx[1 - kC[q].x] && vy[1 - kC[q].y] && vz[1 - kC[q].z]) w |= 1u << q;
    return w;
}

// Byte offset of the in-plane neighbour x + s c_q.
template <typename T>
__device__ __forceinline__ uint32_t plane_off(const PlaneHood &h, int q, int s) {
    return (uint32_t)((int32_t)h.p + h.ox[1 + s * kC[q].x] + h.oy[1 + s * kC[q].y]) *
           (uint32_t)sizeof(T);
}

// Element at a byte offset from a (uniform) base pointer.
template <typename T>
__device__ __forceinline__ T *at_bytes(T *base, uint32_t boff) {
    return (T *)((char *)base + boff);
}

// Per-thread neighbourhood of one cell: index offsets of x + dx, y + dy,
// z + dz for dx, dy, dz in {-1, 0, +1} (periodic wrap applied) and whether
// each exists (false beyond a wall).
struct Hood {
    uint32_t idx;
    uint32_t link;        // the cell's link word (kAllLinks when there are none)
    int64_t pos;          // buffer position of the cell
    int32_t ox[3], oy[3], oz[3];
    int64_t pz[3];        // plane term z' zskip of the planes z - 1, z, z + 1
    bool vx[3], vy[3], vz[3];
};

__device__ __forceinline__ Hood make_hood(uint32_t idx, const Geom &g) {
    Hood h;
    h.idx = idx;
    uint32_t row = fdiv(idx, g.div_nx);
    uint32_t x = idx - row * g.nx;
    uint32_t z = fdiv(row, g.div_ny);
    uint32_t y = row - z * g.ny;
    const int32_t nx = (int32_t)g.nx, nxy = (int32_t)g.nxy, ny = (int32_t)g.ny,
                  nz = (int32_t)g.nz;
    h.ox[1] = 0;
    h.oy[1] = 0;
    h.oz[1] = 0;
    h.vx[1] = h.vy[1] = h.vz[1] = true;
    h.ox[0] = x == 0 ? nx - 1 : -1;
    h.ox[2] = x == g.nx - 1 ? -(nx - 1) : 1;
    h.vx[0] = x != 0 || g.per[0];
    h.vx[2] = x != g.nx - 1 || g.per[0];
    h.oy[0] = y == 0 ? (ny - 1) * nx : -nx;
    h.oy[2] = y == g.ny - 1 ? -(ny - 1) * nx : nx;
    h.vy[0] = y != 0 || g.per[1];
    h.vy[2] = y != g.ny - 1 || g.per[1];
    h.oz[0] = z == 0 ? (nz - 1) * nxy : -nxy;
    h.oz[2] = z == g.nz - 1 ? -(nz - 1) * nxy : nxy;
    h.vz[0] = z != 0 || g.per[2];
    h.vz[2] = z != g.nz - 1 || g.per[2];
    h.pz[0] = (int64_t)(z == 0 ? g.nz - 1 : z - 1) * g.zskip;
    h.pz[1] = (int64_t)z * g.zskip;
    h.pz[2] = (int64_t)(z == g.nz - 1 ? 0 : z + 1) * g.zskip;
    h.pos = (int64_t)idx + h.pz[1];
    h.link = kAllLinks;
    return h;
}

// Link word of a cell from the walls alone (no mask): bit q when x - c_q
// lies inside the domain.
template <int QN>
__device__ __forceinline__ uint32_t wall_links(const Hood &h) {
    uint32_t w = 0;
#pragma unroll
    for (int q = 0; q < QN; ++q)
        if (h.vx[1 - kC[q].x] && h.vy[1 - kC[q].y] && h.vz[1 - kC[q].z]) w |= 1u << q;
    return w;
}

// Neighbourhood of a cell of a lattice with walls or solid cells, with its
// link word: loaded when the lattice has a mask, else derived from the walls
// in registers (a load would only add a dependent memory access).
template <int QN>
__device__ __forceinline__ Hood make_hood_links(uint32_t idx, const Geom &g) {
    Hood h = make_hood(idx, g);
    h.link = g.links ? g.links[idx] : wall_links<QN>(h);
    return h;
}

// Cell x + s c_q (s = -1: pull source, s = +1: push target), its buffer
// position, and whether it is fluid (false for walls and solid cells; the
// position is then meaningless).  GEN = false assumes a fully periodic
// domain without solid cells; GEN = true reads the link word of the hood
// (make_hood_links): x + c_q is x - c_qbar.
template <bool GEN>
__device__ __forceinline__ uint32_t hood_cell(const Hood &h, const Geom &g, int q, int s,
                                              bool &fluid, int64_t &pos) {
    const int dx = s * kC[q].x + 1, dy = s * kC[q].y + 1, dz = s * kC[q].z + 1;
    uint32_t c = (uint32_t)((int32_t)h.idx + h.ox[dx] + h.oy[dy] + h.oz[dz]);
    pos = (int64_t)c + h.pz[dz];
    fluid = !GEN || ((h.link >> (s < 0 ? q : opp(q))) & 1u);
    return c;
}

// D3Q19 MRT moment bases (Sec. 3.2) in the pair coordinates of the
// collision: even monomials 1, x^2, y^2, z^2, xy, xz, yz, x^2y^2, x^2z^2,
// y^2z^2 over [rest, 9 pair half-sums] with entries c^e (rest) and 2 c^e
// (pairs), odd monomials x, y, z, x^2y, x^2z, xy^2, y^2z, xz^2, yz^2 over the
// 9 pair half-differences with entries 2 c^e; the relaxation is
// K = M^-1 S M with S the rate of each monomial's order.  The bases and
// their inverses are compile-time constants, so that the adjoint applies
// K^T = M^T S M^-T on their (mostly zero) entries.
struct MrtBasis {
    double me[10][10], mei[10][10], mo[9][9], moi[9][9];
    int ord_e[10], ord_o[9];
};
constexpr int kMrtEven[10][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0},
                                 {1, 0, 1}, {0, 1, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};
constexpr int kMrtOdd[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 1, 0}, {2, 0, 1},
                               {1, 2, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2}};
constexpr double mrt_mono(const int (&e)[3], int q) {
    const int c[3] = {kC[q].x, kC[q].y, kC[q].z};
    double v = 1.0;
    for (int i = 0; i < 3; ++i)
        for (int t = 0; t < e[i]; ++t) v *= c[i];
    return v;
}
// Gauss-Jordan inverse with partial pivoting of an n x n block (n <= 10) of
// a 10-column array, evaluated at compile time.
template <int N>
constexpr void mrt_invert(const double (&a)[N][N], double (&inv)[N][N]) {
    double w[N][2 * N] = {};
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            w[i][j] = a[i][j];
            w[i][N + j] = i == j ? 1.0 : 0.0;
        }
    for (int col = 0; col < N; ++col) {
        int piv = col;
        for (int r = col + 1; r < N; ++r) {
            const double x = w[r][col] < 0 ? -w[r][col] : w[r][col];
            const double y = w[piv][col] < 0 ? -w[piv][col] : w[piv][col];
            if (x > y) piv = r;
        }
        for (int j = 0; j < 2 * N; ++j) {
            const double t = w[col][j];
            w[col][j] = w[piv][j];
            w[piv][j] = t;
        }
        const double d = w[col][col];
        for (int j = 0; j < 2 * N; ++j) w[col][j] = w[col][j] / d;
        for (int r = 0; r < N; ++r) {
            if (r == col) continue;
            const double f = w[r][col];
            for (int j = 0; j < 2 * N; ++j) w[r][j] = w[r][j] - f * w[col][j];
        }
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) inv[i][j] = w[i][N + j];
}
constexpr MrtBasis make_mrt_basis() {
    MrtBasis b{};
    for (int k = 0; k < 10; ++k) {
        b.me[k][0] = mrt_mono(kMrtEven[k], 0);
        for (int p = 0; p < 9; ++p) b.me[k][p + 1] = 2.0 * mrt_mono(kMrtEven[k], 2 * p + 1);
        b.ord_e[k] = kMrtEven[k][0] + kMrtEven[k][1] + kMrtEven[k][2];
    }
    for (int k = 0; k < 9; ++k) {
        for (int p = 0; p < 9; ++p) b.mo[k][p] = 2.0 * mrt_mono(kMrtOdd[k], 2 * p + 1);
        b.ord_o[k] = kMrtOdd[k][0] + kMrtOdd[k][1] + kMrtOdd[k][2];
    }
    mrt_invert<10>(b.me, b.mei);
    mrt_invert<9>(b.mo, b.moi);
    return b;
}
constexpr MrtBasis kMrt19 = make_mrt_basis();

// Rate of a moment of the given order: 1 for the conserved orders 0 and 1.
template <typename R, typename C>
__device__ __forceinline__ R mrt_rate(const C &P, int order) {
    return order <= 1 ? R(1) : order == 2 ? P.wp : order == 3 ? P.w3 : P.w4;
}

// ---------------------------------------------------------------------------
// Collision parameters (host-prepared, compute type R).
// ---------------------------------------------------------------------------
template <typename R>
struct Coll {
    R wp, wm;       // even / odd relaxation rates (equal for SRT)
    R ah[3];        // a / 2
    R fpair[13];    // (1 - wm/2) * 3 w_p (c_p . a) for the pair of q = 2p + 1
    R fraw[13];     // 3 w_p (c_p . a)
    R kappa;        // d omega_minus / d omega (1 for SRT)
    R s, inv_s;     // storage scale
    int compressible;
    // MRT (D3Q19): relaxation matrices K = M^-1 S M of the even part
    // [rest, 9 pair sums] and the odd part [9 pair differences], row-major.
    R ke[100];
    R ko[81];
    R w3, w4;       // MRT rates of the third- and fourth-order moments
    // KBC (D3Q19), with beta = omega / 2: 1/beta, 2 - 1/beta and the upper
    // bound 2 of the stabiliser gamma
    R kbc_ib, kbc_c, kbc_hi;
    R drho_out;     // open faces: outlet density - 1
};

// Moments of shifted PDFs: drho = sum d, j = sum c d.
template <typename R, int QN = 19>
__device__ __forceinline__ void moments(const R (&d)[QN], R &drho, R &jx, R &jy, R &jz) {
    const R p1 = d[1] - d[2], p3 = d[3] - d[4], p5 = d[5] - d[6], p7 = d[7] - d[8],
            p9 = d[9] - d[10], p11 = d[11] - d[12], p13 = d[13] - d[14], p15 = d[15] - d[16],
            p17 = d[17] - d[18];
    jx = (p1 + p7) + (p9 + p11) + p13;
    jy = (p3 + p7) - p9 + (p15 + p17);
    jz = (p5 + p11) - p13 + (p15 - p17);
    drho = ((d[0] + (d[1] + d[2])) + ((d[3] + d[4]) + (d[5] + d[6]))) +
           (((d[7] + d[8]) + (d[9] + d[10])) + ((d[11] + d[12]) + (d[13] + d[14]))) +
           ((d[15] + d[16]) + (d[17] + d[18]));
    if constexpr (QN == 27) {
        // corners (1,1,1), (1,1,-1), (1,-1,1), (-1,1,1) and their opposites
        const R p19 = d[19] - d[20], p21 = d[21] - d[22], p23 = d[23] - d[24],
                p25 = d[25] - d[26];
        jx += (p19 + p21) + (p23 - p25);
        jy += (p19 + p21) + (p25 - p23);
        jz += (p19 - p21) + (p23 + p25);
        drho += ((d[19] + d[20]) + (d[21] + d[22])) + ((d[23] + d[24]) + (d[25] + d[26]));
    }
}

// Even part E_p of the equilibrium polynomial for the pair of q = 2p + 1
// (f^eq_q - w_q = w_q [drho + rho0 (E_p + 3 c_q.u)]).  Standard:
// E = 9/2 (c.u)^2 - 3/2 u^2.  Improved (eq. new_d3q19_equilibrium): axis
// 6 u_a^2 - 3 u^2, edge 9/2 (c.u)^2 - 3/2 (u_a^2 + u_b^2), rest -u^2.
struct Poly {
    // NP = (QN - 1) / 2 pairs; D3Q27 has the standard form only (Sec. 3.1:
    // moment matching on D3Q27 gives it).
    // Cubic odd terms of the third-order improved equilibrium, per pair
    // (f^eq gains w rho0 O3 on q = 2p + 1 and -w rho0 O3 on its opposite):
    // axis a: -9 u_a (u^2 - u_a^2); edge (a, b) with signs (s_a, s_b):
    // 9 (s_a u_a)(s_b u_b)(c . u).  Derived by the moment-matching
    // construction of Sec. 3.2 at O(u^3).
    template <typename R>
    static __device__ __forceinline__ void odd3(R ux, R uy, R uz, const R (&cu)[9], R (&O3)[9]) {
        const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
        O3[0] = R(-9) * ux * (uy2 + uz2);
        O3[1] = R(-9) * uy * (ux2 + uz2);
        O3[2] = R(-9) * uz * (ux2 + uy2);
        const R xy = R(9) * ux * uy, xz = R(9) * ux * uz, yz = R(9) * uy * uz;
        O3[3] = xy * cu[3];
        O3[4] = -xy * cu[4];
        O3[5] = xz * cu[5];
        O3[6] = -xz * cu[6];
        O3[7] = yz * cu[7];
        O3[8] = -yz * cu[8];
    }

    // Gradients with respect to u, for the adjoint.  Even parts:
    // standard 9 (c.u) c - 3 u; improved axis a: 12 u_a e_a - 6 u; improved
    // edge (a, b): 9 (c.u) c - 3 (u_a e_a + u_b e_b).  The rest part's
    // gradient is g0 u with g0 = rest_grad<EQ, NP>().
    template <int EQ, int NP>
    static constexpr double rest_grad() {
        return ((EQ == LBM_EQ_IMPROVED || EQ == LBM_EQ_IMPROVED3) && NP == 9) ? -2.0 : -3.0;
    }
    template <typename R, int EQ, int NP>
    static __device__ __forceinline__ void grad_even(R ux, R uy, R uz, const R (&cu)[NP],
                                                     R (&gE)[NP][3]) {
        const R u[3] = {ux, uy, uz};
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int c[3] = {kC[2 * p + 1].x, kC[2 * p + 1].y, kC[2 * p + 1].z};
            if ((EQ == LBM_EQ_IMPROVED || EQ == LBM_EQ_IMPROVED3) && NP == 9) {
                if (p < 3) {
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        gE[p][b] = R(-6) * u[b] + (b == p ? R(12) * u[b] : R(0));
                } else {
                    const R k = R(9) * cu[p];
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        gE[p][b] = k * R(c[b]) - (c[b] != 0 ? R(3) * u[b] : R(0));
                }
            } else {
                const R k = R(9) * cu[p];
#pragma unroll
                for (int b = 0; b < 3; ++b) gE[p][b] = k * R(c[b]) - R(3) * u[b];
            }
        }
    }
    // Cubic odd terms of the third-order improved equilibrium: axis a,
    // d/du_a = -9 (u^2 - u_a^2), d/du_b = -18 u_a u_b; edge with components
    // c_b = +-1: d/du_b = 9 c_b ((c.u)^2 - u_b^2), 0 along its zero component.
    template <typename R>
    static __device__ __forceinline__ void grad_odd3(R ux, R uy, R uz, const R (&cu)[9],
                                                     R (&gO3)[9][3]) {
        const R u[3] = {ux, uy, uz};
        const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                gO3[p][b] = b == p ? R(-9) * (uu - u[p] * u[p]) : R(-18) * u[p] * u[b];
#pragma unroll
        for (int p = 3; p < 9; ++p) {
            const int c[3] = {kC[2 * p + 1].x, kC[2 * p + 1].y, kC[2 * p + 1].z};
            const R c2 = cu[p] * cu[p];
#pragma unroll
            for (int b = 0; b < 3; ++b)
                gO3[p][b] = c[b] != 0 ? R(9 * c[b]) * (c2 - u[b] * u[b]) : R(0);
        }
    }

    template <typename R, int EQ, int NP = 9>
    static __device__ __forceinline__ void even(R ux, R uy, R uz, R (&cu)[NP], R (&E)[NP], R &E0) {
        const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz, uu = ux2 + uy2 + uz2;
        cu[0] = ux;
        cu[1] = uy;
        cu[2] = uz;
        cu[3] = ux + uy;
        cu[4] = ux - uy;
        cu[5] = ux + uz;
        cu[6] = ux - uz;
        cu[7] = uy + uz;
        cu[8] = uy - uz;
        if constexpr (NP == 13) {
            cu[9] = (ux + uy) + uz;
            cu[10] = (ux + uy) - uz;
            cu[11] = (ux - uy) + uz;
            cu[12] = (uy - ux) + uz;
        }
        if ((EQ == LBM_EQ_IMPROVED || EQ == LBM_EQ_IMPROVED3) && NP == 9) {
            E0 = -uu;
            E[0] = R(6) * ux2 - R(3) * uu;
            E[1] = R(6) * uy2 - R(3) * uu;
            E[2] = R(6) * uz2 - R(3) * uu;
            const R sxy = R(1.5) * (ux2 + uy2), sxz = R(1.5) * (ux2 + uz2),
                    syz = R(1.5) * (uy2 + uz2);
            E[3] = R(4.5) * cu[3] * cu[3] - sxy;
            E[4] = R(4.5) * cu[4] * cu[4] - sxy;
            E[5] = R(4.5) * cu[5] * cu[5] - sxz;
            E[6] = R(4.5) * cu[6] * cu[6] - sxz;
            E[7] = R(4.5) * cu[7] * cu[7] - syz;
            E[8] = R(4.5) * cu[8] * cu[8] - syz;
        } else {
            const R t = R(1.5) * uu;
            E0 = -t;
#pragma unroll
            for (int p = 0; p < NP; ++p) E[p] = R(4.5) * cu[p] * cu[p] - t;
        }
    }
};

// Stream-collide of one cell in shifted variables, in place on d.  With MRT
// (Sec. 3.2, C = -M^-1 S (M f - m_eq)) the even and odd non-equilibrium
// vectors are relaxed with the matrices K_e, K_o instead of the scalars
// omega, omega_minus; the force enters as (I - K_o/2) F.
template <typename R>
__device__ __forceinline__ R recip(R x) {
    if constexpr (sizeof(R) == 4)
        return __builtin_amdgcn_rcpf(x);   // 1 ulp; the stabiliser needs no more
    else
        return R(1) / x;
}

// KBC collision (Sec. 3.3) of one cell in pair coordinates, from the
// non-equilibrium parts ne0 (rest), ne[p] (half pair sums), no[p] (half pair
// differences) of g - f^eq.  The populations split by the 19 kept monomial
// moments of Sec. 3.2 into a kinematic part (orders 0, 1), a shear part s
// (orders 2, 3; the KBC-N4 choice) and a higher-order part h (order 4):
//   f* = g - omega (g - f^eq) - (gamma beta - omega) dh + (1 - omega/2) F,
// beta = omega / 2, which relaxes s at omega and h at gamma beta.  The order-4
// moments x^2y^2, x^2z^2, y^2z^2 of g - f^eq are the sums over the xy, xz,
// yz edge pairs; their dual basis vectors of the 19 moments are 1 at rest,
// -1/2 on the two axes and 1/4 on the four edges of the plane, so dh is even.
// gamma minimises the entropic norm sum (f* - f^eq)^2 / f^eq over
// 0 <= gamma <= 2 (the higher-order part relaxes at most as fast as the shear
// part; rates closer to 2 let rounding noise grow in moments that dh barely
// contains): gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh> clamped to
// [0, 2], 2 when <dh|dh> = 0, with ds = g - f^eq - dk - dh
// and dk the kinematic part (momentum -a/2: -a_i/4 on the axis pair i's odd
// part).  feq0, feqp, feqm: f^eq of the rest, q and qbar directions.
template <typename R>
__device__ __forceinline__ R kbc_kappa(R ne0, const R (&ne)[9], const R (&no)[9], R feq0,
                                       const R (&feqp)[9], const R (&feqm)[9],
                                       const Coll<R> &P, R (&hp)[9], R &h0) {
    const R Hxy = R(2) * (ne[3] + ne[4]), Hxz = R(2) * (ne[5] + ne[6]),
            Hyz = R(2) * (ne[7] + ne[8]);
    h0 = (Hxy + Hxz) + Hyz;
    hp[0] = R(-0.5) * (Hxy + Hxz);
    hp[1] = R(-0.5) * (Hxy + Hyz);
    hp[2] = R(-0.5) * (Hxz + Hyz);
    hp[3] = hp[4] = R(0.25) * Hxy;
    hp[5] = hp[6] = R(0.25) * Hxz;
    hp[7] = hp[8] = R(0.25) * Hyz;
    R sh = (ne0 - h0) * h0 * recip(feq0), hh = h0 * h0 * recip(feq0);
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        const R se = ne[p] - hp[p];
        const R so = p < 3 ? no[p] + R(0.5) * P.ah[p] : no[p];
        const R ip = recip(feqp[p]), im = recip(feqm[p]);
        sh += hp[p] * ((se + so) * ip + (se - so) * im);
        hh += hp[p] * hp[p] * (ip + im);
    }
    R gamma = R(2);
    if (hh != R(0)) gamma = fmin(fmax(P.kbc_ib - P.kbc_c * (sh / hh), R(0)), P.kbc_hi);
    return P.wp * (R(0.5) * gamma - R(1));   // gamma beta - omega
}

template <typename R, int EQ, int QN = 19, int CO = kCoPair>
__device__ __forceinline__ void collide(R (&d)[QN], const Coll<R> &P) {
    constexpr bool MRT = CO == kCoMrt;
    constexpr int NP = (QN - 1) / 2;
    R drho, jx, jy, jz;
    moments<R, QN>(d, drho, jx, jy, jz);
    R rho0 = R(1), inv = R(1);
    if (P.compressible) {
        rho0 = R(1) + drho;
        inv = R(1) / rho0;
    }
    const R ux = (jx + P.ah[0]) * inv, uy = (jy + P.ah[1]) * inv, uz = (jz + P.ah[2]) * inv;
    R cu[NP], E[NP], E0, O[NP];
    Poly::even<R, EQ, NP>(ux, uy, uz, cu, E, E0);
#pragma unroll
    for (int p = 0; p < NP; ++p) O[p] = R(3) * cu[p];
    if constexpr (EQ == LBM_EQ_IMPROVED3 && NP == 9) {
        R O3[9];
        Poly::odd3<R>(ux, uy, uz, cu, O3);
#pragma unroll
        for (int p = 0; p < 9; ++p) O[p] += O3[p];
    }
    const R w0 = R(wq(QN, 0));
    if constexpr (MRT && QN == 19) {
        R ne[10], no[9];
        ne[0] = d[0] - w0 * (drho + rho0 * E0);
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int q = 2 * p + 1;
            const R w = R(wq(QN, q));
            ne[p + 1] = R(0.5) * (d[q] + d[q + 1]) - w * (drho + rho0 * E[p]);
            no[p] = R(0.5) * (d[q] - d[q + 1]) - w * rho0 * O[p] + R(0.5) * P.fraw[p];
        }
        R te[10], to[9];
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            R v = R(0);
#pragma unroll
            for (int j = 0; j < 10; ++j) v += P.ke[10 * i + j] * ne[j];
            te[i] = v;
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            R v = R(0);
#pragma unroll
            for (int j = 0; j < 9; ++j) v += P.ko[9 * i + j] * no[j];
            to[i] = v - P.fraw[i];
        }
        d[0] = d[0] - te[0];
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int q = 2 * p + 1;
            d[q] = d[q] - te[p + 1] - to[p];
            d[q + 1] = d[q + 1] - te[p + 1] + to[p];
        }
        return;
    }
    if constexpr (CO == kCoKbc && QN == 19) {
        R ne[9], no[9], fp[9], fm[9];
        const R ne0 = d[0] - w0 * (drho + rho0 * E0);
        const R feq0 = w0 * ((R(1) + drho) + rho0 * E0);
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int q = 2 * p + 1;
            const R w = R(wq(QN, q));
            ne[p] = R(0.5) * (d[q] + d[q + 1]) - w * (drho + rho0 * E[p]);
            no[p] = R(0.5) * (d[q] - d[q + 1]) - w * rho0 * O[p];
            fp[p] = w * ((R(1) + drho) + rho0 * (E[p] + O[p]));
            fm[p] = w * ((R(1) + drho) + rho0 * (E[p] - O[p]));
        }
        R hp[9], h0;
        const R kap = kbc_kappa<R>(ne0, ne, no, feq0, fp, fm, P, hp, h0);
        d[0] = d[0] - P.wp * ne0 - kap * h0;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int q = 2 * p + 1;
            const R tp = P.wp * ne[p] + kap * hp[p];
            const R tm = P.wp * no[p] - P.fpair[p];
            d[q] = d[q] - tp - tm;
            d[q + 1] = d[q + 1] - tp + tm;
        }
        return;
    }
    d[0] = d[0] - P.wp * (d[0] - w0 * (drho + rho0 * E0));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int q = 2 * p + 1;
        const R w = R(wq(QN, q));
        const R np = R(0.5) * (d[q] + d[q + 1]) - w * (drho + rho0 * E[p]);
        const R nm = R(0.5) * (d[q] - d[q + 1]) - w * rho0 * O[p];
        const R tp = P.wp * np;
        const R tm = P.wm * nm - P.fpair[p];
        d[q] = d[q] - tp - tm;
        d[q + 1] = d[q + 1] - tp + tm;
    }
}

// Adjoint of one cell (incompressible): on entry lam = lam_{t+1}(x), d = the
// gathered shifted PDFs g - w; on exit lam = mu = (d f*/d g)^T lam_{t+1};
// acc += dJ/domega and dJ/da of this cell.
// With L = sum_q lam_q f*_q written in pair form, the relaxation enters only
// through the relaxed even and odd parts of lam: nu0 (rest), nu+_p, nu-_p
// (omega lam+ and omega_minus lam- for SRT/TRT; halves of K_e^T [lam_0,
// lam_q + lam_qbar] and K_o^T [lam_q - lam_qbar] for MRT), and the
// equilibrium through its gradient in u:
//   mu_0 = lam_0 - nu0 + S,  mu_q/qbar = lam_q/qbar - (nu+ +/- nu-) + S +/- c.V
//   S = w_0 nu0 + sum 2 w nu+,  V = w_0 nu0 dE_0/du + sum 2 w (nu+ dE_p/du + nu- dO_p/du).
template <typename R, int EQ, int QN, bool MRT, typename A>
__device__ __forceinline__ void adjoint_cell(const R (&d)[QN], R (&lam)[QN], const Coll<R> &P,
                                             A (&acc)[4]) {
    constexpr int NP = (QN - 1) / 2;
    constexpr bool CUBIC = EQ == LBM_EQ_IMPROVED3 && NP == 9;
    R drho, jx, jy, jz;
    moments<R, QN>(d, drho, jx, jy, jz);
    const R ux = jx + P.ah[0], uy = jy + P.ah[1], uz = jz + P.ah[2];
    R cu[NP], E[NP], E0;
    Poly::even<R, EQ, NP>(ux, uy, uz, cu, E, E0);
    R gE[NP][3];
    Poly::grad_even<R, EQ, NP>(ux, uy, uz, cu, gE);
    R O3[9], gO3[9][3];
    if constexpr (CUBIC) {
        Poly::odd3<R>(ux, uy, uz, cu, O3);
        Poly::grad_odd3<R>(ux, uy, uz, cu, gO3);
    }
    const R g0s = R(Poly::rest_grad<EQ, NP>());
    const R w0 = R(wq(QN, 0));
    R nu0, nup[NP], num[NP];
    [[maybe_unused]] R te[10];   // M_e^-T [lam_0, lam_q + lam_qbar] (MRT)
    if constexpr (MRT && QN == 19) {
        // K^T l = M^T S M^-T l on the constant bases: the zero entries drop
        // out at compile time
        constexpr const MrtBasis &B = kMrt19;
        R le[10], lo[9];
        le[0] = lam[0];
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            le[p + 1] = lam[2 * p + 1] + lam[2 * p + 2];
            lo[p] = lam[2 * p + 1] - lam[2 * p + 2];
        }
        R ts[10], to[9];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            R v = R(0);
#pragma unroll
            for (int i = 0; i < 10; ++i)
                if (B.mei[i][k] != 0.0) v += R(B.mei[i][k]) * le[i];
            te[k] = v;
            ts[k] = mrt_rate<R>(P, B.ord_e[k]) * v;
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            R v = R(0);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (B.moi[i][k] != 0.0) v += R(B.moi[i][k]) * lo[i];
            to[k] = mrt_rate<R>(P, B.ord_o[k]) * v;
        }
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            R v = R(0);
#pragma unroll
            for (int k = 0; k < 10; ++k)
                if (B.me[k][j] != 0.0) v += R(B.me[k][j]) * ts[k];
            if (j == 0)
                nu0 = v;
            else
                nup[j - 1] = R(0.5) * v;
        }
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            R v = R(0);
#pragma unroll
            for (int k = 0; k < 9; ++k)
                if (B.mo[k][j] != 0.0) v += R(B.mo[k][j]) * to[k];
            num[j] = R(0.5) * v;
        }
    } else {
        nu0 = P.wp * lam[0];   // nu+_p, nu-_p follow in the pair loop
    }
    // rest
    const R n0 = d[0] - w0 * (drho + E0);
    R S0 = w0 * nu0;
    R Vx = w0 * nu0 * g0s * ux, Vy = w0 * nu0 * g0s * uy, Vz = w0 * nu0 * g0s * uz;
    R Ap = -lam[0] * n0, Am = R(0);
    R Gx = 0, Gy = 0, Gz = 0;  // force part of dJ/da
    R ne[NP];                  // even non-equilibrium parts (MRT dJ/domega)
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int q = 2 * p + 1;
        const R w = R(wq(QN, q));
        const R cx = R(kC[q].x), cy = R(kC[q].y), cz = R(kC[q].z);
        const R lp = R(0.5) * (lam[q] + lam[q + 1]);
        const R lm = R(0.5) * (lam[q] - lam[q + 1]);
        if constexpr (!(MRT && QN == 19)) {
            nup[p] = P.wp * lp;
            num[p] = P.wm * lm;
        }
        const R np = R(0.5) * (d[q] + d[q + 1]) - w * (drho + E[p]);
        R O = R(3) * cu[p];
        if constexpr (CUBIC) O = O + O3[p];
        const R nm = R(0.5) * (d[q] - d[q + 1]) - w * O;
        S0 += R(2) * w * nup[p];
        const R t2 = R(2) * w * nup[p], t6 = R(6) * w * num[p];
        Vx += t2 * gE[p][0] + t6 * cx;
        Vy += t2 * gE[p][1] + t6 * cy;
        Vz += t2 * gE[p][2] + t6 * cz;
        if constexpr (CUBIC) {
            const R tm = R(2) * w * num[p];
            Vx += tm * gO3[p][0];
            Vy += tm * gO3[p][1];
            Vz += tm * gO3[p][2];
        }
        if constexpr (MRT && QN == 19) {
            // force [lam_q - lam_qbar] . (I - K_o/2) F with F_p = 3 w c.a:
            // d/da_b = 3 w c_b ((lam_q - lam_qbar) - nu-_p) per pair
            ne[p] = np;
            const R gf = R(3) * w * (R(2) * lm - num[p]);
            Gx += gf * cx;
            Gy += gf * cy;
            Gz += gf * cz;
        } else {
            Ap -= R(2) * lp * np;
            Am -= R(2) * lm * (nm + R(0.5) * P.fraw[p]);
            const R l2w = R(2) * w * lm;
            Gx += l2w * cx;
            Gy += l2w * cy;
            Gz += l2w * cz;
        }
    }
    if constexpr (MRT && QN == 19) {
        // only the second-order moments' rate depends on omega:
        // dJ/domega = -le . M_e^-1 E_2 M_e [n0, ne] = -sum over the
        // second-order rows k of (M_e^-T le)_k (M_e [n0, ne])_k
        constexpr const MrtBasis &B = kMrt19;
        R acc0 = R(0);
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            if (B.ord_e[k] != 2) continue;
            R m = B.me[k][0] != 0.0 ? R(B.me[k][0]) * n0 : R(0);
#pragma unroll
            for (int j = 0; j < 9; ++j)
                if (B.me[k][j + 1] != 0.0) m += R(B.me[k][j + 1]) * ne[j];
            acc0 -= te[k] * m;
        }
        acc[0] += (A)acc0;
        acc[1] += (A)(R(0.5) * Vx + Gx);
        acc[2] += (A)(R(0.5) * Vy + Gy);
        acc[3] += (A)(R(0.5) * Vz + Gz);
    } else {
        acc[0] += (A)(Ap + Am * P.kappa);
        const R fm = R(3) * (R(1) - R(0.5) * P.wm);
        acc[1] += (A)(R(0.5) * Vx + fm * Gx);
        acc[2] += (A)(R(0.5) * Vy + fm * Gy);
        acc[3] += (A)(R(0.5) * Vz + fm * Gz);
    }
    lam[0] = lam[0] - nu0 + S0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int q = 2 * p + 1;
        const R cv = R(kC[q].x) * Vx + R(kC[q].y) * Vy + R(kC[q].z) * Vz;
        lam[q] = lam[q] - (nup[p] + num[p]) + S0 + cv;
        lam[q + 1] = lam[q + 1] - (nup[p] - num[p]) + S0 - cv;
    }
}

}  // namespace lbm
