// Forward kernels around the stream-collide update (which lives in
// step_tg.hip and step_aa.hip): initial state, link words, canonical read-out
// / write-in, moments and reductions.
//
// Update: eq. lb_srt_with_forces (Sec. 2.3) with the Buick forcing term
// F_q = 3 w_q c_q.a, the force-shifted velocity of eq. macroscopic_vel_shift,
// the standard (Sec. 2.2) or improved (Sec. 3.2, eq. new_d3q19_equilibrium)
// equilibrium, half-way bounce-back and periodic wrap (Sec. 5.1).
#include "dispatch.h"
#include "launch.h"
#include "reduce.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------

// Shifted equilibrium f^eq_q - w_q = w_q [drho + rho0 (E + 3 c_q.u)] of all
// QN directions, in FP64.
template <int EQ, int QN>
__device__ __forceinline__ void shifted_feq(double drho, double rho0, double ux, double uy,
                                            double uz, double (&d)[QN]) {
    constexpr int NP = (QN - 1) / 2;
    double cu[NP], E[NP], E0, O[NP];
    Poly::even<double, EQ, NP>(ux, uy, uz, cu, E, E0);
#pragma unroll
    for (int p = 0; p < NP; ++p) O[p] = 3.0 * cu[p];
    if constexpr (EQ == LBM_EQ_IMPROVED3 && NP == 9) {
        double O3[9];
        Poly::odd3<double>(ux, uy, uz, cu, O3);
#pragma unroll
        for (int p = 0; p < 9; ++p) O[p] += O3[p];
    }
    d[0] = wq(QN, 0) * (drho + rho0 * E0);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int q = 2 * p + 1;
        const double w = wq(QN, q);
        d[q] = w * (drho + rho0 * (E[p] + O[p]));
        d[q + 1] = w * (drho + rho0 * (E[p] - O[p]));
    }
}

// Slot of f*_q(x) in a buffer of the given layout.  For kAANeighbor the slot
// lies at x + c_q unless that cell is a wall or solid.
template <bool GEN>
__device__ __forceinline__ void canonical_slot(const Hood &h, const Geom &g, Layout layout,
                                               int q, int &arr, int64_t &pos) {
    if (layout == kDirect) {
        arr = q;
        pos = h.pos;
    } else if (layout == kAALocal) {
        arr = opp(q);
        pos = h.pos;
    } else {
        bool fl;
        int64_t p;
        hood_cell<GEN>(h, g, q, +1, fl, p);
        arr = fl ? q : opp(q);
        pos = fl ? p : h.pos;
    }
}

__device__ __forceinline__ uint32_t cell_index() { return blockIdx.x * kBlock + threadIdx.x; }

__device__ __forceinline__ bool is_solid(const Geom &g, uint32_t idx) {
    return g.links != nullptr && link_solid(g.links[idx]);
}

// ---------------------------------------------------------------------------
// Initial state f = f^eq(rho, u) (no force shift); solid cells f = w.
// Written into A (in the given layout) and, if B != null, into B as well.
// ---------------------------------------------------------------------------
template <int QN, int DT, int EQ>
__global__ __launch_bounds__(kBlock) void k_init(Geom g, int compressible, Layout layout,
                                                 const double *__restrict__ rho,
                                                 const double *__restrict__ u,
                                                 typename Store<DT>::T *A,
                                                 typename Store<DT>::T *B, double s) {
    using S = Store<DT>;
    using R = typename S::R;
    const uint32_t idx = cell_index();
    if (idx >= g.ncells) return;
    double d[QN];
    if (is_solid(g, idx)) {
#pragma unroll
        for (int q = 0; q < QN; ++q) d[q] = 0.0;
    } else {  // shifted equilibrium; written below as w + d (raw) or d (shifted)
        const double r = rho ? rho[idx] : 1.0;
        const double rho0 = compressible ? r : 1.0;
        shifted_feq<EQ, QN>(r - 1.0, rho0, u[idx], u[g.ncells + idx], u[2 * (size_t)g.ncells + idx],
                        d);
    }
    const Hood h = make_hood_links<QN>(idx, g);
#pragma unroll
    for (int q = 0; q < QN; ++q) {
        int arr;
        int64_t pos;
        canonical_slot<true>(h, g, layout, q, arr, pos);
        S::store(A + arr * g.qstride, pos, (R)d[q], (R)wq(QN, q), (R)s);
        if (B) S::store(B + arr * g.qstride, pos, (R)d[q], (R)wq(QN, q), (R)s);
    }
}

// max over fluid cells and q of |f^eq_q - w_q| of the initial state.
template <int QN, int EQ>
__global__ __launch_bounds__(kBlock) void k_init_maxdev(Geom g, int compressible,
                                                        const double *__restrict__ rho,
                                                        const double *__restrict__ u,
                                                        double *partials) {
    const uint32_t idx = cell_index();
    double m[1] = {0.0};
    if (idx < g.ncells && !is_solid(g, idx)) {
        const double r = rho ? rho[idx] : 1.0;
        double d[QN];
        shifted_feq<EQ, QN>(r - 1.0, compressible ? r : 1.0, u[idx], u[g.ncells + idx],
                        u[2 * (size_t)g.ncells + idx], d);
#pragma unroll
        for (int q = 0; q < QN; ++q) m[0] = fmax(m[0], fabs(d[q]));
    }
    block_reduce<1, true>(m, partials + blockIdx.x);
}

// Link words (Geom::links) of a lattice with walls or solid cells, from the
// periodic flags and the caller's mask (nullptr: all fluid).  Built once.
template <int QN>
__global__ __launch_bounds__(kBlock) void k_links(Geom g, const uint8_t *__restrict__ solid,
                                                  uint32_t *__restrict__ links) {
    const uint32_t idx = cell_index();
    if (idx >= g.ncells) return;
    const Hood h = make_hood(idx, g);
    uint32_t w = solid && solid[idx] ? 1u << kSolidBit : 0u;
#pragma unroll
    for (int q = 0; q < QN; ++q) {
        const int dx = 1 - kC[q].x, dy = 1 - kC[q].y, dz = 1 - kC[q].z;
        const bool inside = h.vx[dx] && h.vy[dy] && h.vz[dz];
        const uint32_t c = (uint32_t)((int32_t)idx + h.ox[dx] + h.oy[dy] + h.oz[dz]);
        if (inside && !(solid && solid[c])) w |= 1u << q;
    }
    links[idx] = w;
}

// Whether each 256-cell block holds a fluid cell (for the active list).
__global__ __launch_bounds__(kBlock) void k_block_fluid(Geom g, uint32_t *__restrict__ flags) {
    const uint32_t idx = cell_index();
    const int fluid = idx < g.ncells && !link_solid(g.links[idx]);
    const int any = __syncthreads_or(fluid);
    if (threadIdx.x == 0) flags[blockIdx.x] = any ? 1u : 0u;
}

// ---------------------------------------------------------------------------
// Canonical read-out / write-in (FP64 dense [QN][cells]).
// ---------------------------------------------------------------------------
template <int QN, int DT>
__global__ __launch_bounds__(kBlock) void k_get(Geom g, Layout layout, double inv_s,
                                                const typename Store<DT>::T *__restrict__ A,
                                                double *__restrict__ out) {
    using S = Store<DT>;
    using R = typename S::R;
    const uint32_t idx = cell_index();
    if (idx >= g.ncells) return;
    const bool solid = is_solid(g, idx);
    const Hood h = make_hood_links<QN>(idx, g);
#pragma unroll
    for (int q = 0; q < QN; ++q) {
        double v = wq(QN, q);
        if (!solid) {
            int arr;
            int64_t cell;
            canonical_slot<true>(h, g, layout, q, arr, cell);
            v = load_canonical<DT>(A + arr * g.qstride, cell, wq(QN, q), inv_s);
        }
        out[(size_t)q * g.ncells + idx] = v;
    }
}

// Canonical f*_q at a list of cells: out[k * QN + q].  Indices outside the
// lattice yield NaN (no out-of-range access).
template <int QN, int DT>
__global__ __launch_bounds__(kBlock) void k_sample(Geom g, Layout layout, double inv_s,
                                                   const typename Store<DT>::T *__restrict__ A,
                                                   const int64_t *__restrict__ cells, int64_t n,
                                                   double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t c = cells[k];
    if (c < 0 || c >= (int64_t)g.ncells) {
#pragma unroll
        for (int q = 0; q < QN; ++q) out[k * QN + q] = __builtin_nan("");
        return;
    }
    const uint32_t idx = (uint32_t)c;
    const bool solid = is_solid(g, idx);
    const Hood h = make_hood_links<QN>(idx, g);
#pragma unroll
    for (int q = 0; q < QN; ++q) {
        double v = wq(QN, q);
        if (!solid) {
            int arr;
            int64_t cell;
            canonical_slot<true>(h, g, layout, q, arr, cell);
            v = load_canonical<DT>(A + arr * g.qstride, cell, wq(QN, q), inv_s);
        }
        out[k * QN + q] = v;
    }
}

template <int QN, int DT>
__global__ __launch_bounds__(kBlock) void k_set(Geom g, Layout layout, double s,
                                                const double *__restrict__ in,
                                                typename Store<DT>::T *A) {
    using S = Store<DT>;
    using R = typename S::R;
    const uint32_t idx = cell_index();
    if (idx >= g.ncells) return;
    const bool solid = is_solid(g, idx);
    const Hood h = make_hood_links<QN>(idx, g);
#pragma unroll
    for (int q = 0; q < QN; ++q) {
        if (solid) {
            S::store(A + q * g.qstride, h.pos, (R)0, (R)wq(QN, q), (R)s);
        } else {
            int arr;
            int64_t cell;
            canonical_slot<true>(h, g, layout, q, arr, cell);
            store_canonical<DT>(A + arr * g.qstride, cell, in[(size_t)q * g.ncells + idx],
                                wq(QN, q), s);
        }
    }
}

// rho = sum f*, u = (sum c f* - a/2) / rho0' per cell (FP64), and block
// partials of the FP64 totals of rho and sum c f* over fluid cells.
template <int QN, int DT>
__global__ __launch_bounds__(kBlock) void k_moments(Geom g, Layout layout, double inv_s,
                                                    int compressible, double ahx, double ahy,
                                                    double ahz,
                                                    const typename Store<DT>::T *__restrict__ A,
                                                    double *__restrict__ rho,
                                                    double *__restrict__ u, double *partials) {
    using S = Store<DT>;
    using R = typename S::R;
    const uint32_t idx = cell_index();
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    if (idx < g.ncells) {
        double r = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
        if (!is_solid(g, idx)) {
            const Hood h = make_hood_links<QN>(idx, g);
            double d[QN];
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                int arr;
                int64_t cell;
                canonical_slot<true>(h, g, layout, q, arr, cell);
                d[q] = (double)S::load(A + arr * g.qstride, cell, (R)wq(QN, q), (R)inv_s);
            }
            double drho, jx, jy, jz;
            moments<double, QN>(d, drho, jx, jy, jz);
            r = 1.0 + drho;
            tot[0] = r;
            tot[1] = jx;
            tot[2] = jy;
            tot[3] = jz;
            const double inv = compressible ? 1.0 / r : 1.0;
            ux = (jx - ahx) * inv;
            uy = (jy - ahy) * inv;
            uz = (jz - ahz) * inv;
        }
        if (rho) rho[idx] = r;
        if (u) {
            u[idx] = ux;
            u[g.ncells + idx] = uy;
            u[2 * (size_t)g.ncells + idx] = uz;
        }
    }
    block_reduce<4>(tot, partials + 4 * (size_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Final reduction of block partials (deterministic: fixed fold order).
// ---------------------------------------------------------------------------
template <bool MAX>
__device__ __forceinline__ void fold_chunk(const double *__restrict__ in, uint32_t first,
                                           uint32_t count, int nvals, double (&v)[4]) {
    for (uint32_t i = threadIdx.x; i < count; i += kBlock)
        for (int k = 0; k < nvals; ++k) {
            const double x = in[(size_t)(first + i) * nvals + k];
            v[k] = MAX ? fmax(v[k], x) : v[k] + x;
        }
}

// One pass: block b folds entries [b * kReduceChunk, (b + 1) * kReduceChunk).
__global__ __launch_bounds__(kBlock) void k_reduce_stage(const double *__restrict__ in,
                                                         uint32_t n, int nvals, int op,
                                                         double *__restrict__ out) {
    const uint32_t first = blockIdx.x * kReduceChunk;
    const uint32_t count = min(kReduceChunk, n - first);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    __shared__ double res[4];
    if (op) {
        fold_chunk<true>(in, first, count, nvals, v);
        block_reduce<4, true>(v, res);
    } else {
        fold_chunk<false>(in, first, count, nvals, v);
        block_reduce<4, false>(v, res);
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < nvals; ++k) out[(size_t)blockIdx.x * nvals + k] = res[k];
}

// Last pass (n <= kReduceChunk): one block writes or accumulates out.
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ partials,
                                                     uint32_t nblocks, int nvals, int op,
                                                     double *out, int accumulate) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    __shared__ double res[4];
    if (op) {
        fold_chunk<true>(partials, 0, nblocks, nvals, v);
        block_reduce<4, true>(v, res);
    } else {
        fold_chunk<false>(partials, 0, nblocks, nvals, v);
        block_reduce<4, false>(v, res);
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < nvals; ++k) out[k] = accumulate ? out[k] + res[k] : res[k];
}

// Plain 16-byte-wide copy (checkpoints, and the byte-count reference of the
// profiler runs).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kBlock) void k_copy(const u32x4 *__restrict__ src,
                                                 u32x4 *__restrict__ dst, size_t n16) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_init(const Geom &g, int qn, int dtype, int eq, int compressible, Layout layout,
                       const double *rho, const double *u, void *A, void *B, double s,
                       hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_EQ(eq, {
        using T = typename Store<DT>::T;
        hipLaunchKernelGGL((k_init<QN, DT, EQ>), grid, block, 0, st, g, compressible, layout, rho, u,
                           (T *)A, (T *)B, s);
    }));
    return hipGetLastError();
}

hipError_t launch_init_maxdev(const Geom &g, int qn, int eq, int compressible, const double *rho,
                              const double *u, const Scratch &sc, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    LBM_DISPATCH_EQ(eq, {
        hipLaunchKernelGGL((k_init_maxdev<QN, EQ>), grid, block, 0, st, g, compressible, rho, u,
                           sc.partials);
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(sc, cell_blocks(g), 1, 1, sc.result, false, st);
}

hipError_t launch_links(const Geom &g, int qn, const uint8_t *solid, uint32_t *links,
                        hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    if (qn == 27)
        hipLaunchKernelGGL((k_links<27>), grid, block, 0, st, g, solid, links);
    else
        hipLaunchKernelGGL((k_links<19>), grid, block, 0, st, g, solid, links);
    return hipGetLastError();
}

hipError_t launch_block_fluid(const Geom &g, uint32_t *flags, hipStream_t st) {
    hipLaunchKernelGGL(k_block_fluid, dim3(cell_blocks(g)), dim3(kBlock), 0, st, g, flags);
    return hipGetLastError();
}

hipError_t launch_get(const Geom &g, int qn, int dtype, Layout layout, double inv_s, const void *A,
                      double *out, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_Q({
        using T = typename Store<DT>::T;
        hipLaunchKernelGGL((k_get<QN, DT>), grid, block, 0, st, g, layout, inv_s, (const T *)A,
                           out);
    }));
    return hipGetLastError();
}

hipError_t launch_sample(const Geom &g, int qn, int dtype, Layout layout, double inv_s,
                         const void *A, const int64_t *cells, int64_t n, double *out,
                         hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((uint32_t)((n + kBlock - 1) / kBlock)), block(kBlock);
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_Q({
        using T = typename Store<DT>::T;
        hipLaunchKernelGGL((k_sample<QN, DT>), grid, block, 0, st, g, layout, inv_s,
                           (const T *)A, cells, n, out);
    }));
    return hipGetLastError();
}

hipError_t launch_set(const Geom &g, int qn, int dtype, Layout layout, double s, const double *in,
                      void *A, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_Q({
        using T = typename Store<DT>::T;
        hipLaunchKernelGGL((k_set<QN, DT>), grid, block, 0, st, g, layout, s, in, (T *)A);
    }));
    return hipGetLastError();
}

hipError_t launch_moments(const Geom &g, int qn, int dtype, Layout layout, double inv_s,
                          int compressible, const double ah[3], const void *A, double *rho,
                          double *u, const Scratch &sc, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_Q({
        using T = typename Store<DT>::T;
        hipLaunchKernelGGL((k_moments<QN, DT>), grid, block, 0, st, g, layout, inv_s,
                           compressible, ah[0], ah[1], ah[2], (const T *)A, rho, u, sc.partials);
    }));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(sc, cell_blocks(g), 4, 0, sc.result, false, st);
}

hipError_t launch_finalize(const Scratch &sc, uint32_t nblocks, int nvals, int op, double *out,
                           bool accumulate, hipStream_t st) {
    const double *src = sc.partials;
    uint32_t n = nblocks;
    int half = 0;
    while (n > kReduceChunk) {
        const uint32_t m = (n + kReduceChunk - 1) / kReduceChunk;
        double *dst = sc.stage + half * sc.stage_half;
        hipLaunchKernelGGL(k_reduce_stage, dim3(m), dim3(kBlock), 0, st, src, n, nvals, op, dst);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        src = dst;
        n = m;
        half ^= 1;
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, st, src, n, nvals, op, out,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t nbytes, hipStream_t st) {
    if (nbytes % 16) return hipErrorInvalidValue;
    const size_t n16 = nbytes / 16;
    const size_t blocks = (n16 + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_copy, dim3((uint32_t)blocks), dim3(kBlock), 0, st, (const u32x4 *)src,
                       (u32x4 *)dst, n16);
    return hipGetLastError();
}

}  // namespace lbm
