// Adjoint kernels: the exact transpose of one two-grid pull step, the
// objective seeds and the initial-state VJP.  The adjoint is not in the
// paper; it differentiates the discrete update of eq. lb_srt_with_forces
// (Sec. 2.3) in the incompressible form (rho0 = 1), for every stencil,
// equilibrium and collision of the forward path: D3Q19 and D3Q27, the
// equilibria of Sec. 2.2 / Sec. 3.2 (also at third order), SRT, TRT and
// MRT.
#include "dispatch.h"
#include "launch.h"
#include "reduce.h"

namespace lbm {

template <int LT>
struct Lam;
template <>
struct Lam<LBM_F64> {
    using T = double;
};
template <>
struct Lam<LBM_F32> {
    using T = float;
};

// One adjoint step.  Per fluid cell x: gather g as the forward pull, load
// lam_{t+1}(x), mu = J_C^T lam_{t+1}, push mu_r to lam_t[r][x - c_r] (or to
// lam_t[rbar][x] when x - c_r is a wall or solid).  Each f_t slot is read by
// exactly one cell in the forward step, so each lam_t slot is written
// exactly once.  Solid cells copy lam through (copy_solid) or are skipped.
//
// Pushes along x would leave every wave's store one element off the
// 256-byte segments of the array, so two waves write parts of the same
// memory sectors.  Those pushes go through LDS instead: the value for slot
// (x - c_r, y - c_ry, z - c_rz) is parked at the block-local index of
// cell (x - c_r, y, z) (the x shift wraps within the row), and after one
// barrier the thread of that cell stores it at its own x, so each store is
// as aligned as the forward's.  A thread reads its parked slot exactly when
// its writer cell (x + c_r, wrapped) lies in the block, is fluid, and
// pulls from a fluid cell: the writer has then filled the slot.  A push
// that cannot be parked (target cell in another block, or bounce-back)
// goes to the writer's own outbox slot and is stored after the barrier.
// The writer loop thus holds no global stores for these directions, which
// keeps its register footprint below that of storing every push directly.
template <int QN, int DT, int LT, int EQ, bool GEN, bool MRT, bool GRAD, bool NT>
__global__ __launch_bounds__(kBlock) LBM_ADJ_OCCUPANCY void k_adjoint(
    Geom g, Coll<typename Store<DT>::R> P, const typename Store<DT>::T *__restrict__ state,
    const typename Lam<LT>::T *__restrict__ lam_next, typename Lam<LT>::T *__restrict__ lam_prev,
    double *partials, int copy_solid) {
    using S = Store<DT>;
    using R = typename S::R;
    using L = typename Lam<LT>::T;
    constexpr const XTab &X = QN == 19 ? kXTab19 : kXTab27;
    // [k][0, kBlock): parked by target cell; [k][kBlock, 2 kBlock): outbox
    __shared__ L xbuf[X.n][2 * kBlock];
    // the block's link words, for the parked-slot checks after the barrier
    __shared__ uint32_t lw[GEN ? kBlock : 1];
    const int j = threadIdx.x;
    // with an active list (solid cells left unwritten) only blocks that hold
    // a fluid cell are launched
    const uint32_t slot = GEN ? xcd_slot() : blockIdx.x;
    const uint32_t idx = gen_block(g, slot) * kBlock + j;
    const bool valid = idx < g.ncells;
    // solid cells exist only where there is a mask (and its link words)
    const uint32_t link = GEN && valid && g.links ? g.links[idx] : kAllLinks;
    if constexpr (GEN) lw[j] = link;
    const bool fluid = valid && !link_solid(link);
    // one hint for every direction: plain unrolled loops suffice
    constexpr bool HL = NT && LBM_NT_ADJ_LOADS != 0, HS = NT && LBM_NT_ADJ_STORES != 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (fluid) {
        Hood h = make_hood(idx, g);
        if (GEN) h.link = g.links ? link : wall_links<QN>(h);
        R d[QN], lam[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            bool fl;
            int64_t pos;
            hood_cell<GEN>(h, g, q, -1, fl, pos);
            const typename S::T *p = state + (fl ? q : opp(q)) * g.qstride;
            d[q] = S::template load<HL>(p, fl ? pos : h.pos, (R)wq(QN, q), P.inv_s);
            lam[q] = (R)ld<HL>(lam_next + q * g.qstride + h.pos);
        }
        adjoint_cell<R, EQ, QN, MRT>(d, lam, P, acc);
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            bool fl;
            int64_t pos;
            hood_cell<GEN>(h, g, q, -1, fl, pos);
            if (kC[q].x != 0) {
                const int jr = j + h.ox[1 - kC[q].x];
                const bool park = fl && jr >= 0 && jr < kBlock;
                xbuf[X.rank[q]][park ? jr : kBlock + j] = (L)lam[q];
            } else {
                L *p = lam_prev + (fl ? q : opp(q)) * g.qstride;
                st<HS>(p + (fl ? pos : h.pos), (L)lam[q]);
            }
        }
    } else if (valid && copy_solid) {
        const int64_t pos = cell_pos(idx, g);
#pragma unroll
        for (int q = 0; q < QN; ++q)
            st<NT>(lam_prev + q * g.qstride + pos, ld<NT>(lam_next + q * g.qstride + pos));
    }
    __syncthreads();
    if (valid) {
        // Rebuild the neighbourhood from an opaque copy of idx, so that the
        // compiler recomputes these few integer terms here instead of
        // keeping the pull positions live through the collision.
        uint32_t idx2 = idx;
        asm volatile("" : "+v"(idx2));
        Hood h = make_hood(idx2, g);
        if (GEN) h.link = g.links ? link : wall_links<QN>(h);
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            if (kC[q].x == 0) continue;
            bool fl;
            int64_t pos;
            // parked slot: the push of writer x + c_x into this cell's x
            const int dw = h.ox[1 + kC[q].x];
            const int jw = j + dw;
            if (jw >= 0 && jw < kBlock) {
                hood_cell<false>(h, g, X.q0[q], -1, fl, pos);   // the position only
                // the writer filled the slot when it is fluid and pulls from a
                // fluid cell in direction q (its link bit q)
                bool filled = true;
                if constexpr (GEN) {
                    if (g.links) {
                        const uint32_t wl = lw[jw];
                        filled = !link_solid(wl) && ((wl >> q) & 1u);
                    } else {   // walls only: the writer exists and its source is inside
                        filled = h.vx[1 + kC[q].x] && h.vy[1 - kC[q].y] && h.vz[1 - kC[q].z];
                    }
                }
                if (filled) st<HS>(lam_prev + q * g.qstride + pos, xbuf[X.rank[q]][j]);
            }
            // outbox: this cell's own push that was not parked
            if (fluid) {
                hood_cell<GEN>(h, g, q, -1, fl, pos);
                const int jr = j + h.ox[1 - kC[q].x];
                if (!(fl && jr >= 0 && jr < kBlock)) {
                    L *p = lam_prev + (fl ? q : opp(q)) * g.qstride;
                    st<HS>(p + (fl ? pos : h.pos), xbuf[X.rank[q]][kBlock + j]);
                }
            }
        }
    }
    if (GRAD) block_reduce<4>(acc, partials + 4 * (size_t)slot);
}

// Planar form of k_adjoint, for lattices whose planes hold a whole number
// of 256-cell blocks (each block inside one z-plane): the same gathers,
// pushes, parking and outbox, with every direction's plane base uniform
// over the block and a 32-bit in-plane byte offset per lane.  Without walls
// or a mask (GEN = false) every access is such a base plus offset.  With
// them, a direction's pull source and its bounce-back slot lie in
// different planes; the launch then requires each field to span less than
// 4 GiB, so that both are 32-bit byte offsets from the field's base and one
// select chooses between them.  The general kernel keeps 64-bit positions
// per lane.
// Value of direction q in plane zq at in-plane byte offset boff.  W32: the
// field spans less than 4 GiB and the plane term joins the 32-bit offset;
// otherwise it stays in a uniform 64-bit base.
template <bool W32, int QN, typename E>
__device__ __forceinline__ E *plane_at(E *base, const Geom &g, uint32_t zq, int q, uint32_t boff) {
    if constexpr (W32)
        return at_bytes(base, (zq * QN + q) * ((uint32_t)g.qstride * (uint32_t)sizeof(E)) + boff);
    else
        return at_bytes(base + (int64_t)(zq * QN + q) * g.qstride, boff);
}

// Pull source x - c_q of direction q, or with GEN and no link (fl false)
// the cell's own slot of opp(q): one select between two 32-bit offsets.
template <bool GEN, int QN, int q, typename E>
__device__ __forceinline__ E *pull_or_own(E *base, const Geom &g, const PlaneHood &h, uint32_t z,
                                          bool fl) {
    if constexpr (GEN) {
        const uint32_t qs = (uint32_t)g.qstride * (uint32_t)sizeof(E);
        const uint32_t pull = (h.zp[1 - kC[q].z] * QN + q) * qs + plane_off<E>(h, q, -1);
        const uint32_t own = (z * QN + opp(q)) * qs + h.p * (uint32_t)sizeof(E);
        return at_bytes(base, fl ? pull : own);
    } else {
        return plane_at<false, QN>(base, g, h.zp[1 - kC[q].z], q, plane_off<E>(h, q, -1));
    }
}

template <int QN, int DT, int LT, int EQ, bool GEN, bool MRT, bool GRAD, bool NT>
__global__ __launch_bounds__(kBlock) LBM_ADJ_OCCUPANCY void k_adjoint_planar(
    Geom g, Coll<typename Store<DT>::R> P, const typename Store<DT>::T *__restrict__ state,
    const typename Lam<LT>::T *__restrict__ lam_next, typename Lam<LT>::T *__restrict__ lam_prev,
    double *partials, int copy_solid) {
    using S = Store<DT>;
    using R = typename S::R;
    using L = typename Lam<LT>::T;
    constexpr const XTab &X = QN == 19 ? kXTab19 : kXTab27;
    constexpr uint32_t LB = sizeof(L);
    __shared__ L xbuf[X.n][2 * kBlock];
    __shared__ uint32_t lw[GEN ? kBlock : 1];
    const int j = threadIdx.x;
    const uint32_t slot = GEN ? xcd_slot() : blockIdx.x;
    const uint32_t c0 = gen_block(g, slot) * kBlock;
    const uint32_t z = fdiv(c0, g.div_nxy);
    const uint32_t p = c0 - z * g.nxy + j;
    uint32_t link = kAllLinks;
    if constexpr (GEN) {
        link = g.links ? g.links[c0 + j] : plane_wall_links<QN>(p, z, g);
        lw[j] = link;
    }
    const bool fluid = !link_solid(link);
    constexpr bool HL = NT && LBM_NT_ADJ_LOADS != 0, HS = NT && LBM_NT_ADJ_STORES != 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // the cell's own lambda does not depend on its link word: with walls or
    // a mask these loads are issued before the word is waited for (solid
    // cells of the block load it too)
    R lam[QN];
    if constexpr (GEN)
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            lam[q] = (R)ld<HL>(plane_at<GEN, QN>(lam_next, g, z, q, p * LB));
        });
    if (fluid) {
        const PlaneHood h = make_plane_hood(p, z, g);
        R d[QN];
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const bool fl = !GEN || ((link >> q) & 1u);
            d[q] = S::template load<HL>(pull_or_own<GEN, QN, q>(state, g, h, z, fl), 0,
                                        (R)wq(QN, q), P.inv_s);
            if constexpr (!GEN) lam[q] = (R)ld<HL>(plane_at<GEN, QN>(lam_next, g, z, q, p * LB));
        });
        adjoint_cell<R, EQ, QN, MRT>(d, lam, P, acc);
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const bool fl = !GEN || ((link >> q) & 1u);
            if constexpr (kC[q].x != 0) {
                const int jr = j + h.ox[1 - kC[q].x];
                const bool park = fl && jr >= 0 && jr < kBlock;
                xbuf[X.rank[q]][park ? jr : kBlock + j] = (L)lam[q];
            } else {
                st<HS>(pull_or_own<GEN, QN, q>(lam_prev, g, h, z, fl), (L)lam[q]);
            }
        });
    } else if (copy_solid) {
#pragma unroll
        for (int q = 0; q < QN; ++q)
            st<NT>(plane_at<GEN, QN>(lam_prev, g, z, q, p * LB),
                   ld<NT>(plane_at<GEN, QN>(lam_next, g, z, q, p * LB)));
    }
    __syncthreads();
    // the in-plane terms again from an opaque copy of p, so that they are
    // recomputed here rather than held through the collision
    uint32_t p2 = p;
    asm volatile("" : "+v"(p2));
    const PlaneHood h = make_plane_hood(p2, z, g);
    static_for<QN>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (kC[q].x != 0) {
            // parked slot: the push of writer x + c_x into this cell's x
            const int jw = j + h.ox[1 + kC[q].x];
            if (jw >= 0 && jw < kBlock) {
                bool filled = true;
                if constexpr (GEN) {
                    const uint32_t wl = lw[jw];
                    filled = !link_solid(wl) && ((wl >> q) & 1u);
                }
                if (filled)
                    st<HS>(plane_at<GEN, QN>(lam_prev, g, h.zp[1 - kC[q].z], q,
                                             plane_off<L>(h, X.q0[q], -1)),
                           xbuf[X.rank[q]][j]);
            }
            // outbox: this cell's own push that was not parked
            if (fluid) {
                const bool fl = !GEN || ((link >> q) & 1u);
                const int jr = j + h.ox[1 - kC[q].x];
                if (!(fl && jr >= 0 && jr < kBlock))
                    st<HS>(pull_or_own<GEN, QN, q>(lam_prev, g, h, z, fl),
                           xbuf[X.rank[q]][kBlock + j]);
            }
        }
    });
    if (GRAD) block_reduce<4>(acc, partials + 4 * (size_t)slot);
}

// Objective of a two-grid state and its seed lam = dJ/df.
//   kind 0: J = 1/2 sum |u|^2,  lam_q = c_q.u,  dJ/da = -1/2 sum u
//   kind 1: J = sum_{x = nx-1} u_x,  lam_q = c_qx there,  dJ/da_x = -1/2 count
// u = sum c f* - a/2 (rho0 = 1).  Solid cells: lam = 0.
template <int QN, int DT, int LT>
__global__ __launch_bounds__(kBlock) void k_objective(Geom g, int kind, double inv_s, double ahx,
                                                      double ahy, double ahz,
                                                      const typename Store<DT>::T *__restrict__ A,
                                                      typename Lam<LT>::T *__restrict__ lam,
                                                      double *partials) {
    using S = Store<DT>;
    using R = typename S::R;
    using L = typename Lam<LT>::T;
    const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (idx < g.ncells) {
        const int64_t pos = cell_pos(idx, g);
        double seed[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) seed[q] = 0.0;
        if (!(g.links && link_solid(g.links[idx]))) {
            double d[QN];
#pragma unroll
            for (int q = 0; q < QN; ++q)
                d[q] = (double)S::load(A + q * g.qstride, pos, (R)wq(QN, q), (R)inv_s);
            double drho, jx, jy, jz;
            moments<double, QN>(d, drho, jx, jy, jz);
            const double ux = jx - ahx, uy = jy - ahy, uz = jz - ahz;
            if (kind == LBM_OBJ_KINETIC_ENERGY) {
                acc[0] = 0.5 * (ux * ux + uy * uy + uz * uz);
                acc[1] = -0.5 * ux;
                acc[2] = -0.5 * uy;
                acc[3] = -0.5 * uz;
#pragma unroll
                for (int q = 0; q < QN; ++q) seed[q] = kC[q].x * ux + kC[q].y * uy + kC[q].z * uz;
            } else {
                const uint32_t row = fdiv(idx, g.div_nx);
                if (idx - row * g.nx == g.nx - 1) {
                    acc[0] = ux;
                    acc[1] = -0.5;
#pragma unroll
                    for (int q = 0; q < QN; ++q) seed[q] = (double)kC[q].x;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < QN; ++q) lam[q * g.qstride + pos] = (L)seed[q];
    }
    block_reduce<4>(acc, partials + 4 * (size_t)blockIdx.x);
}

// grad_u[b][x] = sum_q lam0_q(x) d f^eq_q / d u_b at (rho0 = 1, u_init(x)), in
// pair form: w_0 lam_0 dE_0/du + sum_p w_p [(lam_q + lam_qbar) dE_p/du +
// (lam_q - lam_qbar) dO_p/du], O_p = 3 c.u (+ the cubic terms at third order).
template <int QN, int LT, int EQ>
__global__ __launch_bounds__(kBlock) void k_init_vjp(Geom g, const double *__restrict__ u,
                                                     const typename Lam<LT>::T *__restrict__ lam0,
                                                     double *__restrict__ grad_u) {
    constexpr int NP = (QN - 1) / 2;
    const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= g.ncells) return;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (!(g.links && link_solid(g.links[idx]))) {
        const double ux = u[idx], uy = u[g.ncells + idx], uz = u[2 * (size_t)g.ncells + idx];
        double cu[NP], E[NP], E0, gE[NP][3];
        Poly::even<double, EQ, NP>(ux, uy, uz, cu, E, E0);
        Poly::grad_even<double, EQ, NP>(ux, uy, uz, cu, gE);
        double gO3[9][3];
        if constexpr (EQ == LBM_EQ_IMPROVED3 && NP == 9) Poly::grad_odd3<double>(ux, uy, uz, cu, gO3);
        const double g0 = Poly::rest_grad<EQ, NP>();
        const int64_t pos = cell_pos(idx, g);
        const double l0 = (double)lam0[pos];
        gx = wq(QN, 0) * l0 * g0 * ux;
        gy = wq(QN, 0) * l0 * g0 * uy;
        gz = wq(QN, 0) * l0 * g0 * uz;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int q = 2 * p + 1;
            const double w = wq(QN, q);
            const double ls = (double)lam0[q * g.qstride + pos] +
                              (double)lam0[(q + 1) * g.qstride + pos];
            const double ld = (double)lam0[q * g.qstride + pos] -
                              (double)lam0[(q + 1) * g.qstride + pos];
            double ox = 3.0 * kC[q].x, oy = 3.0 * kC[q].y, oz = 3.0 * kC[q].z;
            if constexpr (EQ == LBM_EQ_IMPROVED3 && NP == 9) {
                ox += gO3[p][0];
                oy += gO3[p][1];
                oz += gO3[p][2];
            }
            gx += w * (ls * gE[p][0] + ox * ld);
            gy += w * (ls * gE[p][1] + oy * ld);
            gz += w * (ls * gE[p][2] + oz * ld);
        }
    }
    grad_u[idx] = gx;
    grad_u[g.ncells + idx] = gy;
    grad_u[2 * (size_t)g.ncells + idx] = gz;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// The adjoint field has the precision of the forward arithmetic: FP64 with
// FP64 storage, FP32 otherwise.
#define LBM_LT_OF(DT) ((DT) == LBM_F64 ? LBM_F64 : LBM_F32)

// One adjoint launch (inside the dispatch below).
#define LBM_ADJ_LAUNCH(KERNEL, G)                                                             \
    hipLaunchKernelGGL((KERNEL<QN, DT, LT, EQ, GEN, MRT, G, NT>), grid, block,                 \
                       LBM_ADJ_LDS_BYTES, st, ga, pick<DT>(P), (const T *)state,               \
                       (const L *)lam_next, (L *)lam_prev, sc.partials, (int)copy_solid)

hipError_t launch_adjoint(const Geom &g, int qn, int dtype, int ltype, int eq, bool mrt, bool gen,
                          bool nt, bool copy_solid, const CollBoth &P, const void *state,
                          const void *lam_next, void *lam_prev, double *grad, const Scratch &sc,
                          hipStream_t st) {
    // Solid cells copy lambda through unless it is left unwritten: only then
    // may the launch skip the blocks without a fluid cell (active list).
    Geom ga = g;
    if (copy_solid || !gen) ga.active = nullptr;
    const dim3 grid(gen_blocks(ga)), block(kBlock);
    const bool want = grad != nullptr;
    if (ltype != (dtype == LBM_F64 ? LBM_F64 : LBM_F32)) return hipErrorInvalidValue;
    if (grid.x == 0) return hipSuccess;   // every cell solid, nothing written
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_EQ(eq, LBM_DISPATCH_GEN(gen, LBM_DISPATCH_MRT(
        LBM_DISPATCH_NT({
        constexpr int LT = LBM_LT_OF(DT);
        using T = typename Store<DT>::T;
        using L = typename Lam<LT>::T;
        const uint64_t elems = (uint64_t)ga.nz * qn * ga.qstride;
        const bool planar = planar_ok(ga) && ga.nxy % kBlock == 0 &&
                            (!GEN || (elems * sizeof(T) <= 0xffffffffull &&
                                      elems * sizeof(L) <= 0xffffffffull));
        if (planar && want) {
            LBM_ADJ_LAUNCH(k_adjoint_planar, true);
        } else if (planar) {
            LBM_ADJ_LAUNCH(k_adjoint_planar, false);
        } else if (want) {
            LBM_ADJ_LAUNCH(k_adjoint, true);
        } else {
            LBM_ADJ_LAUNCH(k_adjoint, false);
        }
    })))));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !want) return e;
    return launch_finalize(sc, grid.x, 4, 0, grad, true, st);
}

#undef LBM_ADJ_LAUNCH

hipError_t launch_objective(const Geom &g, int qn, int dtype, int ltype, int kind, double inv_s,
                            const double ah[3], const void *state, double *out, void *lam,
                            const Scratch &sc, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    if (ltype != (dtype == LBM_F64 ? LBM_F64 : LBM_F32)) return hipErrorInvalidValue;
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_Q({
        constexpr int LT = LBM_LT_OF(DT);
        hipLaunchKernelGGL((k_objective<QN, DT, LT>), grid, block, 0, st, g, kind, inv_s, ah[0],
                           ah[1], ah[2], (const typename Store<DT>::T *)state,
                           (typename Lam<LT>::T *)lam, sc.partials);
    }));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(sc, cell_blocks(g), 4, 0, out, false, st);
}

hipError_t launch_init_vjp(const Geom &g, int qn, int ltype, int eq, const double *u,
                           const void *lam0, double *grad_u, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    if (ltype != LBM_F64 && ltype != LBM_F32) return hipErrorInvalidValue;
    LBM_DISPATCH_EQ(eq, {
        if (ltype == LBM_F64)
            hipLaunchKernelGGL((k_init_vjp<QN, LBM_F64, EQ>), grid, block, 0, st, g, u,
                               (const double *)lam0, grad_u);
        else
            hipLaunchKernelGGL((k_init_vjp<QN, LBM_F32, EQ>), grid, block, 0, st, g, u,
                               (const float *)lam0, grad_u);
    });
    return hipGetLastError();
}

#undef LBM_LT_OF

}  // namespace lbm
