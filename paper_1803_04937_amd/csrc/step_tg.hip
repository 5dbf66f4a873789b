// Two-grid pull stream-collide: the fused update of eq. lb_srt_with_forces
// (Sec. 2.3) with the Buick forcing term F_q = 3 w_q c_q.a, the force-shifted
// velocity of eq. macroscopic_vel_shift, the standard (Sec. 2.2) or improved
// (Sec. 3.2) equilibrium, SRT / TRT / MRT / KBC collision (Sec. 3.2, 3.3),
// half-way bounce-back, periodic wrap (Sec. 5.1) and open x faces (Sec. 5.2).
#include "step.h"

namespace lbm {

// Open x faces (Sec. 5.2: a prescribed inflow, a constant-pressure outflow).
// The gather bounced back every pull from beyond the faces (x is not
// periodic): d_q holds d*_qbar(x).  Inlet (x = 0, c_qx = +1): Ladd's
// moving-wall bounce-back, g_q = f*_qbar(x) + 6 w_q c_q . u_in with u_in the
// inflow velocity of the cell's row.  Outlet (x = nx - 1, c_qx = -1):
// anti-bounce-back (Ginzburg, Verhaeghe and d'Humieres), g_q = -f*_qbar(x) +
// 2 f^eq+_q(rho_out, u_b), f^eq+ the even part of the equilibrium and u_b the
// read-out velocity sum c f*(x) - a/2 of the cell's own stored state.  In
// shifted variables: d_q = -d*_qbar + 2 w_q (rho_out - 1 + E_q(u_b)).
// x, row = z ny + y: the cell's column and row; own(q): the address of the
// cell's own stored f*_q in src.
template <int QN, int DT, int EQ, typename Own>
__device__ __forceinline__ void open_faces(const Geom &g, const Coll<typename Store<DT>::R> &P,
                                           uint32_t x, uint32_t row, Own own,
                                           typename Store<DT>::R (&d)[QN]) {
    using S = Store<DT>;
    using R = typename S::R;
    constexpr int NP = (QN - 1) / 2;
    if (x == 0) {
        const size_t nyz = (size_t)g.ny * g.nz, r = row;
        const R ux = (R)g.inlet[r], uy = (R)g.inlet[nyz + r], uz = (R)g.inlet[2 * nyz + r];
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (kC[q].x == 1)
                d[q] += R(6.0 * wq(QN, q)) * ((ux + R(kC[q].y) * uy) + R(kC[q].z) * uz);
        });
    }
    if (x == g.nx - 1) {
        R jx = R(0), jy = R(0), jz = R(0);
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (q > 0) {
                const R v = S::template load<false>(own(q), 0, (R)wq(QN, q), P.inv_s);
                if constexpr (kC[q].x != 0) jx += R(kC[q].x) * v;
                if constexpr (kC[q].y != 0) jy += R(kC[q].y) * v;
                if constexpr (kC[q].z != 0) jz += R(kC[q].z) * v;
            }
        });
        R cu[NP], E[NP], E0;
        Poly::even<R, EQ, NP>(jx - P.ah[0], jy - P.ah[1], jz - P.ah[2], cu, E, E0);
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (kC[q].x == -1)
                d[q] = R(2.0 * wq(QN, q)) * (P.drho_out + E[(q - 1) / 2]) - d[q];
        });
    }
}

// ---------------------------------------------------------------------------
// Two-grid pull step: dst[q][x] = f*_q(x) from src.
// ---------------------------------------------------------------------------
template <int QN, int DT, int EQ, int GEN, int CO, bool SR, bool NT>
__global__ __launch_bounds__(kBlock) void k_step_tg(Geom g, Coll<typename Store<DT>::R> P,
                                                    const typename Store<DT>::T *__restrict__ src,
                                                    typename Store<DT>::T *__restrict__ dst,
                                                    uint32_t key) {
    using S = Store<DT>;
    using R = typename S::R;
    using T = typename S::T;
    R d[QN];
    if constexpr (GEN == kGenPeriodic) {
        // periodic, no mask: planar launch (blockIdx.y = z)
        const uint32_t z = blockIdx.y, p = blockIdx.x * kBlock + threadIdx.x;
        if (p >= g.nxy) return;
        const PlaneHood h = make_plane_hood(p, z, g);
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const T *base = src + ((int64_t)h.zp[1 - kC[q].z] * QN + q) * g.qstride;
            d[q] = S::template load<fwd_load_hint<NT>(kC[q].x)>(
                at_bytes(base, plane_off<T>(h, q, -1)), 0, (R)wq(QN, q), P.inv_s);
        });
        collide<R, EQ, QN, CO>(d, P);
        SrBits rb{SR ? mix32((z * g.nxy + p) ^ key) : 0u};
        const uint32_t off = p * (uint32_t)sizeof(T);
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr bool H = fwd_store_hint<NT>(0);   // aligned stores
            T *o = at_bytes(dst + ((int64_t)z * QN + q) * g.qstride, off);
            if constexpr (SR)
                store_sr<DT, H>(o, 0, d[q], P.s, rb.next(q));
            else
                S::template store<H>(o, 0, d[q], (R)wq(QN, q), P.s);
        });
    } else if constexpr (GEN == kGenWallsPlanar || GEN == kGenOpenPlanar) {
        // walls and / or a mask, every block inside one z-plane (over the
        // active list when there is one): uniform plane bases, 32-bit
        // in-plane offsets; a missing link reads the cell's own opposite slot
        const uint32_t c0 = gen_block(g) * kBlock;
        const uint32_t z = fdiv(c0, g.div_nxy);
        const uint32_t p = c0 - z * g.nxy + threadIdx.x, idx = c0 + threadIdx.x;
        if (p >= g.nxy) return;
        const uint32_t link = g.links ? g.links[idx] : plane_wall_links<QN>(p, z, g);
        if (link_solid(link)) return;
        const PlaneHood h = make_plane_hood(p, z, g);
        const uint32_t off = p * (uint32_t)sizeof(T);
        // one load per direction, from the pull source or, for a missing
        // link, from the cell's own opposite slot: both as 32-bit byte
        // offsets from the state's base (the launch checks that the state
        // spans less than 4 GiB), so the choice is one select per direction
        const uint32_t qsb = (uint32_t)g.qstride * (uint32_t)sizeof(T);
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const uint32_t pull = (h.zp[1 - kC[q].z] * QN + q) * qsb + plane_off<T>(h, q, -1);
            const uint32_t self = (z * QN + opp(q)) * qsb + off;
            d[q] = S::template load<fwd_load_hint<NT>(kC[q].x)>(
                at_bytes(src, (link >> q) & 1u ? pull : self), 0, (R)wq(QN, q), P.inv_s);
        });
        if constexpr (GEN == kGenOpenPlanar) {
            const uint32_t y = fdiv(p, g.div_nx);
            open_faces<QN, DT, EQ>(g, P, p - y * g.nx, z * g.ny + y,
                                   [&](int q) { return at_bytes(src, (z * QN + q) * qsb + off); },
                                   d);
        }
        collide<R, EQ, QN, CO>(d, P);
        SrBits rb{SR ? mix32(idx ^ key) : 0u};
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr bool H = fwd_store_hint<NT>(0);   // aligned stores
            T *o = at_bytes(dst + ((int64_t)z * QN + q) * g.qstride, off);
            if constexpr (SR)
                store_sr<DT, H>(o, 0, d[q], P.s, rb.next(q));
            else
                S::template store<H>(o, 0, d[q], (R)wq(QN, q), P.s);
        });
    } else {
        const uint32_t idx = gen_block(g) * kBlock + threadIdx.x;
        if (idx >= g.ncells) return;
        const Hood h = make_hood_links<QN>(idx, g);
        if (link_solid(h.link)) return;
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            bool fl;
            int64_t pos;
            hood_cell<true>(h, g, q, -1, fl, pos);
            const T *p = src + (fl ? q : opp(q)) * g.qstride;
            d[q] = S::template load<fwd_load_hint<NT>(kC[q].x)>(p, fl ? pos : h.pos, (R)wq(QN, q),
                                                                 P.inv_s);
        });
        if constexpr (GEN == kGenOpen) {
            const uint32_t row = fdiv(idx, g.div_nx);
            open_faces<QN, DT, EQ>(g, P, idx - row * g.nx, row,
                                   [&](int q) { return src + q * g.qstride + h.pos; }, d);
        }
        collide<R, EQ, QN, CO>(d, P);
        SrBits rb{SR ? mix32(idx ^ key) : 0u};
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr bool H = fwd_store_hint<NT>(0);   // aligned stores
            if constexpr (SR)
                store_sr<DT, H>(dst + q * g.qstride, h.pos, d[q], P.s, rb.next(q));
            else
                S::template store<H>(dst + q * g.qstride, h.pos, d[q], (R)wq(QN, q), P.s);
        });
    }
}


hipError_t launch_step_tg(const Geom &g, int qn, int dtype, int eq, int co, int gen,
                          bool sr, bool nt, uint32_t key, const CollBoth &P, const void *src,
                          void *dst, hipStream_t st) {
    // kGenPeriodic runs the planar launch; lattices it cannot address take the
    // general kernel, which is exact for periodic lattices without a mask too.
    // Walls, masks and open faces take the planar addressing when every
    // 256-cell block lies inside one plane and the state spans less than
    // 4 GiB (its byte offsets then fit 32 bits).
    if (gen == kGenPeriodic && !planar_ok(g)) gen = kGenWalls;
    const uint64_t state_bytes = (uint64_t)g.nz * qn * g.qstride *
                                 (dtype == LBM_F64 ? 8 : dtype == LBM_F16_SHIFTED ||
                                  dtype == LBM_BF16_SHIFTED ? 2 : 4);
    if (planar_ok(g) && g.nxy % kBlock == 0 && state_bytes <= 0xffffffffull) {
        if (gen == kGenWalls) gen = kGenWallsPlanar;
        if (gen == kGenOpen) gen = kGenOpenPlanar;
    }
    const dim3 grid = gen != kGenPeriodic ? dim3(gen_blocks(g)) : plane_grid(g), block(kBlock);
    if (grid.x == 0) return hipSuccess;   // every cell solid
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_EQ(eq, LBM_DISPATCH_GEN3(gen, LBM_DISPATCH_CO(
        LBM_DISPATCH_SR(LBM_DISPATCH_NT({
        using T = typename Store<DT>::T;
        hipLaunchKernelGGL((k_step_tg<QN, DT, EQ, GEN, CO, SR, NT>), grid, block,
                           step_lds_bytes(QN, DT, GEN != kGenPeriodic), st, g, pick<DT>(P),
                           (const T *)src, (T *)dst, key);
    }))))));
    return hipGetLastError();
}


}  // namespace lbm
