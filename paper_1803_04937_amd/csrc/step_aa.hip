// AA-pattern stream-collide: one buffer updated in place, the same fused
// update as the two-grid step (Sec. 2.3), alternating a step on the
// neighbours' slots with a step on the cell's own slots.
#include "step.h"

namespace lbm {

// ---------------------------------------------------------------------------
// AA pattern, one buffer updated in place.
//   neighbour step: g_q(x) = A[qbar][x - c_q] (A[q][x] if x - c_q is not
//                   fluid); f*_q(x) -> A[q][x + c_q] (A[qbar][x] if x + c_q
//                   is not fluid).
//   local step:     g_q(x) = A[q][x];  f*_q(x) -> A[qbar][x].
// Every slot a cell reads is written by the same cell, so the in-place
// update is race-free.
// ---------------------------------------------------------------------------
template <int QN, int DT, int EQ, bool GEN, int CO, bool SR, bool NT>
__global__ __launch_bounds__(kBlock) void k_step_aa_nb(Geom g, Coll<typename Store<DT>::R> P,
                                                       typename Store<DT>::T *A, uint32_t key) {
    using S = Store<DT>;
    using R = typename S::R;
    using T = typename S::T;
    R d[QN];
    if constexpr (!GEN) {
        // periodic, no mask: planar launch (blockIdx.y = z).  The pushes
        // along x (c_x != 0) would leave each wave's stores one element off
        // the line boundaries; they are stored through LDS instead, as the
        // adjoint's: the writer converts its value and parks it at the block
        // index of the cell x + c_x in its row (wrapped), and after one
        // barrier that cell's thread stores it at its own x, aligned.  A
        // target outside the block is stored directly.  Values parked early
        // also leave the registers (FP32: 72 VGPRs instead of 97).  Only
        // the 4-byte formats park: at 256^3 it took the FP32 neighbour step
        // from 403 to 395 us, while the FP16 one went from 213 to 221 us
        // (227 with 32-bit LDS words), its added instructions and barrier
        // costing more than the aligned stores save; FP64 keeps 3 waves per
        // SIMD either way.
        constexpr bool PARK = sizeof(T) == 4;
        constexpr const XTab &X = QN == 19 ? kXTab19 : kXTab27;
        __shared__ T xs[PARK ? X.n : 1][PARK ? kBlock : 1];
        const int j = threadIdx.x;
        const uint32_t z = blockIdx.y, p = blockIdx.x * kBlock + j;
        const bool valid = p < g.nxy;
        const PlaneHood h = make_plane_hood(valid ? p : 0, z, g);
        if (valid) {
            static_for<QN>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const T *base = A + ((int64_t)h.zp[1 - kC[q].z] * QN + opp(q)) * g.qstride;
                d[q] = S::template load<fwd_load_hint<NT>(kC[q].x)>(
                    at_bytes(base, plane_off<T>(h, q, -1)), 0, (R)wq(QN, q), P.inv_s);
            });
            collide<R, EQ, QN, CO>(d, P);
            SrBits rb{SR ? mix32((z * g.nxy + p) ^ key) : 0u};
            static_for<QN>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr bool H = fwd_store_hint<NT>(kC[q].x);
                const uint32_t bits = SR ? rb.next(q) : 0u;
                // a parked value is converted like a stored one (the same
                // rounding bits) and copied unchanged after the barrier
                auto put = [&](T *o, auto hint) {
                    if constexpr (SR)
                        store_sr<DT, decltype(hint)::value>(o, 0, d[q], P.s, bits);
                    else
                        S::template store<decltype(hint)::value>(o, 0, d[q], (R)wq(QN, q), P.s);
                };
                bool parked = false;
                if constexpr (PARK && kC[q].x != 0) {
                    const int jt = j + h.ox[1 + kC[q].x];
                    if (jt >= 0 && jt < kBlock) {
                        put(&xs[X.rank[q]][jt], std::false_type{});
                        parked = true;
                    }
                }
                if (!parked)
                    put(at_bytes(A + ((int64_t)h.zp[1 + kC[q].z] * QN + q) * g.qstride,
                                 plane_off<T>(h, q, +1)),
                        std::integral_constant<bool, H>{});
            });
        }
        if constexpr (PARK) __syncthreads();
        if (PARK && valid) {
            static_for<QN>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if constexpr (PARK && kC[q].x != 0) {
                    const int jw = j + h.ox[1 - kC[q].x];   // the writer x - c_x
                    if (jw >= 0 && jw < kBlock) {
                        T *o = at_bytes(A + ((int64_t)h.zp[1 + kC[q].z] * QN + q) * g.qstride,
                                        plane_off<T>(h, X.q0[q], +1));
                        st<fwd_store_hint<NT>(0)>(o, xs[X.rank[q]][j]);
                    }
                }
            });
        }
    } else {
        const uint32_t idx = gen_block(g) * kBlock + threadIdx.x;
        if (idx >= g.ncells) return;
        const Hood h = make_hood_links<QN>(idx, g);
        if (link_solid(h.link)) return;
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            bool fl;
            int64_t pos;
            hood_cell<GEN>(h, g, q, -1, fl, pos);
            const typename S::T *p = A + (fl ? opp(q) : q) * g.qstride;
            d[q] = S::template load<fwd_load_hint<NT>(kC[q].x)>(p, fl ? pos : h.pos, (R)wq(QN, q),
                                                                 P.inv_s);
        });
        collide<R, EQ, QN, CO>(d, P);
        SrBits rb{SR ? mix32(idx ^ key) : 0u};
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr bool H = fwd_store_hint<NT>(kC[q].x);
            bool fl;
            int64_t pos;
            hood_cell<GEN>(h, g, q, +1, fl, pos);
            typename S::T *p = A + (fl ? q : opp(q)) * g.qstride;
            if constexpr (SR)
                store_sr<DT, H>(p, fl ? pos : h.pos, d[q], P.s, rb.next(q));
            else
                S::template store<H>(p, fl ? pos : h.pos, d[q], (R)wq(QN, q), P.s);
        });
    }
}

template <int QN, int DT, int EQ, bool GEN, int CO, bool SR, bool NT>
__global__ __launch_bounds__(kBlock) void k_step_aa_loc(Geom g, Coll<typename Store<DT>::R> P,
                                                        typename Store<DT>::T *A, uint32_t key) {
    using S = Store<DT>;
    using R = typename S::R;
    using T = typename S::T;
    R d[QN];
    if constexpr (!GEN) {
        // periodic, no mask: planar launch (blockIdx.y = z)
        const uint32_t z = blockIdx.y, p = blockIdx.x * kBlock + threadIdx.x;
        if (p >= g.nxy) return;
        const uint32_t off = p * (uint32_t)sizeof(T);
        T *plane = A + (int64_t)z * QN * g.qstride;
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            d[q] = S::template load<fwd_load_hint<NT>(0)>(at_bytes(plane + q * g.qstride, off), 0,
                                                          (R)wq(QN, q), P.inv_s);
        });
        collide<R, EQ, QN, CO>(d, P);
        SrBits rb{SR ? mix32((z * g.nxy + p) ^ key) : 0u};
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr bool H = fwd_store_hint<NT>(0);
            T *o = at_bytes(plane + opp(q) * g.qstride, off);
            if constexpr (SR)
                store_sr<DT, H>(o, 0, d[q], P.s, rb.next(q));
            else
                S::template store<H>(o, 0, d[q], (R)wq(QN, q), P.s);
        });
    } else {
        const uint32_t idx = gen_block(g) * kBlock + threadIdx.x;
        if (idx >= g.ncells) return;
        if (g.links != nullptr && link_solid(g.links[idx])) return;
        const int64_t pos = cell_pos(idx, g);
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            d[q] = S::template load<fwd_load_hint<NT>(0)>(A + q * g.qstride, pos, (R)wq(QN, q),
                                                          P.inv_s);
        });
        collide<R, EQ, QN, CO>(d, P);
        SrBits rb{SR ? mix32(idx ^ key) : 0u};
        static_for<QN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr bool H = fwd_store_hint<NT>(0);
            if constexpr (SR)
                store_sr<DT, H>(A + opp(q) * g.qstride, pos, d[q], P.s, rb.next(q));
            else
                S::template store<H>(A + opp(q) * g.qstride, pos, d[q], (R)wq(QN, q), P.s);
        });
    }
}

hipError_t launch_step_aa(const Geom &g, int qn, int dtype, int eq, int co, bool gen,
                          bool sr, bool nt, uint32_t key, bool neighbor, const CollBoth &P,
                          void *A, hipStream_t st) {
    gen = gen || !planar_ok(g);   // as in launch_step_tg
    const dim3 grid = gen ? dim3(gen_blocks(g)) : plane_grid(g), block(kBlock);
    if (grid.x == 0) return hipSuccess;   // every cell solid
    LBM_DISPATCH_DT(dtype, LBM_DISPATCH_EQ(eq, LBM_DISPATCH_GEN(gen, LBM_DISPATCH_CO(
        LBM_DISPATCH_SR(LBM_DISPATCH_NT({
        using T = typename Store<DT>::T;
        // the periodic neighbour step's LDS for the parked x-pushes counts
        // against the block's residency cap
        const unsigned parked =
            GEN || sizeof(T) != 4 ? 0u : (QN == 19 ? 10u : 18u) * kBlock * 4u;
        const unsigned cap = step_lds_bytes(QN, DT, GEN);
        if (neighbor)
            hipLaunchKernelGGL((k_step_aa_nb<QN, DT, EQ, GEN, CO, SR, NT>), grid, block,
                               cap > parked ? cap - parked : 0u, st, g, pick<DT>(P), (T *)A, key);
        else
            hipLaunchKernelGGL((k_step_aa_loc<QN, DT, EQ, GEN, CO, SR, NT>), grid, block,
                               step_lds_bytes(QN, DT, GEN), st, g, pick<DT>(P), (T *)A, key);
    }))))));
    return hipGetLastError();
}


}  // namespace lbm
