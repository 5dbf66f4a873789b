// Adjoint kernels: the exact transpose of one two-grid pull step, the
// objective seeds and the initial-state VJP.  The adjoint is not in the
// paper; it differentiates the discrete update of eq. lb_srt_with_forces
// (Sec. 2.3) with the equilibria of Sec. 2.2 / Sec. 3.2 in the
// incompressible form (rho0 = 1).
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
// exactly once.  Solid cells copy lam through.
template <int DT, int LT, int EQ, bool GEN, bool GRAD>
__global__ __launch_bounds__(kBlock) LBM_ADJ_OCCUPANCY void k_adjoint(
    Geom g, Coll<typename Store<DT>::R> P, const typename Store<DT>::T *__restrict__ state,
    const typename Lam<LT>::T *__restrict__ lam_next, typename Lam<LT>::T *__restrict__ lam_prev,
    double *partials) {
    using S = Store<DT>;
    using R = typename S::R;
    using L = typename Lam<LT>::T;
    const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (idx < g.ncells) {
        if (GEN && g.solid && g.solid[idx]) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                st(lam_prev + q * g.qstride + idx, ld(lam_next + q * g.qstride + idx));
        } else {
            const Hood h = make_hood(idx, g);
            R d[Q], lam[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                bool fl;
                const uint32_t c = hood_cell<GEN>(h, g, q, -1, fl);
                const typename S::T *p = state + (fl ? q : opp(q)) * g.qstride;
                d[q] = S::load(p, fl ? c : idx, (R)weight(q), P.inv_s, nt_load_adj(kC[q].x));
                lam[q] = (R)ld(lam_next + q * g.qstride + idx);
            }
            adjoint_cell<R, EQ>(d, lam, P, acc);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                bool fl;
                const uint32_t c = hood_cell<GEN>(h, g, q, -1, fl);
                L *p = lam_prev + (fl ? q : opp(q)) * g.qstride;
                st(p + (fl ? c : idx), (L)lam[q], nt_store(kC[q].x));
            }
        }
    }
    if (GRAD) block_reduce<4>(acc, partials + 4 * (size_t)blockIdx.x);
}

// Objective of a two-grid state and its seed lam = dJ/df.
//   kind 0: J = 1/2 sum |u|^2,  lam_q = c_q.u,  dJ/da = -1/2 sum u
//   kind 1: J = sum_{x = nx-1} u_x,  lam_q = c_qx there,  dJ/da_x = -1/2 count
// u = sum c f* - a/2 (rho0 = 1).  Solid cells: lam = 0.
template <int DT, int LT>
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
        double seed[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) seed[q] = 0.0;
        if (!(g.solid && g.solid[idx])) {
            double d[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q)
                d[q] = (double)S::load(A + q * g.qstride, idx, (R)weight(q), (R)inv_s);
            double drho, jx, jy, jz;
            moments<double>(d, drho, jx, jy, jz);
            const double ux = jx - ahx, uy = jy - ahy, uz = jz - ahz;
            if (kind == LBM_OBJ_KINETIC_ENERGY) {
                acc[0] = 0.5 * (ux * ux + uy * uy + uz * uz);
                acc[1] = -0.5 * ux;
                acc[2] = -0.5 * uy;
                acc[3] = -0.5 * uz;
#pragma unroll
                for (int q = 0; q < Q; ++q) seed[q] = kC[q].x * ux + kC[q].y * uy + kC[q].z * uz;
            } else {
                const uint32_t row = fdiv(idx, g.div_nx);
                if (idx - row * g.nx == g.nx - 1) {
                    acc[0] = ux;
                    acc[1] = -0.5;
#pragma unroll
                    for (int q = 0; q < Q; ++q) seed[q] = (double)kC[q].x;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) lam[q * g.qstride + idx] = (L)seed[q];
    }
    block_reduce<4>(acc, partials + 4 * (size_t)blockIdx.x);
}

// grad_u[b][x] = sum_q lam0_q(x) d f^eq_q / d u_b at (rho0 = 1, u_init(x)).
template <int LT, int EQ>
__global__ __launch_bounds__(kBlock) void k_init_vjp(Geom g, const double *__restrict__ u,
                                                     const typename Lam<LT>::T *__restrict__ lam0,
                                                     double *__restrict__ grad_u) {
    const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= g.ncells) return;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (!(g.solid && g.solid[idx])) {
        const double ux = u[idx], uy = u[g.ncells + idx], uz = u[2 * (size_t)g.ncells + idx];
        double cu[9], E[9], E0;
        Poly::even<double, EQ>(ux, uy, uz, cu, E, E0);
        const double g0 = (EQ == LBM_EQ_IMPROVED) ? -2.0 : -3.0;
        const double l0 = (double)lam0[idx];
        gx = weight(0) * l0 * g0 * ux;
        gy = weight(0) * l0 * g0 * uy;
        gz = weight(0) * l0 * g0 * uz;
        const double cxp[9] = {1, 0, 0, 1, 1, 1, 1, 0, 0};
        const double cyp[9] = {0, 1, 0, 1, -1, 0, 0, 1, 1};
        const double czp[9] = {0, 0, 1, 0, 0, 1, -1, 1, -1};
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int q = 2 * p + 1;
            const double w = weight(q);
            const double ls = (double)lam0[q * g.qstride + idx] +
                              (double)lam0[(q + 1) * g.qstride + idx];
            const double ld = (double)lam0[q * g.qstride + idx] -
                              (double)lam0[(q + 1) * g.qstride + idx];
            double ex, ey, ez;  // gradient of the even part E_p
            if (EQ == LBM_EQ_IMPROVED && p < 3) {
                ex = -6.0 * ux + (p == 0 ? 12.0 * ux : 0.0);
                ey = -6.0 * uy + (p == 1 ? 12.0 * uy : 0.0);
                ez = -6.0 * uz + (p == 2 ? 12.0 * uz : 0.0);
            } else if (EQ == LBM_EQ_IMPROVED) {
                ex = 9.0 * cu[p] * cxp[p] - (cxp[p] != 0.0 ? 3.0 * ux : 0.0);
                ey = 9.0 * cu[p] * cyp[p] - (cyp[p] != 0.0 ? 3.0 * uy : 0.0);
                ez = 9.0 * cu[p] * czp[p] - (czp[p] != 0.0 ? 3.0 * uz : 0.0);
            } else {
                ex = 9.0 * cu[p] * cxp[p] - 3.0 * ux;
                ey = 9.0 * cu[p] * cyp[p] - 3.0 * uy;
                ez = 9.0 * cu[p] * czp[p] - 3.0 * uz;
            }
            gx += w * (ls * ex + 3.0 * cxp[p] * ld);
            gy += w * (ls * ey + 3.0 * cyp[p] * ld);
            gz += w * (ls * ez + 3.0 * czp[p] * ld);
        }
    }
    grad_u[idx] = gx;
    grad_u[g.ncells + idx] = gy;
    grad_u[2 * (size_t)g.ncells + idx] = gz;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_adjoint(const Geom &g, int dtype, int ltype, int eq, bool gen,
                          const CollBoth &P, const void *state, const void *lam_next,
                          void *lam_prev, double *grad, const Scratch &sc, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
    const bool want = grad != nullptr;
    if (eq != LBM_EQ_STANDARD && eq != LBM_EQ_IMPROVED) return hipErrorInvalidValue;
#define LBM_ADJ(DT, LT, EQ, GEN, GRAD, COLL)                                                     \
    hipLaunchKernelGGL((k_adjoint<DT, LT, EQ, GEN, GRAD>), grid, block, LBM_ADJ_LDS_BYTES, st, g, COLL,          \
                       (const typename Store<DT>::T *)state, (const typename Lam<LT>::T *)lam_next, \
                       (typename Lam<LT>::T *)lam_prev, sc.partials)
#define LBM_ADJ_G(DT, LT, COLL)                                                  \
    do {                                                                         \
        if (eq == LBM_EQ_IMPROVED) {                                             \
            if (gen) { if (want) LBM_ADJ(DT, LT, 1, true, true, COLL); else LBM_ADJ(DT, LT, 1, true, false, COLL); } \
            else { if (want) LBM_ADJ(DT, LT, 1, false, true, COLL); else LBM_ADJ(DT, LT, 1, false, false, COLL); } \
        } else {                                                                 \
            if (gen) { if (want) LBM_ADJ(DT, LT, 0, true, true, COLL); else LBM_ADJ(DT, LT, 0, true, false, COLL); } \
            else { if (want) LBM_ADJ(DT, LT, 0, false, true, COLL); else LBM_ADJ(DT, LT, 0, false, false, COLL); } \
        }                                                                        \
    } while (0)
    if (dtype == LBM_F64 && ltype == LBM_F64) {
        LBM_ADJ_G(LBM_F64, LBM_F64, P.d);
    } else if (ltype == LBM_F32) {
        switch (dtype) {
        case LBM_F32: LBM_ADJ_G(LBM_F32, LBM_F32, P.f); break;
        case LBM_F32_SHIFTED: LBM_ADJ_G(LBM_F32_SHIFTED, LBM_F32, P.f); break;
        case LBM_F16_SHIFTED: LBM_ADJ_G(LBM_F16_SHIFTED, LBM_F32, P.f); break;
        case LBM_BF16_SHIFTED: LBM_ADJ_G(LBM_BF16_SHIFTED, LBM_F32, P.f); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef LBM_ADJ_G
#undef LBM_ADJ
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !want) return e;
    return launch_finalize(sc, cell_blocks(g), 4, 0, grad, true, st);
}

hipError_t launch_objective(const Geom &g, int dtype, int ltype, int kind, double inv_s,
                            const double ah[3], const void *state, double *out, void *lam,
                            const Scratch &sc, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
#define LBM_OBJ(DT, LT)                                                                        \
    hipLaunchKernelGGL((k_objective<DT, LT>), grid, block, 0, st, g, kind, inv_s, ah[0], ah[1], \
                       ah[2], (const typename Store<DT>::T *)state, (typename Lam<LT>::T *)lam,   \
                       sc.partials)
    if (dtype == LBM_F64 && ltype == LBM_F64) {
        LBM_OBJ(LBM_F64, LBM_F64);
    } else if (ltype == LBM_F32) {
        switch (dtype) {
        case LBM_F32: LBM_OBJ(LBM_F32, LBM_F32); break;
        case LBM_F32_SHIFTED: LBM_OBJ(LBM_F32_SHIFTED, LBM_F32); break;
        case LBM_F16_SHIFTED: LBM_OBJ(LBM_F16_SHIFTED, LBM_F32); break;
        case LBM_BF16_SHIFTED: LBM_OBJ(LBM_BF16_SHIFTED, LBM_F32); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef LBM_OBJ
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(sc, cell_blocks(g), 4, 0, out, false, st);
}

hipError_t launch_init_vjp(const Geom &g, int ltype, int eq, const double *u, const void *lam0,
                           double *grad_u, hipStream_t st) {
    const dim3 grid(cell_blocks(g)), block(kBlock);
#define LBM_VJP(LT, EQ)                                                                     \
    hipLaunchKernelGGL((k_init_vjp<LT, EQ>), grid, block, 0, st, g, u,                        \
                       (const typename Lam<LT>::T *)lam0, grad_u)
    if (ltype == LBM_F64) {
        if (eq == LBM_EQ_IMPROVED) LBM_VJP(LBM_F64, 1); else LBM_VJP(LBM_F64, 0);
    } else if (ltype == LBM_F32) {
        if (eq == LBM_EQ_IMPROVED) LBM_VJP(LBM_F32, 1); else LBM_VJP(LBM_F32, 0);
    } else {
        return hipErrorInvalidValue;
    }
#undef LBM_VJP
    return hipGetLastError();
}

}  // namespace lbm
