// Host-side launch interface between the C ABI (api.hip) and the kernel
// translation units (forward.hip, adjoint.hip).  qn is the stencil size (19
// or 27).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

// State layouts of a PDF buffer.
enum Layout {
    kDirect = 0,    // slot [q][x] holds f*_q(x)           (two-grid; AA unused)
    kAALocal = 1,   // slot [qbar][x] holds f*_q(x)        (AA after an even step count)
    kAANeighbor = 2 // slot [q][x + c_q] holds f*_q(x), or [qbar][x] when x + c_q
                    // is a wall or solid                  (AA after an odd step count)
};

// Collision parameters in both compute precisions; kernels take the one of
// their storage type.
struct CollBoth {
    Coll<double> d;
    Coll<float> f;
};

// The parameters in the compute precision of storage type DT.
template <int DT>
inline const Coll<typename Store<DT>::R> &pick(const CollBoth &P) {
    if constexpr (DT == LBM_F64)
        return P.d;
    else
        return P.f;
}

// Reduction scratch: nblocks x 4 doubles of block partials, a two-half
// staging area for the multi-pass final reduction, and a small result slot.
struct Scratch {
    double *partials;
    double *stage;        // 2 x stage_half doubles
    size_t stage_half;    // ceil(nblocks / kReduceChunk) * 4
    double *result;       // device double[8]
};

constexpr uint32_t kReduceChunk = 1024;  // partials folded per block and pass

hipError_t launch_init(const Geom &g, int qn, int dtype, int eq, int compressible, Layout layout,
                       const double *rho, const double *u, void *A, void *B, double s,
                       hipStream_t st);
hipError_t launch_init_maxdev(const Geom &g, int qn, int eq, int compressible, const double *rho,
                              const double *u, const Scratch &sc, hipStream_t st);
// sr: stochastic rounding of the 16-bit stores with the step key `key`;
// nt: non-temporal hints (false: every access cached).
// Link words of the lattice (Geom::links) from the walls and the mask.
hipError_t launch_links(const Geom &g, int qn, const uint8_t *solid, uint32_t *links,
                        hipStream_t st);
// flags[b] = 1 when 256-cell block b holds a fluid cell (g.links set), else 0.
hipError_t launch_block_fluid(const Geom &g, uint32_t *flags, hipStream_t st);
// co: collision operator (kCo*); gen: boundary handling (kGen*); the AA
// steps take no open faces.
hipError_t launch_step_tg(const Geom &g, int qn, int dtype, int eq, int co, int gen,
                          bool sr, bool nt, uint32_t key, const CollBoth &P, const void *src,
                          void *dst, hipStream_t st);
hipError_t launch_step_aa(const Geom &g, int qn, int dtype, int eq, int co, bool gen,
                          bool sr, bool nt, uint32_t key, bool neighbor, const CollBoth &P,
                          void *A, hipStream_t st);
hipError_t launch_get(const Geom &g, int qn, int dtype, Layout layout, double inv_s, const void *A,
                      double *out, hipStream_t st);
hipError_t launch_sample(const Geom &g, int qn, int dtype, Layout layout, double inv_s,
                         const void *A, const int64_t *cells, int64_t n, double *out,
                         hipStream_t st);
hipError_t launch_set(const Geom &g, int qn, int dtype, Layout layout, double s, const double *in,
                      void *A, hipStream_t st);
hipError_t launch_moments(const Geom &g, int qn, int dtype, Layout layout, double inv_s,
                          int compressible, const double ah[3], const void *A, double *rho,
                          double *u, const Scratch &sc, hipStream_t st);
hipError_t launch_adjoint(const Geom &g, int qn, int dtype, int ltype, int eq, bool mrt, bool gen,
                          bool nt, bool copy_solid, const CollBoth &P, const void *state,
                          const void *lam_next, void *lam_prev, double *grad, const Scratch &sc,
                          hipStream_t st);
hipError_t launch_objective(const Geom &g, int qn, int dtype, int ltype, int kind, double inv_s,
                            const double ah[3], const void *state, double *out, void *lam,
                            const Scratch &sc, hipStream_t st);
hipError_t launch_init_vjp(const Geom &g, int qn, int ltype, int eq, const double *u,
                           const void *lam0, double *grad_u, hipStream_t st);

// Sum (op 0) or max (op 1) of nvals columns of nblocks partials into out
// (accumulate: out += result; else out = result).  Passes of 1024-way folds,
// then one block; the order of every addition is fixed.
hipError_t launch_finalize(const Scratch &sc, uint32_t nblocks, int nvals, int op, double *out,
                           bool accumulate, hipStream_t st);

// Plain copy of nbytes (a multiple of 16) from src to dst.
hipError_t launch_copy(const void *src, void *dst, size_t nbytes, hipStream_t st);

inline uint32_t cell_blocks(const Geom &g) { return (g.ncells + kBlock - 1) / kBlock; }
// Workgroups of a launch over the active list (see Geom::active).
inline uint32_t gen_blocks(const Geom &g) { return g.active ? g.nactive : cell_blocks(g); }
// Planar launch (blocks of one z-plane each): possible when the planes fit
// the grid's second dimension and a plane's FP64 bytes fit 32-bit offsets.
inline bool planar_ok(const Geom &g) {
    return g.nz <= kMaxPlanes && (uint64_t)g.nxy * sizeof(double) <= 0xffffffffull;
}
inline dim3 plane_grid(const Geom &g) { return dim3((g.nxy + kBlock - 1) / kBlock, g.nz); }

}  // namespace lbm
