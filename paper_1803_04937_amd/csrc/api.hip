// C ABI of the D3Q19 / D3Q27 stream-collide library: parameter validation, context
// state, launch configuration and error reporting.  Kernels live in
// forward.hip and adjoint.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "launch.h"
#include "lbm.h"

using namespace lbm;

struct lbm_ctx {
    lbm_params p;
    Geom g;
    int gen;           // kGenPeriodic, kGenWalls (walls or solid cells), kGenOpen
    int co;            // collision operator of the stream-collide kernels (kCo*)
    bool nt;           // stream-collide with non-temporal hints (cache policy)
    bool adj_nt;       // adjoint with non-temporal hints
    void *buf[2];
    int cur;           // two-grid: index of the buffer holding the state
    hipStream_t stream;
    int64_t t;
    double scale;
    double mass0;
    CollBoth coll;
    Scratch sc;
    uint32_t nblocks;
    uint32_t *links;   // link words (Geom::links), caller-owned; nullptr without a mask
    std::string err;
};

static thread_local std::string g_init_error;

static int fail(lbm_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_init_error = buf;
    return code;
}

static int hip_fail(lbm_ctx *c, hipError_t e, const char *where) {
    return fail(c, LBM_EHIP, "%s: %s", where, hipGetErrorString(e));
}

extern "C" const char *lbm_version(void) { return "lbm-d3q19-d3q27-gfx950 1.3"; }

extern "C" void lbm_velocity_set(int32_t stencil, int32_t *c, double *w, int32_t *o) {
    const int qn = stencil == 27 ? 27 : 19;
    for (int q = 0; q < qn; ++q) {
        if (c) {
            c[3 * q + 0] = kC[q].x;
            c[3 * q + 1] = kC[q].y;
            c[3 * q + 2] = kC[q].z;
        }
        if (w) w[q] = wq(qn, q);
        if (o) o[q] = opp(q);
    }
}

static bool is_pow2(double s) {
    if (!(s > 0.0) || !isfinite(s)) return false;
    int e;
    return frexp(s, &e) == 0.5;
}

static int validate(const lbm_params *p, std::string &why) {
    if (!p) {
        why = "params is NULL";
        return LBM_EINVAL;
    }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) {
        why = "nx, ny, nz must be >= 1";
        return LBM_EINVAL;
    }
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    if (n >= (int64_t(1) << 31) - 4096) {
        why = "nx*ny*nz must be below 2^31";
        return LBM_EINVAL;
    }
    for (int d = 0; d < 3; ++d)
        if (p->periodic[d] != 0 && p->periodic[d] != 1) {
            why = "periodic[] entries must be 0 or 1";
            return LBM_EINVAL;
        }
    if (p->equilibrium != LBM_EQ_STANDARD && p->equilibrium != LBM_EQ_IMPROVED &&
        p->equilibrium != LBM_EQ_IMPROVED3) {
        why = "unknown equilibrium";
        return LBM_EINVAL;
    }
    if (p->collision != LBM_SRT && p->collision != LBM_TRT && p->collision != LBM_MRT &&
        p->collision != LBM_KBC) {
        why = "unknown collision";
        return LBM_EINVAL;
    }
    if (p->dtype < LBM_F64 || p->dtype > LBM_BF16_SHIFTED) {
        why = "unknown dtype";
        return LBM_EINVAL;
    }
    if (p->pattern != LBM_TWO_GRID && p->pattern != LBM_AA) {
        why = "unknown pattern";
        return LBM_EINVAL;
    }
    if (p->compressible != 0 && p->compressible != 1) {
        why = "compressible must be 0 or 1";
        return LBM_EINVAL;
    }
    if (p->stencil != 19 && p->stencil != 27) {
        why = "stencil must be 19 or 27";
        return LBM_EINVAL;
    }
    const int want_lt = p->dtype == LBM_F64 ? LBM_F64 : LBM_F32;
    if (p->adjoint_dtype != want_lt) {
        why = "adjoint_dtype must be LBM_F64 with dtype LBM_F64 and LBM_F32 otherwise";
        return LBM_EINVAL;
    }
    if (!(p->omega > 0.0 && p->omega < 2.0)) {
        why = "omega must lie in (0, 2)";
        return LBM_EINVAL;
    }
    if (p->collision == LBM_TRT && !(p->trt_magic > 0.0 && isfinite(p->trt_magic))) {
        why = "trt_magic must be a positive finite number";
        return LBM_EINVAL;
    }
    if (p->collision == LBM_MRT) {
        if (p->stencil != 19) {
            why = "MRT is defined for stencil 19 only";
            return LBM_EINVAL;
        }
        if (!(p->mrt_omega3 > 0.0 && p->mrt_omega3 < 2.0) ||
            !(p->mrt_omega4 > 0.0 && p->mrt_omega4 < 2.0)) {
            why = "mrt_omega3 and mrt_omega4 must lie in (0, 2)";
            return LBM_EINVAL;
        }
    }
    if (p->collision == LBM_KBC && p->stencil != 19) {
        why = "KBC is defined for stencil 19 only";
        return LBM_EINVAL;
    }
    if (p->open_x != 0 && p->open_x != 1) {
        why = "open_x must be 0 or 1";
        return LBM_EINVAL;
    }
    if (p->open_x) {
        if (p->periodic[0]) {
            why = "open x faces need periodic[0] == 0";
            return LBM_EINVAL;
        }
        if (p->pattern != LBM_TWO_GRID) {
            why = "open x faces need the two-grid pattern";
            return LBM_EINVAL;
        }
        if (p->compressible) {
            why = "open x faces need the incompressible form (compressible == 0)";
            return LBM_EINVAL;
        }
        if (!(p->rho_out > 0.0 && isfinite(p->rho_out))) {
            why = "rho_out must be a positive finite number";
            return LBM_EINVAL;
        }
    }
    for (int d = 0; d < 3; ++d)
        if (!isfinite(p->accel[d])) {
            why = "accel must be finite";
            return LBM_EINVAL;
        }
    if (p->cache_policy != LBM_CACHE_AUTO && p->cache_policy != LBM_CACHE_STREAM &&
        p->cache_policy != LBM_CACHE_KEEP) {
        why = "cache_policy must be LBM_CACHE_AUTO, LBM_CACHE_STREAM or LBM_CACHE_KEEP";
        return LBM_EINVAL;
    }
    if (p->adjoint_solid != LBM_ADJ_SOLID_COPY && p->adjoint_solid != LBM_ADJ_SOLID_SKIP) {
        why = "adjoint_solid must be LBM_ADJ_SOLID_COPY or LBM_ADJ_SOLID_SKIP";
        return LBM_EINVAL;
    }
    if (p->rounding != LBM_ROUND_NEAREST && p->rounding != LBM_ROUND_STOCHASTIC) {
        why = "rounding must be LBM_ROUND_NEAREST or LBM_ROUND_STOCHASTIC";
        return LBM_EINVAL;
    }
    const bool q16 = p->dtype == LBM_F16_SHIFTED || p->dtype == LBM_BF16_SHIFTED;
    if (q16 && p->scale != 0.0 && !is_pow2(p->scale)) {
        why = "scale must be 0 or a positive power of two";
        return LBM_EINVAL;
    }
    return LBM_OK;
}

extern "C" int lbm_validate(const lbm_params *p, char *msg, size_t len) {
    std::string why;
    int rc = validate(p, why);
    if (msg && len) {
        snprintf(msg, len, "%s", why.c_str());
    }
    return rc;
}

static size_t dtype_size(int dt) {
    switch (dt) {
    case LBM_F64: return 8;
    case LBM_F32:
    case LBM_F32_SHIFTED: return 4;
    default: return 2;
    }
}

// Buffers are plane-blocked: the Q direction arrays of one z-plane are
// contiguous, each nx*ny cells rounded up to 64 elements (one wave's
// accesses start on a 128-byte line for every storage type), and the planes
// follow each other.  Measured on MI355X at 256^3 FP32: 8 % more bytes per
// second for the forward pull and 13 % for the adjoint pattern than with one
// array per direction over the whole lattice, whose 19 streams lie 67 MB
// apart.
static int64_t qstride_of(const lbm_params *p) {
    const int64_t nxy = (int64_t)p->nx * p->ny;
    return ((nxy + 63) / 64) * 64;
}

// Elements of one buffer of Q direction arrays.
static int64_t buffer_elems(const lbm_params *p) {
    return (int64_t)p->nz * p->stencil * qstride_of(p);
}

extern "C" int lbm_qstride(const lbm_params *p, int64_t *qs) {
    std::string why;
    if (validate(p, why) != LBM_OK || !qs) return LBM_EINVAL;
    *qs = qstride_of(p);
    return LBM_OK;
}

extern "C" int lbm_state_bytes(const lbm_params *p, size_t *bytes) {
    std::string why;
    if (validate(p, why) != LBM_OK || !bytes) return LBM_EINVAL;
    *bytes = (size_t)buffer_elems(p) * dtype_size(p->dtype);
    return LBM_OK;
}

extern "C" int lbm_adjoint_bytes(const lbm_params *p, size_t *bytes) {
    std::string why;
    if (validate(p, why) != LBM_OK || !bytes) return LBM_EINVAL;
    *bytes = (size_t)buffer_elems(p) * dtype_size(p->adjoint_dtype);
    return LBM_OK;
}

// In-place inverse of an n x n matrix (n <= 10) by Gauss-Jordan elimination
// with partial pivoting.  The moment matrices passed here are nonsingular.
static void invert(double *a, int n) {
    double w[10][20];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            w[i][j] = j < n ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(w[r][col]) > fabs(w[piv][col])) piv = r;
        for (int j = 0; j < 2 * n; ++j) std::swap(w[col][j], w[piv][j]);
        const double inv = 1.0 / w[col][col];
        for (int j = 0; j < 2 * n; ++j) w[col][j] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = w[r][col];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j) w[r][j] -= f * w[col][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[i * n + j] = w[i][n + j];
}

// MRT relaxation matrices (Sec. 3.2) acting on the pair coordinates of the
// collide kernel.  D3Q19 keeps the monomials xi^e, e_i in {0,1,2}, other than
// the 8 that Sec. 3.2 drops; they split by parity into 10 even and 9 odd
// ones.  On a non-equilibrium vector n the even moments are
// sum_q c_q^e n_q = c_0^e n_0 + sum_p 2 c_q^e (n_q + n_qbar)/2 and the odd
// ones sum_p 2 c_q^e (n_q - n_qbar)/2 (q = 2p+1, qbar = q+1), so
// M_e = [c_0^e | 2 c_q^e] (10 x 10) and M_o = [2 c_q^e] (9 x 9); the
// relaxation in pair coordinates is K = M^-1 S M.
static void mrt_matrices(const lbm_params &p, double ke[100], double ko[81]) {
    static const int even[10][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0},
                                    {1, 0, 1}, {0, 1, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};
    static const int odd[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 1, 0}, {2, 0, 1},
                                  {1, 2, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2}};
    auto mono = [](const int e[3], int q) {
        const int c[3] = {kC[q].x, kC[q].y, kC[q].z};
        double v = 1.0;
        for (int i = 0; i < 3; ++i)
            for (int t = 0; t < e[i]; ++t) v *= c[i];
        return v;
    };
    auto rate = [&](const int e[3]) {
        const int order = e[0] + e[1] + e[2];
        return order <= 1 ? 1.0 : order == 2 ? p.omega : order == 3 ? p.mrt_omega3 : p.mrt_omega4;
    };
    auto relax = [](const double *m, const double *s, int n, double *k) {
        double mi[100];
        for (int i = 0; i < n * n; ++i) mi[i] = m[i];
        invert(mi, n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double v = 0.0;
                for (int l = 0; l < n; ++l) v += mi[i * n + l] * s[l] * m[l * n + j];
                k[i * n + j] = v;
            }
    };
    double me[100], se[10], mo[81], so[9];
    for (int k = 0; k < 10; ++k) {
        me[k * 10] = mono(even[k], 0);
        for (int pp = 0; pp < 9; ++pp) me[k * 10 + pp + 1] = 2.0 * mono(even[k], 2 * pp + 1);
        se[k] = rate(even[k]);
    }
    for (int k = 0; k < 9; ++k) {
        for (int pp = 0; pp < 9; ++pp) mo[k * 9 + pp] = 2.0 * mono(odd[k], 2 * pp + 1);
        so[k] = rate(odd[k]);
    }
    relax(me, se, 10, ke);
    relax(mo, so, 9, ko);
}

// Relaxation and force constants of the update in both precisions.
static void set_coll(lbm_ctx *c) {
    const lbm_params &p = c->p;
    const double wp = p.omega;
    double wm = wp, kappa = 1.0;
    if (p.collision == LBM_TRT) {
        const double tau_p = 1.0 / wp - 0.5;
        wm = 1.0 / (0.5 + p.trt_magic / tau_p);
        kappa = -wm * wm * p.trt_magic / (tau_p * tau_p * wp * wp);
    }
    Coll<double> d = {};
    d.wp = wp;
    d.wm = wm;
    d.kappa = kappa;
    // KBC: beta = omega / 2; 1/beta, 2 - 1/beta, upper bound 2 of gamma
    d.kbc_ib = 2.0 / wp;
    d.kbc_c = 2.0 - 2.0 / wp;
    d.kbc_hi = 2.0;
    d.drho_out = p.open_x ? p.rho_out - 1.0 : 0.0;
    for (int k = 0; k < 3; ++k) d.ah[k] = 0.5 * p.accel[k];
    for (int pp = 0; pp < (p.stencil - 1) / 2; ++pp) {
        const int q = 2 * pp + 1;
        const double ca = kC[q].x * p.accel[0] + kC[q].y * p.accel[1] + kC[q].z * p.accel[2];
        d.fraw[pp] = 3.0 * wq(p.stencil, q) * ca;
        d.fpair[pp] = (1.0 - 0.5 * wm) * d.fraw[pp];
    }
    d.s = c->scale;
    d.inv_s = 1.0 / c->scale;
    d.compressible = p.compressible;
    if (p.collision == LBM_MRT) mrt_matrices(p, d.ke, d.ko);
    d.w3 = p.mrt_omega3;
    d.w4 = p.mrt_omega4;
    Coll<float> f = {};
    f.wp = (float)d.wp;
    f.wm = (float)d.wm;
    f.kappa = (float)d.kappa;
    for (int k = 0; k < 3; ++k) f.ah[k] = (float)d.ah[k];
    for (int pp = 0; pp < 13; ++pp) {
        f.fraw[pp] = (float)d.fraw[pp];
        f.fpair[pp] = (float)d.fpair[pp];
    }
    f.s = (float)d.s;
    f.inv_s = (float)d.inv_s;
    f.compressible = d.compressible;
    f.kbc_ib = (float)d.kbc_ib;
    f.kbc_c = (float)d.kbc_c;
    f.kbc_hi = (float)d.kbc_hi;
    f.drho_out = (float)d.drho_out;
    for (int i = 0; i < 100; ++i) f.ke[i] = (float)d.ke[i];
    f.w3 = (float)d.w3;
    f.w4 = (float)d.w4;
    for (int i = 0; i < 81; ++i) f.ko[i] = (float)d.ko[i];
    c->coll.d = d;
    c->coll.f = f;
}

// Stochastic rounding applies to the 16-bit formats only.
static bool sr(const lbm_ctx *c) {
    return c->p.rounding == LBM_ROUND_STOCHASTIC &&
           (c->p.dtype == LBM_F16_SHIFTED || c->p.dtype == LBM_BF16_SHIFTED);
}

static Layout layout_of(const lbm_ctx *c) {
    if (c->p.pattern == LBM_TWO_GRID) return kDirect;
    return (c->t & 1) ? kAANeighbor : kAALocal;
}

static void *state_of(const lbm_ctx *c) {
    return c->p.pattern == LBM_TWO_GRID ? c->buf[c->cur] : c->buf[0];
}

static int totals(lbm_ctx *c, double *rho, double *u, double *sums) {
    hipError_t e = launch_moments(c->g, c->p.stencil, c->p.dtype, layout_of(c), 1.0 / c->scale,
                                  c->p.compressible, c->coll.d.ah, state_of(c), rho, u, c->sc,
                                  c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "moments");
    if (sums) {
        e = hipMemcpyAsync(sums, c->sc.result, 4 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "moments (copy totals)");
    }
    return LBM_OK;
}

extern "C" void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    if (c->sc.partials) (void)hipFree(c->sc.partials);
    if (c->sc.stage) (void)hipFree(c->sc.stage);
    if (c->sc.result) (void)hipFree(c->sc.result);
    delete c;
}

// Link-word buffer: one word per cell, then one word per 256-cell block
// (the list of blocks that hold a fluid cell).
static size_t links_words(const lbm_params *p) {
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    return n + (n + kBlock - 1) / kBlock;
}

extern "C" int lbm_links_bytes(const lbm_params *p, size_t *bytes) {
    std::string why;
    if (validate(p, why) != LBM_OK || !bytes) return LBM_EINVAL;
    *bytes = links_words(p) * sizeof(uint32_t);
    return LBM_OK;
}

// Scale of the 16-bit formats from the largest |f^eq - w| of the initial
// state: s = 2^floor(log2(1024 / maxdev)), at most 2^14 and at least 2^-10.
// FP16 keeps 11 significant bits whatever s is, so s only has to keep
// s |f - w| below the format's maximum (65504) and above its normal range
// (2^-14).  2^14 does both for every |f - w| in [2^-28, 4); a larger s,
// which a state close to rest would ask for, would overflow once the flow
// develops, so the exponent is capped there (a state at rest gets 2^14).
extern "C" int lbm_choose_scale(int32_t dtype, double maxdev, double *scale) {
    if (!scale || !(maxdev >= 0.0) || !isfinite(maxdev)) return LBM_EINVAL;
    if (dtype != LBM_F16_SHIFTED && dtype != LBM_BF16_SHIFTED) {
        *scale = 1.0;
        return LBM_OK;
    }
    int ex = maxdev > 0.0 ? (int)floor(log2(1024.0 / maxdev)) : 14;
    if (ex > 14) ex = 14;
    if (ex < -10) ex = -10;
    *scale = ldexp(1.0, ex);
    return LBM_OK;
}

static double *noalloc_scratch(std::string &why);

// Lattice geometry of validated parameters (no GPU call).
static void make_geom(const lbm_params *p, const uint32_t *links, Geom &g) {
    g.nx = p->nx;
    g.ny = p->ny;
    g.nz = p->nz;
    g.nxy = (uint32_t)p->nx * p->ny;
    g.ncells = g.nxy * (uint32_t)p->nz;
    g.div_nx = make_fastdiv(g.nx);
    g.div_ny = make_fastdiv(g.ny);
    g.div_nxy = make_fastdiv(g.nxy);
    for (int d = 0; d < 3; ++d) g.per[d] = p->periodic[d];
    g.qstride = qstride_of(p);
    g.zskip = (int64_t)p->stencil * g.qstride - (int64_t)g.nxy;
    g.links = links;
    g.inlet = nullptr;
    g.active = nullptr;
    g.nactive = 0;
}

extern "C" int lbm_init(lbm_ctx **out, const lbm_params *p, const uint8_t *solid, uint32_t *links,
                        void *pdf0, void *pdf1, void *stream, const double *rho_init,
                        const double *u_init) {
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (validate(p, why) != LBM_OK) return fail(nullptr, LBM_EINVAL, "%s", why.c_str());
    if (!pdf0) return fail(nullptr, LBM_EINVAL, "pdf0 is NULL");
    if (p->pattern == LBM_TWO_GRID && (!pdf1 || pdf1 == pdf0))
        return fail(nullptr, LBM_EINVAL, "two-grid needs a second, distinct buffer pdf1");
    if (p->pattern == LBM_AA && pdf1)
        return fail(nullptr, LBM_EINVAL, "the AA pattern uses one buffer; pdf1 must be NULL");
    if (!u_init) return fail(nullptr, LBM_EINVAL, "u_init is NULL");
    if (solid && !links)
        return fail(nullptr, LBM_EINVAL,
                    "a solid mask needs a link-word buffer of lbm_links_bytes bytes");

    lbm_ctx *c = new lbm_ctx();
    c->p = *p;
    c->buf[0] = pdf0;
    c->buf[1] = pdf1;
    c->cur = 0;
    c->stream = (hipStream_t)stream;
    c->t = 0;
    c->scale = 1.0;
    Geom &g = c->g;
    make_geom(p, nullptr, g);
    c->links = nullptr;
    c->gen = p->open_x ? kGenOpen
             : (solid != nullptr || !(p->periodic[0] && p->periodic[1] && p->periodic[2]))
                 ? kGenWalls
                 : kGenPeriodic;
    c->co = p->collision == LBM_MRT ? kCoMrt : p->collision == LBM_KBC ? kCoKbc : kCoPair;
    {
        size_t state_bytes = 0;
        lbm_state_bytes(p, &state_bytes);
        size_t adj_bytes = 0;
        lbm_adjoint_bytes(p, &adj_bytes);
        const size_t touched = (p->pattern == LBM_TWO_GRID ? 2 : 1) * state_bytes;
        const size_t touched_adj = state_bytes + 2 * adj_bytes;   // f_t, lam_next, lam_prev
        c->nt = p->cache_policy == LBM_CACHE_STREAM ||
                (p->cache_policy == LBM_CACHE_AUTO && touched > kCacheResidentBytes);
        c->adj_nt = p->cache_policy == LBM_CACHE_STREAM ||
                    (p->cache_policy == LBM_CACHE_AUTO && touched_adj > kCacheResidentBytes);
    }
    // host self-check of the division constants on the extreme values
    const uint32_t probes[4] = {0u, g.nx - 1, g.nx, g.ncells - 1};
    for (uint32_t v : probes)
        if (fdiv(v, g.div_nx) != v / g.nx || fdiv(v, g.div_ny) != v / g.ny ||
            fdiv(v, g.div_nxy) != v / g.nxy) {
            delete c;
            return fail(nullptr, LBM_EINVAL, "internal: fast division check failed");
        }
    c->nblocks = cell_blocks(g);
    {
        // look up the allocation-free entry point's scratch on this device
        // now, outside any graph capture (a failure is reported by that
        // entry point itself)
        std::string ignored;
        (void)noalloc_scratch(ignored);
    }
    c->sc.stage_half = (size_t)((c->nblocks + kReduceChunk - 1) / kReduceChunk) * 4;
    hipError_t e = hipMalloc(&c->sc.partials, (size_t)c->nblocks * 4 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->sc.stage, 2 * c->sc.stage_half * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->sc.result, 8 * sizeof(double));
    if (e != hipSuccess) {
        lbm_destroy(c);
        return fail(nullptr, LBM_ENOMEM, "scratch allocation: %s", hipGetErrorString(e));
    }
    // Link words for the kernels of a lattice with a mask, written into the
    // caller's buffer; walls alone are handled in registers.  The caller's
    // mask is read here only.
    if (solid) {
        c->links = links;
        g.links = c->links;
        e = launch_links(g, p->stencil, solid, c->links, c->stream);
        if (e != hipSuccess) {
            lbm_destroy(c);
            return fail(nullptr, LBM_EHIP, "link words: %s", hipGetErrorString(e));
        }
        // The blocks that hold a fluid cell, listed in ascending order after
        // the link words: the kernels that skip solid cells launch only
        // those.  The flags go through the host once, at set-up.
        uint32_t *list = c->links + g.ncells;
        const uint32_t nb = c->nblocks;
        std::vector<uint32_t> flags(nb);
        e = launch_block_fluid(g, list, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(flags.data(), list, nb * sizeof(uint32_t), hipMemcpyDeviceToHost,
                               c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        uint32_t na = 0;
        for (uint32_t b = 0; b < nb; ++b)
            if (flags[b]) flags[na++] = b;
        if (e == hipSuccess && na < nb) {
            e = hipMemcpyAsync(list, flags.data(), na * sizeof(uint32_t), hipMemcpyHostToDevice,
                               c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            g.active = list;
            g.nactive = na;
        }
        if (e != hipSuccess) {
            lbm_destroy(c);
            return fail(nullptr, LBM_EHIP, "active blocks: %s", hipGetErrorString(e));
        }
    }
    const bool q16 = p->dtype == LBM_F16_SHIFTED || p->dtype == LBM_BF16_SHIFTED;
    if (q16) {
        if (p->scale > 0.0) {
            c->scale = p->scale;
        } else {
            double maxdev = 0.0;
            e = launch_init_maxdev(g, p->stencil, p->equilibrium, p->compressible, rho_init, u_init, c->sc,
                                   c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&maxdev, c->sc.result, sizeof(double), hipMemcpyDeviceToHost,
                                   c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) {
                lbm_destroy(c);
                return fail(nullptr, LBM_EHIP, "scale search: %s", hipGetErrorString(e));
            }
            lbm_choose_scale(p->dtype, maxdev, &c->scale);
        }
    }
    set_coll(c);
    const Layout lay = p->pattern == LBM_TWO_GRID ? kDirect : kAALocal;
    e = launch_init(g, p->stencil, p->dtype, p->equilibrium, p->compressible, lay, rho_init, u_init, pdf0,
                    p->pattern == LBM_TWO_GRID ? pdf1 : nullptr, c->scale, c->stream);
    if (e != hipSuccess) {
        lbm_destroy(c);
        return fail(nullptr, LBM_EHIP, "init: %s", hipGetErrorString(e));
    }
    double sums[4];
    if (totals(c, nullptr, nullptr, sums) != LBM_OK) {
        g_init_error = c->err;
        lbm_destroy(c);
        return LBM_EHIP;
    }
    c->mass0 = sums[0];
    *out = c;
    return LBM_OK;
}

extern "C" const char *lbm_last_error(const lbm_ctx *c) {
    return c ? c->err.c_str() : g_init_error.c_str();
}

static int need_inlet(lbm_ctx *c) {
    if (c->p.open_x && !c->g.inlet)
        return fail(c, LBM_ESTATE, "open x faces: set the inflow with lbm_set_inlet first");
    return LBM_OK;
}

extern "C" int lbm_set_inlet(lbm_ctx *c, const double *u_in) {
    if (!c) return LBM_EINVAL;
    if (!c->p.open_x) return fail(c, LBM_ESTATE, "the context has no open faces");
    if (!u_in) return fail(c, LBM_EINVAL, "u_in is NULL");
    c->g.inlet = u_in;
    return LBM_OK;
}

extern "C" int lbm_step(lbm_ctx *c, int64_t n) {
    if (!c) return LBM_EINVAL;
    if (n < 0) return fail(c, LBM_EINVAL, "nsteps must be >= 0");
    if (need_inlet(c) != LBM_OK) return LBM_ESTATE;
    for (int64_t i = 0; i < n; ++i) {
        hipError_t e;
        if (c->p.pattern == LBM_TWO_GRID) {
            e = launch_step_tg(c->g, c->p.stencil, c->p.dtype, c->p.equilibrium, c->co,
                               c->gen, sr(c), c->nt,
                               step_key(c->p.seed, c->t), c->coll, c->buf[c->cur],
                               c->buf[1 - c->cur], c->stream);
            if (e == hipSuccess) c->cur ^= 1;
        } else {
            // even step count: the state is in local layout, so the next step
            // is a neighbour step; odd: a local step.
            e = launch_step_aa(c->g, c->p.stencil, c->p.dtype, c->p.equilibrium, c->co,
                               c->gen != kGenPeriodic, sr(c), c->nt,
                               step_key(c->p.seed, c->t), (c->t & 1) == 0, c->coll, c->buf[0],
                               c->stream);
        }
        if (e != hipSuccess) return hip_fail(c, e, "step");
        c->t += 1;
    }
    return LBM_OK;
}

extern "C" int lbm_stream_collide(lbm_ctx *c, const void *src, void *dst, int64_t t) {
    if (!c) return LBM_EINVAL;
    if (!src || !dst || src == dst) return fail(c, LBM_EINVAL, "src and dst must be distinct buffers");
    if (t < 0) return fail(c, LBM_EINVAL, "t must be >= 0");
    if (need_inlet(c) != LBM_OK) return LBM_ESTATE;
    hipError_t e = launch_step_tg(c->g, c->p.stencil, c->p.dtype, c->p.equilibrium, c->co,
                                  c->gen, sr(c), c->nt,
                                  step_key(c->p.seed, t), c->coll, src, dst, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "stream_collide");
    return LBM_OK;
}

extern "C" void *lbm_current_state(lbm_ctx *c) { return c ? state_of(c) : nullptr; }

extern "C" int lbm_copy_state(lbm_ctx *c, const void *src, void *dst) {
    if (!c) return LBM_EINVAL;
    if (!src || !dst || src == dst) return fail(c, LBM_EINVAL, "src and dst must be distinct buffers");
    size_t bytes = 0;
    lbm_state_bytes(&c->p, &bytes);
    hipError_t e = launch_copy(src, dst, bytes, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy_state");
    return LBM_OK;
}

extern "C" int64_t lbm_time(const lbm_ctx *c) { return c ? c->t : -1; }

extern "C" double lbm_scale(const lbm_ctx *c) { return c ? c->scale : 0.0; }

extern "C" int lbm_moments(lbm_ctx *c, double *rho, double *u, double *sums) {
    if (!c) return LBM_EINVAL;
    return totals(c, rho, u, sums);
}

extern "C" int lbm_get_pdfs(lbm_ctx *c, double *canonical) {
    if (!c) return LBM_EINVAL;
    if (!canonical) return fail(c, LBM_EINVAL, "canonical is NULL");
    hipError_t e = launch_get(c->g, c->p.stencil, c->p.dtype, layout_of(c), 1.0 / c->scale, state_of(c),
                              canonical, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "get_pdfs");
    return LBM_OK;
}

extern "C" int lbm_sample_pdfs(lbm_ctx *c, const int64_t *cells, int64_t n, double *out) {
    if (!c) return LBM_EINVAL;
    if (n < 0 || (n > 0 && (!cells || !out))) return fail(c, LBM_EINVAL, "cells/out must be set, n >= 0");
    if (n > ((int64_t)1 << 40)) return fail(c, LBM_EINVAL, "n too large");
    hipError_t e = launch_sample(c->g, c->p.stencil, c->p.dtype, layout_of(c), 1.0 / c->scale,
                                 state_of(c), cells, n, out, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "sample_pdfs");
    return LBM_OK;
}

extern "C" int lbm_set_pdfs(lbm_ctx *c, const double *canonical) {
    if (!c) return LBM_EINVAL;
    if (!canonical) return fail(c, LBM_EINVAL, "canonical is NULL");
    hipError_t e = launch_set(c->g, c->p.stencil, c->p.dtype, layout_of(c), c->scale, canonical, state_of(c),
                              c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_pdfs");
    return LBM_OK;
}

extern "C" int lbm_watchdog(lbm_ctx *c, double rel_tol) {
    if (!c) return LBM_EINVAL;
    double sums[4];
    int rc = totals(c, nullptr, nullptr, sums);
    if (rc != LBM_OK) return rc;
    for (int k = 0; k < 4; ++k)
        if (!isfinite(sums[k]))
            return fail(c, LBM_EDIVERGED, "non-finite total (mass %g, momentum %g %g %g)", sums[0],
                        sums[1], sums[2], sums[3]);
    if (fabs(sums[0] - c->mass0) > rel_tol * fabs(c->mass0))
        return fail(c, LBM_EDIVERGED, "mass drift %.3e relative (mass %.17g, initial %.17g)",
                    (sums[0] - c->mass0) / c->mass0, sums[0], c->mass0);
    return LBM_OK;
}

extern "C" int lbm_set_rates(lbm_ctx *c, double omega, const double *accel) {
    if (!c) return LBM_EINVAL;
    lbm_params p = c->p;
    p.omega = omega;
    if (accel)
        for (int d = 0; d < 3; ++d) p.accel[d] = accel[d];
    std::string why;
    if (validate(&p, why) != LBM_OK) return fail(c, LBM_EINVAL, "%s", why.c_str());
    c->p = p;
    set_coll(c);
    return LBM_OK;
}

// The adjoint family covers the incompressible form with SRT, TRT and MRT
// and without open faces.
static int adjoint_ok(lbm_ctx *c) {
    if (c->p.compressible)
        return fail(c, LBM_ESTATE, "the adjoint covers the incompressible form only");
    if (c->p.collision == LBM_KBC || c->p.open_x)
        return fail(c, LBM_ESTATE, "the adjoint covers SRT, TRT and MRT without open faces");
    return LBM_OK;
}

extern "C" int lbm_adjoint_step(lbm_ctx *c, const void *state_t, const void *lam_next,
                                void *lam_prev, double *grad) {
    if (!c) return LBM_EINVAL;
    if (adjoint_ok(c) != LBM_OK) return LBM_ESTATE;
    if (!state_t || !lam_next || !lam_prev || lam_next == lam_prev)
        return fail(c, LBM_EINVAL, "state_t, lam_next, lam_prev must be set, lam_next != lam_prev");
    if (c->p.pattern == LBM_AA && state_t == c->buf[0])
        return fail(c, LBM_ESTATE, "the AA buffer holds an AA layout; pass a state in the "
                                   "two-grid layout (lbm_stream_collide writes one)");
    hipError_t e = launch_adjoint(c->g, c->p.stencil, c->p.dtype, c->p.adjoint_dtype,
                                  c->p.equilibrium, c->p.collision == LBM_MRT,
                                  c->gen != kGenPeriodic, c->adj_nt,
                                  c->p.adjoint_solid == LBM_ADJ_SOLID_COPY, c->coll, state_t,
                                  lam_next, lam_prev, grad, c->sc, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step");
    return LBM_OK;
}

extern "C" int lbm_objective(lbm_ctx *c, int kind, const void *state, double *out, void *lam) {
    if (!c) return LBM_EINVAL;
    if (adjoint_ok(c) != LBM_OK) return LBM_ESTATE;
    if (kind != LBM_OBJ_KINETIC_ENERGY && kind != LBM_OBJ_OUTLET_FLUX)
        return fail(c, LBM_EINVAL, "unknown objective kind %d", kind);
    if (!state || !out || !lam) return fail(c, LBM_EINVAL, "state, out and lam must be set");
    if (c->p.pattern == LBM_AA && state == c->buf[0])
        return fail(c, LBM_ESTATE, "the AA buffer holds an AA layout; pass a state in the "
                                   "two-grid layout (lbm_stream_collide writes one)");
    hipError_t e = launch_objective(c->g, c->p.stencil, c->p.dtype, c->p.adjoint_dtype, kind,
                                    1.0 / c->scale, c->coll.d.ah, state, out, lam, c->sc,
                                    c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "objective");
    return LBM_OK;
}

extern "C" int lbm_init_vjp(lbm_ctx *c, const double *u_init, const void *lam0, double *grad_u) {
    if (!c) return LBM_EINVAL;
    if (adjoint_ok(c) != LBM_OK) return LBM_ESTATE;
    if (!u_init || !lam0 || !grad_u) return fail(c, LBM_EINVAL, "u_init, lam0, grad_u must be set");
    hipError_t e = launch_init_vjp(c->g, c->p.stencil, c->p.adjoint_dtype, c->p.equilibrium,
                                   u_init, lam0, grad_u, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "init_vjp");
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free moments.  The reduction scratch of lbm_moments_noalloc is
// this file-scope device array: one copy per GPU, held until the process
// ends.  Host code never passes its name to a kernel (in host code the name
// is a host-side stand-in); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current.  Layout: block partials (4 doubles per 256 cells), the two halves
// of the multi-pass fold, and a result slot.
// ---------------------------------------------------------------------------
constexpr uint32_t kNoAllocMaxBlocks = (uint32_t)(LBM_NOALLOC_MAX_CELLS / kBlock);
constexpr size_t kNoAllocStageHalf = (size_t)((kNoAllocMaxBlocks + kReduceChunk - 1) /
                                              kReduceChunk) * 4;
constexpr size_t kNoAllocDoubles = (size_t)kNoAllocMaxBlocks * 4 + 2 * kNoAllocStageHalf + 8;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (nullptr on failure).
static double *noalloc_scratch(std::string &why) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        why = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_ptr[dev] = (double *)ptr;
    }
    return g_scratch_ptr[dev];
}

extern "C" int lbm_moments_noalloc(const lbm_params *p, const uint32_t *links, const void *state,
                                   int64_t t, double scale, double *rho, double *u, double *sums,
                                   void *stream) {
    std::string why;
    if (validate(p, why) != LBM_OK) return fail(nullptr, LBM_EINVAL, "%s", why.c_str());
    const int64_t ncells = (int64_t)p->nx * p->ny * p->nz;
    if (ncells > LBM_NOALLOC_MAX_CELLS)
        return fail(nullptr, LBM_EINVAL,
                    "lbm_moments_noalloc: %lld cells exceed the maximum of %lld (its static "
                    "scratch holds the partials of 2^27 cells)",
                    (long long)ncells, (long long)LBM_NOALLOC_MAX_CELLS);
    if (!state) return fail(nullptr, LBM_EINVAL, "state is NULL");
    if (t < 0) return fail(nullptr, LBM_EINVAL, "t must be >= 0");
    const bool q16 = p->dtype == LBM_F16_SHIFTED || p->dtype == LBM_BF16_SHIFTED;
    if (q16 && !is_pow2(scale))
        return fail(nullptr, LBM_EINVAL, "scale must be the context's power of two (lbm_scale)");
    double *base = noalloc_scratch(why);
    if (!base) return fail(nullptr, LBM_EHIP, "%s", why.c_str());
    Geom g;
    make_geom(p, links, g);
    const uint32_t nblocks = cell_blocks(g);
    Scratch sc;
    sc.partials = base;
    sc.stage = base + (size_t)kNoAllocMaxBlocks * 4;
    sc.stage_half = (size_t)((nblocks + kReduceChunk - 1) / kReduceChunk) * 4;
    sc.result = sums ? sums : sc.stage + 2 * kNoAllocStageHalf;
    const Layout lay = p->pattern == LBM_TWO_GRID ? kDirect : ((t & 1) ? kAANeighbor : kAALocal);
    const double ah[3] = {0.5 * p->accel[0], 0.5 * p->accel[1], 0.5 * p->accel[2]};
    hipError_t e = launch_moments(g, p->stencil, p->dtype, lay, q16 ? 1.0 / scale : 1.0,
                                  p->compressible, ah, state, rho, u, sc, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, LBM_EHIP, "moments: %s", hipGetErrorString(e));
    return LBM_OK;
}
