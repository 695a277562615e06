// api.hip -- C ABI of the ERPP coupling step (see include/erpp.h): argument
// validation, plan construction, stage dispatch, HIP-graph replay and the tile
// autotuner.  No C++ exception leaves this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "erpp_internal.hpp"

namespace erpp {

thread_local std::string g_err;

erpp_status fail(erpp_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

erpp_status hip_fail(hipError_t e, const char *what) {
    return fail(ERPP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace erpp

namespace {

using erpp::fail;
using erpp::g_err;
using erpp::hip_fail;

#define HIP_OR_RETURN(expr)                              \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_fail(_e, #expr); \
    } while (0)

__global__ void k_set_step(int64_t *s, int64_t n) { *s = n; }

// After an update with the memory terms: each box using the added mass or the
// Basset term now has a previous value of its path history.
__global__ void k_am_mark(const erpp::DevBox *__restrict__ Bs, int nbox) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbox && Bs[b].am_mf != 0.0) *Bs[b].am_valid = 1;
    if (b < nbox && Bs[b].bs_k != 0.0) *Bs[b].bs_valid = 1;
}
__global__ void k_advance_step(int64_t *s) { *s += 1; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Stencil offsets that can reach the cut-off sphere: m in [-floor(Rn), floor(Rn)+1]
// with Rn = cutoff sigma / dx (a small margin keeps the range a superset when
// Rn rounds just below an integer).
void stencil_range(double rc, double dx, int32_t &mlo, int32_t &mhi) {
    double Rn = rc / dx;
    int32_t f = (int32_t)std::floor(Rn + 1e-6);
    mlo = -f;
    mhi = f + 1;
}

void free_scratch(erpp_plan *p) {
    erpp::Scratch &s = p->s;
    (void)hipFree(s.count);
    (void)hipFree(s.start);
    (void)hipFree(s.rank);
    (void)hipFree(s.rec);
    (void)hipFree(s.up);
    (void)hipFree(s.bsum);
    (void)hipFree(s.pscale);
    (void)hipFree(s.pctr);
    (void)hipFree(s.xs);
    (void)hipFree(s.part);
    (void)hipFree(s.pamp);
    (void)hipFree(s.pphi);
    (void)hipFree(s.pbase);
    (void)hipFree(s.step);
    (void)hipFree(s.am_valid);
    (void)hipFree(s.aux);
    (void)hipFree(s.vrec);
    s = erpp::Scratch();
    (void)hipFree(p->dbox);
    p->dbox = nullptr;
}

void drop_coupled_graph(erpp_plan *p) {
    if (p->cgraph_exec) (void)hipGraphExecDestroy(p->cgraph_exec);
    if (p->cgraph) (void)hipGraphDestroy(p->cgraph);
    p->cgraph_exec = nullptr;
    p->cgraph = nullptr;
    p->cfluid_ids.clear();
}

void drop_graph(erpp_plan *p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    drop_coupled_graph(p);
}

template <typename T>
hipError_t alloc(T **ptr, size_t count) {
    if (count == 0) count = 1;
    return hipMalloc((void **)ptr, sizeof(T) * count);
}

erpp_status upload_boxes(erpp_plan *p) {
    if (p->prec == ERPP_F32_FAST) {
        HIP_OR_RETURN(erpp::fast_prepare_lds(p->lds_bytes));
        HIP_OR_RETURN(erpp::fast_prepare_bound_lds(p->bound_lds));
    }
    HIP_OR_RETURN(hipMemcpy(p->dbox, p->hbox.data(), sizeof(erpp::DevBox) * p->hbox.size(),
                            hipMemcpyHostToDevice));
    return ERPP_OK;
}

// Cell histogram, its scan and the scan partials (sized by the cells of all boxes).
erpp_status alloc_bins(erpp_plan *p) {
    const size_t nc = (size_t)std::max<int64_t>(p->ncell_total, 1);
    const size_t nchunk = (nc + erpp::kScanChunk - 1) / erpp::kScanChunk;
    if (alloc(&p->s.count, nc) != hipSuccess || alloc(&p->s.start, nc + 1) != hipSuccess ||
        alloc(&p->s.part, nchunk + 1) != hipSuccess)
        return fail(ERPP_ENOMEM, "cell arrays (%lld cells)", (long long)p->ncell_total);
    HIP_OR_RETURN(hipMemset(p->s.count, 0, sizeof(int32_t) * nc));
    HIP_OR_RETURN(hipMemset(p->s.start, 0, sizeof(int32_t) * (nc + 1)));
    return ERPP_OK;
}

erpp_status check_tile(const int32_t tile[3]) {
    if (!tile) return fail(ERPP_EINVAL, "tile is NULL");
    if (tile[0] != 0 && tile[0] != 512 && tile[0] != 1024)
        return fail(ERPP_EINVAL, "tile[0]=%d: scatter workgroup threads must be 0, 512 or 1024",
                    tile[0]);
    if (tile[1] < 1 || tile[1] > erpp::kMaxTileY)
        return fail(ERPP_EINVAL, "tile[1]=%d outside [1, %d]", tile[1], erpp::kMaxTileY);
    if (tile[2] < 1 || tile[2] > erpp::kMaxTileZ)
        return fail(ERPP_EINVAL, "tile[2]=%d outside [1, %d]", tile[2], erpp::kMaxTileZ);
    return ERPP_OK;
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

erpp_status run_stages(erpp_plan *p, hipStream_t st, bool update) {
    hipError_t e;
    if (p->prec == ERPP_F32_FAST) {
        e = erpp::fast_scatter_stages(p, st);
        if (e == hipSuccess && update) e = erpp::fast_update_stage(p, st);
    } else {
        e = erpp::plain_scatter_stages(p, st);
        if (e == hipSuccess && update) e = erpp::plain_update_stage(p, st);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return ERPP_OK;
}

}  // namespace

namespace erpp {

hipError_t set_step(erpp_plan *p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, st, p->s.step, n);
    return hipGetLastError();
}

hipError_t mark_memory_terms(erpp_plan *p, hipStream_t st) {
    hipLaunchKernelGGL(k_am_mark, dim3((unsigned)((p->nbox + 63) / 64)), dim3(64), 0, st, p->dbox,
                       p->nbox);
    return hipGetLastError();
}

hipError_t advance_step(erpp_plan *p, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(1), 0, st, p->s.step);
    return hipGetLastError();
}

static int32_t round4(int64_t v) { return (int32_t)((v + 3) & ~int64_t(3)); }

// Record-order buffers of the optional forces' grid terms, allocated on first use
// (outside any step, by the setters).
erpp_status ensure_aux(erpp_plan *p) {
    if (p->prec != ERPP_F32_FAST || p->s.aux) return ERPP_OK;
    HIP_OR_RETURN(hipDeviceSynchronize());
    if (alloc(&p->s.aux, (size_t)kAux * (size_t)std::max<int64_t>(p->np_total, 1)) != hipSuccess ||
        alloc(&p->s.vrec, (size_t)std::max<int64_t>(p->np_total, 1)) != hipSuccess) {
        (void)hipFree(p->s.aux);
        (void)hipFree(p->s.vrec);
        p->s.aux = nullptr;
        p->s.vrec = nullptr;
        (void)hipGetLastError();
        return fail(ERPP_ENOMEM, "record-order buffers of the particle forces");
    }
    return ERPP_OK;
}

// Pencils, block offsets and the scatter's LDS layout of every box for the
// plan's tile.  Returns false when a pencil does not fit the LDS.
bool fill_box_tiles(erpp_plan *p) {
    int64_t cell = 0, key = 0, bp = 0, bt = 0, br = 0, bb = 0, rows = 0;
    int64_t lds_max = 0, bound_max = 0;
    for (auto &B : p->hbox) {
        int32_t ext[3];
        for (int d = 0; d < 3; ++d) ext[d] = B.mhi[d] - B.mlo[d] + 1;
        B.T[0] = B.n[0];
        B.ntile[0] = 1;
        for (int d = 1; d < 3; ++d) {
            int32_t T = std::min(p->tile[d], B.n[d] - ext[d]);
            if (T < 1) T = 1;
            B.T[d] = T;
            B.ntile[d] = (B.n[d] + T - 1) / T;
        }
        B.cell_off = cell;
        cell += (int64_t)B.n[0] * B.n[1] * B.n[2];
        B.nxb = (B.n[0] + (1 << kXBlockShift) - 1) >> kXBlockShift;
        B.key_off = key;
        key += (int64_t)B.nxb * B.n[1] * B.n[2];
        B.blk_p = bp;
        bp += (B.np + kBlock - 1) / kBlock;
        B.blk_t = bt;
        bt += (int64_t)B.ntile[1] * B.ntile[2];
        B.rows = (int64_t)(B.mhi[1] - B.mlo[1] + 1) * (B.mhi[2] - B.mlo[2] + 1);
        B.blk_r = br;
        br += (B.np * B.rows + kBlock - 1) / kBlock;
        // scatter LDS: int32 pencil [T2][T1][pxa][3], then the window's record-start
        // table [(T2 + ext2 - 1)][(T1 + ext1 - 1) + 2]
        B.pxa = B.n[0] + ext[0];
        const int64_t accw = 3 * (int64_t)B.T[2] * B.T[1] * B.pxa;
        B.lds_tab = round4(accw);
        const int64_t wy = B.T[1] + ext[1] - 1, wz = B.T[2] + ext[2] - 1;
        const int64_t tabw = wz * (wy + 2);
        lds_max = std::max<int64_t>(lds_max, 4 * (B.lds_tab + round4(tabw)));
        bound_max = std::max<int64_t>(bound_max, 4 * wz * wy * kBoundXChunk);
        B.blk_b = bb;
        bb += ((int64_t)B.nxb * B.n[1] * B.n[2] + kBlock - 1) / kBlock;
        rows += (int64_t)B.n[1] * B.n[2];
    }
    p->ncell_total = cell;
    p->nkey_total = key;
    p->nrows_total = rows;
    p->bblocks = bb;
    p->pblocks = bp;
    p->tblocks = bt;
    p->pblocks_rows = br;
    p->lds_bytes = (size_t)lds_max;
    p->bound_lds = (size_t)bound_max;
    return p->lds_bytes <= kMaxScatterLds && p->bound_lds <= kMaxScatterLds;
}

}  // namespace erpp

namespace {

// One coupled step on `st`: stages 1-5 of every box, then each box's fluid step
// on its own u and f.  `capturing`: the plain path advances the step index
// inside the graph (the fast path's scan does it itself).
erpp_status coupled_step(erpp_plan *p, erpp_fluid *const *fluids, hipStream_t st, bool capturing) {
    erpp_status s = run_stages(p, st, true);
    if (s != ERPP_OK) return s;
    if (capturing && p->prec == ERPP_F64_PLAIN) {
        hipError_t e = erpp::advance_step(p, st);
        if (e != hipSuccess) return hip_fail(e, "advance_step");
    }
    for (int32_t b = 0; b < p->nbox; ++b) {
        s = erpp::fluid_launch(fluids[b], const_cast<void *>(p->boxes[b].u), p->boxes[b].f, st);
        if (s != ERPP_OK) return s;
    }
    return ERPP_OK;
}

}  // namespace

extern "C" {

const char *erpp_status_string(erpp_status s) {
    switch (s) {
        case ERPP_OK: return "ERPP_OK";
        case ERPP_EINVAL: return "ERPP_EINVAL: invalid argument";
        case ERPP_ENOMEM: return "ERPP_ENOMEM: device allocation failed";
        case ERPP_EHIP: return "ERPP_EHIP: HIP runtime error";
        case ERPP_EGEOM: return "ERPP_EGEOM: grid too small for the stencil or bad geometry";
        case ERPP_EUNSUPPORTED: return "ERPP_EUNSUPPORTED: outside the library's limits";
    }
    return "unknown erpp_status";
}

const char *erpp_last_error(void) { return g_err.c_str(); }

erpp_status erpp_plan_create(erpp_plan **out, const erpp_box *boxes, int32_t nbox, int32_t M,
                             double dt, erpp_precision prec, int32_t self_correction,
                             void *stream) {
    (void)stream;
    g_err.clear();
    if (!out) return fail(ERPP_EINVAL, "plan pointer is NULL");
    *out = nullptr;
    if (!boxes || nbox < 1) return fail(ERPP_EINVAL, "need nbox >= 1 boxes (got %d)", nbox);
    if (M < 1) return fail(ERPP_EINVAL, "M must be >= 1 (got %d)", M);
    if (!finite_pos(dt)) return fail(ERPP_EINVAL, "dt must be finite and > 0");
    if (prec != ERPP_F64_PLAIN && prec != ERPP_F32_FAST)
        return fail(ERPP_EINVAL, "unknown precision %d", (int)prec);
    if (self_correction != 0 && self_correction != 1)
        return fail(ERPP_EINVAL, "self_correction must be 0 or 1");
    int64_t np_total = 0;
    std::vector<erpp::DevBox> hb(nbox);
    for (int b = 0; b < nbox; ++b) {
        const erpp_box &X = boxes[b];
        erpp::DevBox &B = hb[b];
        std::memset(&B, 0, sizeof B);
        for (int d = 0; d < 3; ++d) {
            if (X.n[d] < 1) return fail(ERPP_EINVAL, "box %d: n[%d]=%d < 1", b, d, X.n[d]);
            if (!finite_pos(X.L[d])) return fail(ERPP_EGEOM, "box %d: L[%d] must be > 0", b, d);
        }
        if (X.np < 0) return fail(ERPP_EINVAL, "box %d: np < 0", b);
        if (X.np > INT32_MAX) return fail(ERPP_EUNSUPPORTED, "box %d: np > 2^31-1", b);
        if ((int64_t)X.n[0] * X.n[1] * X.n[2] > INT32_MAX)
            return fail(ERPP_EUNSUPPORTED, "box %d: more than 2^31-1 nodes", b);
        if (!X.u || !X.f) return fail(ERPP_EINVAL, "box %d: u or f is NULL", b);
        if (X.np > 0 && (!X.x || !X.v || !X.ring_x || !X.ring_d || !X.tau))
            return fail(ERPP_EINVAL, "box %d: a particle array is NULL", b);
        if (!finite_pos(X.m_p) || !finite_pos(X.rho_f))
            return fail(ERPP_EINVAL, "box %d: m_p and rho_f must be > 0", b);
        if (!std::isfinite(X.nu) || X.nu < 0.0) return fail(ERPP_EINVAL, "box %d: nu < 0", b);
        if (!finite_pos(X.sigma) || !finite_pos(X.cutoff))
            return fail(ERPP_EGEOM, "box %d: sigma and cutoff must be > 0", b);
        if (!std::isfinite(X.shear)) return fail(ERPP_EINVAL, "box %d: shear not finite", b);
        const double rc = X.cutoff * X.sigma;
        for (int d = 0; d < 3; ++d) {
            B.n[d] = X.n[d];
            B.L[d] = X.L[d];
            B.dx[d] = X.L[d] / (double)X.n[d];
            B.dxf[d] = (float)B.dx[d];
            int32_t R = (int32_t)std::ceil(rc / B.dx[d]);
            if (X.n[d] < 2 * R + 2)
                return fail(ERPP_EGEOM, "box %d: N[%d]=%d < 2*R_c+2 = %d", b, d, X.n[d], 2 * R + 2);
            stencil_range(rc, B.dx[d], B.mlo[d], B.mhi[d]);
            if (B.mhi[d] - B.mlo[d] + 1 > 16)
                return fail(ERPP_EUNSUPPORTED, "box %d: stencil of %d nodes in dim %d (> 16)", b,
                            B.mhi[d] - B.mlo[d] + 1, d);
        }
        // every position must have a node inside its sphere (the farthest point
        // from all nodes is a cell centre), or the lattice normalisation is 0
        if (rc * rc < 0.25 * (B.dx[0] * B.dx[0] + B.dx[1] * B.dx[1] + B.dx[2] * B.dx[2]))
            return fail(ERPP_EGEOM, "box %d: cutoff * sigma is below half the cell diagonal", b);
        if (prec == ERPP_F32_FAST && (X.n[0] > 2048 || X.n[1] > 2048 || X.n[2] > 1024))
            return fail(ERPP_EUNSUPPORTED, "box %d: grid beyond 2048 x 2048 x 1024", b);
        B.np = X.np;
        B.poff = np_total;
        np_total += X.np;
        B.dV = B.dx[0] * B.dx[1] * B.dx[2];
        B.R2 = rc * rc;
        B.two_s2 = 2.0 * X.sigma * X.sigma;
        B.m_p = X.m_p;
        B.rho_f = X.rho_f;
        B.shear = X.shear;
        B.s2s = X.sigma * X.sigma + 2.0 * X.nu * dt;
        B.pref = -(dt / X.rho_f) * std::pow(2.0 * M_PI * B.s2s, -1.5);
        B.R2f = (float)B.R2;
        B.guard = (float)(4.0e-6 * B.R2);
        B.cexp = (float)(1.0 / (B.two_s2 * std::log(2.0)));
        B.s2sf = (float)B.s2s;
        B.preff = (float)B.pref;
        B.rhof_inv = (float)(1.0 / X.rho_f);
        B.idxf0 = (float)(1.0 / B.dx[0]);
        B.x = X.x;
        B.v = X.v;
        B.ring_x = X.ring_x;
        B.ring_d = X.ring_d;
        B.tau = X.tau;
        B.u = X.u;
        B.f = X.f;
    }
    if (np_total > INT32_MAX) return fail(ERPP_EUNSUPPORTED, "more than 2^31-1 particles in a plan");

    erpp_plan *p = new (std::nothrow) erpp_plan();
    if (!p) return fail(ERPP_ENOMEM, "host allocation of the plan");
    (void)hipGetDevice(&p->device);
    p->nbox = nbox;
    p->M = M;
    p->dt = dt;
    p->prec = prec;
    p->self_correction = self_correction;
    p->boxes.assign(boxes, boxes + nbox);
    p->hbox = hb;
    p->np_total = np_total;
    if (!erpp::fill_box_tiles(p)) {
        // the default pencil is too large for these boxes: fall back to the thinnest
        p->tile[1] = p->tile[2] = 1;
        if (!erpp::fill_box_tiles(p)) {
            delete p;
            return fail(ERPP_EUNSUPPORTED, "stencil too wide for the scatter's LDS tile");
        }
    }
    bool ok = alloc(&p->dbox, (size_t)nbox) == hipSuccess && alloc(&p->s.step, 2) == hipSuccess &&
              alloc(&p->s.rank, (size_t)np_total) == hipSuccess &&
              alloc(&p->s.am_valid, 2 * (size_t)nbox) == hipSuccess;
    if (ok && prec == ERPP_F32_FAST)
        ok = alloc(&p->s.rec, 2 * (size_t)np_total) == hipSuccess &&
             alloc(&p->s.bsum, (size_t)std::max<int64_t>(p->nkey_total, 1)) == hipSuccess &&
             alloc(&p->s.pscale, (size_t)std::max<int64_t>(p->nrows_total, 1)) == hipSuccess &&
             alloc(&p->s.pctr, 8) == hipSuccess &&
             alloc(&p->s.up, (size_t)np_total) == hipSuccess &&
             alloc(&p->s.xs, (size_t)np_total) == hipSuccess;
    if (ok && prec == ERPP_F64_PLAIN)
        ok = alloc(&p->s.pamp, 4 * (size_t)np_total) == hipSuccess &&
             alloc(&p->s.pphi, 3 * (size_t)np_total) == hipSuccess &&
             alloc(&p->s.pbase, 3 * (size_t)np_total) == hipSuccess;
    if (!ok) {
        free_scratch(p);
        delete p;
        (void)hipGetLastError();
        return fail(ERPP_ENOMEM, "plan scratch for %lld particles", (long long)np_total);
    }
    for (int b = 0; b < nbox; ++b) {
        p->hbox[b].am_valid = p->s.am_valid + b;
        p->hbox[b].bs_valid = p->s.am_valid + nbox + b;
    }
    erpp_status s = alloc_bins(p);
    if (s == ERPP_OK && hipMemset(p->s.am_valid, 0, 2 * sizeof(int32_t) * nbox) != hipSuccess)
        s = fail(ERPP_EHIP, "hipMemset of the added-mass and Basset flags");
    if (s == ERPP_OK) s = upload_boxes(p);
    if (s == ERPP_OK && hipMemset(p->s.step, 0, 2 * sizeof(int64_t)) != hipSuccess)
        s = fail(ERPP_EHIP, "hipMemset of the step counter");
    if (s != ERPP_OK) {
        free_scratch(p);
        delete p;
        return s;
    }
    *out = p;
    return ERPP_OK;
}

erpp_status erpp_plan_set_tile(erpp_plan *p, const int32_t tile[3]) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    erpp_status s = check_tile(tile);
    if (s != ERPP_OK) return s;
    int32_t old[3];
    for (int d = 0; d < 3; ++d) {
        old[d] = p->tile[d];
        p->tile[d] = (d == 0 && tile[0] == 0) ? 512 : tile[d];
    }
    if (!erpp::fill_box_tiles(p)) {
        const size_t need = p->lds_bytes;
        for (int d = 0; d < 3; ++d) p->tile[d] = old[d];
        erpp::fill_box_tiles(p);
        return fail(ERPP_EINVAL, "pencil %d x %d does not fit the scatter's LDS (%zu bytes)",
                    tile[1], tile[2], need);
    }
    drop_graph(p);
    return upload_boxes(p);
}

erpp_status erpp_plan_set_rows_per_item(erpp_plan *p, int32_t rows) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (rows < erpp::kMinBand || rows > erpp::kMaxBand)
        return fail(ERPP_EINVAL, "rows per item %d outside [%d, %d]", rows, erpp::kMinBand,
                    erpp::kMaxBand);
    if (rows != p->band) {
        p->band = rows;
        drop_graph(p);   // the captured step holds the scatter instance
    }
    return ERPP_OK;
}

erpp_status erpp_plan_get_rows_per_item(const erpp_plan *p, int32_t *rows) {
    if (!p || !rows) return fail(ERPP_EINVAL, "NULL argument");
    *rows = p->band;
    return ERPP_OK;
}

erpp_status erpp_plan_set_body_force(erpp_plan *p, int32_t ibox, const double g[3]) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (ibox < 0 || ibox >= p->nbox) return fail(ERPP_EINVAL, "ibox %d out of range", ibox);
    if (!g) return fail(ERPP_EINVAL, "g is NULL");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(g[d])) return fail(ERPP_EINVAL, "g[%d] is not finite", d);
    for (int d = 0; d < 3; ++d) p->hbox[ibox].gb[d] = g[d];
    HIP_OR_RETURN(hipDeviceSynchronize());
    HIP_OR_RETURN(hipMemcpy(p->dbox + ibox, &p->hbox[ibox], sizeof(erpp::DevBox),
                            hipMemcpyHostToDevice));
    return ERPP_OK;
}

erpp_status erpp_plan_set_faxen(erpp_plan *p, int32_t ibox, double a_p) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (ibox < 0 || ibox >= p->nbox) return fail(ERPP_EINVAL, "ibox %d out of range", ibox);
    if (!std::isfinite(a_p) || a_p < 0.0) return fail(ERPP_EINVAL, "a_p must be finite and >= 0");
    if (a_p > 0.0) {
        erpp_status s = erpp::ensure_aux(p);
        if (s != ERPP_OK) return s;
    }
    p->hbox[ibox].fax = a_p * a_p / 6.0;
    drop_graph(p);     // the update kernel's instance depends on it
    HIP_OR_RETURN(hipDeviceSynchronize());
    HIP_OR_RETURN(hipMemcpy(p->dbox + ibox, &p->hbox[ibox], sizeof(erpp::DevBox),
                            hipMemcpyHostToDevice));
    return ERPP_OK;
}


erpp_status erpp_plan_set_added_mass(erpp_plan *p, int32_t ibox, double a, double *hist) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (ibox < 0 || ibox >= p->nbox) return fail(ERPP_EINVAL, "ibox %d out of range", ibox);
    if (!std::isfinite(a) || a < 0.0) return fail(ERPP_EINVAL, "a must be finite and >= 0");
    erpp::DevBox &B = p->hbox[ibox];
    if (a > 0.0) {
        if (!hist && B.np > 0) return fail(ERPP_EINVAL, "hist is NULL");
        if (B.integ != 0)
            return fail(ERPP_EUNSUPPORTED, "added mass runs with the explicit Euler integrator only");
        if (B.shear != 0.0)
            return fail(ERPP_EUNSUPPORTED, "box %d: added mass needs shear = 0 (the path "
                                           "derivative would see the Lees-Edwards jump)", ibox);
    }
    if (a > 0.0) {
        erpp_status s = erpp::ensure_aux(p);
        if (s != ERPP_OK) return s;
    }
    B.am_mf = a > 0.0 ? B.rho_f * (4.0 / 3.0) * M_PI * a * a * a : 0.0;
    B.am_fax = a * a / 10.0;
    B.am_hist = a > 0.0 ? hist : nullptr;
    drop_graph(p);     // the update kernel's instance depends on it
    HIP_OR_RETURN(hipDeviceSynchronize());
    HIP_OR_RETURN(hipMemset(B.am_valid, 0, sizeof(int32_t)));   // no previous value yet
    HIP_OR_RETURN(hipMemcpy(p->dbox + ibox, &B, sizeof(erpp::DevBox), hipMemcpyHostToDevice));
    return ERPP_OK;
}

erpp_status erpp_plan_set_basset(erpp_plan *p, int32_t ibox, double a, double *hist) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (ibox < 0 || ibox >= p->nbox) return fail(ERPP_EINVAL, "ibox %d out of range", ibox);
    if (!std::isfinite(a) || a < 0.0) return fail(ERPP_EINVAL, "a must be finite and >= 0");
    erpp::DevBox &B = p->hbox[ibox];
    if (a > 0.0) {
        if (!hist && B.np > 0) return fail(ERPP_EINVAL, "hist is NULL");
        if (B.integ != 0)
            return fail(ERPP_EUNSUPPORTED, "the Basset term runs with the explicit Euler "
                                           "integrator only");
        if (B.shear != 0.0)
            return fail(ERPP_EUNSUPPORTED, "box %d: the Basset term needs shear = 0 (the path "
                                           "difference would see the Lees-Edwards jump)", ibox);
        const double nu = p->boxes[ibox].nu;
        if (!(nu > 0.0))
            return fail(ERPP_EINVAL, "box %d: the Basset term needs nu > 0", ibox);
        erpp_status s = erpp::ensure_aux(p);
        if (s != ERPP_OK) return s;
    }
    // 6 pi mu a^2 int_0^dt (pi nu s)^(-1/2) ds / dt = 12 pi mu a^2 / sqrt(pi nu dt)
    const double nu = p->boxes[ibox].nu;
    B.bs_k = a > 0.0 ? 12.0 * M_PI * B.rho_f * nu * a * a / std::sqrt(M_PI * nu * p->dt) : 0.0;
    B.bs_fax = a * a / 6.0;
    B.bs_hist = a > 0.0 ? hist : nullptr;
    drop_graph(p);     // the update kernel's instance depends on it
    HIP_OR_RETURN(hipDeviceSynchronize());
    HIP_OR_RETURN(hipMemset(B.bs_valid, 0, sizeof(int32_t)));   // no previous value yet
    HIP_OR_RETURN(hipMemcpy(p->dbox + ibox, &B, sizeof(erpp::DevBox), hipMemcpyHostToDevice));
    return ERPP_OK;
}

erpp_status erpp_plan_set_integrator(erpp_plan *p, erpp_integrator kind) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (kind != ERPP_EULER && kind != ERPP_EXPONENTIAL && kind != ERPP_HEUN)
        return fail(ERPP_EINVAL, "unknown integrator %d", (int)kind);
    if (kind != ERPP_EULER)
        for (int32_t b = 0; b < p->nbox; ++b)
            if (p->hbox[b].am_mf != 0.0 || p->hbox[b].bs_k != 0.0)
                return fail(ERPP_EUNSUPPORTED, "box %d: the added-mass and Basset terms run "
                                               "with the explicit Euler integrator only", b);
    if (kind == ERPP_HEUN)
        for (int32_t b = 0; b < p->nbox; ++b)
            if (p->boxes[b].shear != 0.0)
                return fail(ERPP_EUNSUPPORTED, "box %d: Heun needs shear = 0 (its second "
                                               "stage would straddle the Lees-Edwards jump)", b);
    if (kind == ERPP_HEUN) {
        erpp_status s = erpp::ensure_aux(p);
        if (s != ERPP_OK) return s;
    }
    for (auto &B : p->hbox) B.integ = (int32_t)kind;
    drop_graph(p);     // the update kernel's instance depends on it
    HIP_OR_RETURN(hipDeviceSynchronize());
    HIP_OR_RETURN(hipMemcpy(p->dbox, p->hbox.data(), sizeof(erpp::DevBox) * p->hbox.size(),
                            hipMemcpyHostToDevice));
    return ERPP_OK;
}

erpp_status erpp_plan_get_tile(const erpp_plan *p, int32_t tile[3]) {
    if (!p || !tile) return fail(ERPP_EINVAL, "NULL argument");
    for (int d = 0; d < 3; ++d) tile[d] = p->tile[d];
    return ERPP_OK;
}

erpp_status erpp_plan_bins(const erpp_plan *p, int32_t ibox, int32_t *nbin) {
    if (!p || !nbin) return fail(ERPP_EINVAL, "NULL argument");
    if (ibox < 0 || ibox >= p->nbox) return fail(ERPP_EINVAL, "ibox %d out of range", ibox);
    const erpp::DevBox &B = p->hbox[ibox];
    *nbin = B.n[0] * B.n[1] * B.n[2];
    return ERPP_OK;
}

erpp_status erpp_bin(erpp_plan *p, int32_t ibox, const double *pos, int32_t *key, int32_t *perm,
                     int32_t *bin_start, void *stream) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (ibox < 0 || ibox >= p->nbox) return fail(ERPP_EINVAL, "ibox %d out of range", ibox);
    if (!bin_start) return fail(ERPP_EINVAL, "bin_start is NULL");
    if (p->hbox[ibox].np > 0 && (!pos || !key || !perm))
        return fail(ERPP_EINVAL, "pos, key or perm is NULL");
    hipError_t e = erpp::fast_bin_positions(p, ibox, pos, key, perm, bin_start, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "erpp_bin launch");
    return ERPP_OK;
}

erpp_status erpp_scatter(erpp_plan *p, int64_t step, void *stream) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (step < 0) return fail(ERPP_EINVAL, "step < 0");
    hipStream_t st = as_stream(stream);
    hipError_t e = erpp::set_step(p, step, st);
    if (e != hipSuccess) return hip_fail(e, "set_step");
    return run_stages(p, st, false);
}

erpp_status erpp_gather(erpp_plan *p, double *u_p, void *stream) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (!u_p && p->np_total > 0) return fail(ERPP_EINVAL, "u_p is NULL");
    hipError_t e = erpp::fast_gather(p, u_p, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "erpp_gather launch");
    return ERPP_OK;
}

erpp_status erpp_step(erpp_plan *p, int64_t step, void *stream) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (step < 0) return fail(ERPP_EINVAL, "step < 0");
    hipStream_t st = as_stream(stream);
    hipError_t e = erpp::set_step(p, step, st);
    if (e != hipSuccess) return hip_fail(e, "set_step");
    return run_stages(p, st, true);
}

erpp_status erpp_run(erpp_plan *p, int64_t step0, int64_t nsteps, int32_t use_graph,
                     void *stream) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (step0 < 0 || nsteps < 0) return fail(ERPP_EINVAL, "step0 and nsteps must be >= 0");
    hipStream_t st = as_stream(stream);
    if (!use_graph) {
        for (int64_t i = 0; i < nsteps; ++i) {
            erpp_status s = erpp_step(p, step0 + i, stream);
            if (s != ERPP_OK) return s;
        }
        return ERPP_OK;
    }
    if (!p->graph_exec) {
        hipStream_t cap;
        HIP_OR_RETURN(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return hip_fail(e, "hipStreamBeginCapture");
        }
        erpp_status s = run_stages(p, cap, true);
        // the fast path's scan advances the step index itself
        hipError_t e2 = p->prec == ERPP_F64_PLAIN ? erpp::advance_step(p, cap) : hipSuccess;
        hipGraph_t g = nullptr;
        hipError_t e3 = hipStreamEndCapture(cap, &g);
        (void)hipStreamDestroy(cap);
        if (s != ERPP_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e2 != hipSuccess || e3 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(e2 != hipSuccess ? e2 : e3, "graph capture");
        }
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        p->graph = g;
        p->graph_exec = ex;
    }
    HIP_OR_RETURN(erpp::set_step(p, step0, st));
    for (int64_t i = 0; i < nsteps; ++i) HIP_OR_RETURN(hipGraphLaunch(p->graph_exec, st));
    return ERPP_OK;
}

erpp_status erpp_run_coupled(erpp_plan *p, erpp_fluid *const *fluids, int64_t step0,
                             int64_t nsteps, int32_t use_graph, void *stream) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (!fluids) return fail(ERPP_EINVAL, "fluids is NULL");
    if (step0 < 0 || nsteps < 0) return fail(ERPP_EINVAL, "step0 and nsteps must be >= 0");
    for (int32_t b = 0; b < p->nbox; ++b) {
        if (!fluids[b]) return fail(ERPP_EINVAL, "fluids[%d] is NULL", b);
        erpp_status s = erpp::fluid_check(fluids[b], p->boxes[b], p->dt, p->prec, b);
        if (s != ERPP_OK) return s;
    }
    hipStream_t st = as_stream(stream);
    if (!use_graph) {
        for (int64_t i = 0; i < nsteps; ++i) {
            HIP_OR_RETURN(erpp::set_step(p, step0 + i, st));
            erpp_status s = coupled_step(p, fluids, st, false);
            if (s != ERPP_OK) return s;
        }
        return ERPP_OK;
    }
    std::vector<uint64_t> ids(p->nbox);
    for (int32_t b = 0; b < p->nbox; ++b) ids[b] = erpp::fluid_id(fluids[b]);
    if (p->cgraph_exec && ids != p->cfluid_ids) drop_coupled_graph(p);
    if (!p->cgraph_exec) {
        hipStream_t cap;
        HIP_OR_RETURN(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return hip_fail(e, "hipStreamBeginCapture");
        }
        erpp_status s = coupled_step(p, fluids, cap, true);
        hipGraph_t g = nullptr;
        hipError_t e3 = hipStreamEndCapture(cap, &g);
        (void)hipStreamDestroy(cap);
        if (s != ERPP_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e3 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(e3, "graph capture of the coupled step");
        }
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        p->cgraph = g;
        p->cgraph_exec = ex;
        p->cfluid_ids = ids;
    }
    HIP_OR_RETURN(erpp::set_step(p, step0, st));
    for (int64_t i = 0; i < nsteps; ++i) HIP_OR_RETURN(hipGraphLaunch(p->cgraph_exec, st));
    return ERPP_OK;
}

erpp_status erpp_plan_tune(erpp_plan *p, const char *cache_path, void *stream) {
    if (!p) return fail(ERPP_EINVAL, "plan is NULL");
    if (p->prec != ERPP_F32_FAST) return ERPP_OK;
    hipStream_t st = as_stream(stream);
    // geometry key
    std::ostringstream key;
    key << "v7 M" << p->M << " nbox" << p->nbox;
    for (const auto &B : p->hbox)
        key << " " << B.n[0] << "x" << B.n[1] << "x" << B.n[2] << ":" << B.np << ":" << B.mlo[0]
            << "," << B.mhi[0];
    const std::string k = key.str();
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            size_t bar = line.rfind('|');
            if (bar == std::string::npos || line.substr(0, bar) != k) continue;
            int32_t t[3], rows = 0;
            if (std::sscanf(line.c_str() + bar + 1, "%d %d %d %d", &t[0], &t[1], &t[2], &rows) ==
                    4 &&
                check_tile(t) == ERPP_OK && rows >= erpp::kMinBand && rows <= erpp::kMaxBand) {
                erpp_status s = erpp_plan_set_rows_per_item(p, rows);
                return s == ERPP_OK ? erpp_plan_set_tile(p, t) : s;
            }
        }
    }
    static const int32_t fixed[][3] = {{512, 16, 1},  {512, 8, 2},   {512, 8, 1},  {512, 4, 4},
                                       {512, 4, 2},   {512, 32, 1},  {512, 2, 2},  {512, 4, 1},
                                       {1024, 32, 1}, {1024, 16, 2}, {1024, 16, 1}, {1024, 8, 4},
                                       {1024, 64, 1}, {1024, 8, 2}};
    std::vector<std::array<int32_t, 3>> cand;
    for (const auto &c : fixed) cand.push_back({c[0], c[1], c[2]});
    // balanced heights: the fewest pencils per y extent of the tallest box whose
    // equal split fits the LDS, and one more (a plane of Ny rows in k pencils of
    // ceil(Ny / k) rows rather than full pencils and a short last one)
    {
        int32_t ny = 1;
        for (const auto &B : p->hbox) ny = std::max(ny, B.n[1]);
        const int32_t keep[3] = {p->tile[0], p->tile[1], p->tile[2]};
        int found = 0;
        for (int32_t k = 1; k <= ny && found < 2; ++k) {
            const int32_t t1 = (ny + k - 1) / k;
            if (t1 > erpp::kMaxTileY) continue;
            const int32_t c[3] = {1024, t1, 1};
            if (found == 0 && erpp_plan_set_tile(p, c) != ERPP_OK) continue;
            bool dup = false;
            for (const auto &d : cand) dup |= d[0] == c[0] && d[1] == c[1] && d[2] == c[2];
            if (!dup) cand.push_back({c[0], c[1], c[2]});
            ++found;
        }
        const erpp_status s = erpp_plan_set_tile(p, keep);
        if (s != ERPP_OK) return s;
    }
    const int ncand = (int)cand.size();
    int32_t best[3] = {p->tile[0], p->tile[1], p->tile[2]};
    float best_ms = 1e30f;
    hipEvent_t a, b;
    HIP_OR_RETURN(hipEventCreate(&a));
    HIP_OR_RETURN(hipEventCreate(&b));
    // the scatter reads ring level n-M of the step n following the last one run;
    // before M steps that level has not been written
    int64_t n = 0;
    HIP_OR_RETURN(hipStreamSynchronize(st));
    HIP_OR_RETURN(hipMemcpy(&n, p->s.step, sizeof n, hipMemcpyDeviceToHost));
    if (n < p->M) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return fail(ERPP_EINVAL,
                    "erpp_plan_tune: %lld steps run, the scatter needs ring level n - M (run at "
                    "least M = %d steps first)", (long long)n, p->M);
    }
    erpp_status status = ERPP_OK;
    // time the scatter of step n (warm-up, then 5 launches); ms < 0 on failure
    auto time_scatter = [&](float &ms) {
        status = erpp_scatter(p, n, stream);
        if (status != ERPP_OK) return;
        (void)hipEventRecord(a, st);
        const int reps = 5;
        for (int r = 0; r < reps && status == ERPP_OK; ++r) status = erpp_scatter(p, n, stream);
        (void)hipEventRecord(b, st);
        if (hipEventSynchronize(b) != hipSuccess) {
            status = fail(ERPP_EHIP, "autotuner synchronisation");
            return;
        }
        (void)hipEventElapsedTime(&ms, a, b);
    };
    // pencils at the default rows per item, then the rows per item (the number of
    // particles a wavefront pass covers for the same rows) at the best pencil
    int32_t best_rows = erpp::kDefaultBand;
    if (p->band != best_rows) status = erpp_plan_set_rows_per_item(p, best_rows);
    for (int c = 0; c < ncand && status == ERPP_OK; ++c) {
        if (check_tile(cand[c].data()) != ERPP_OK) continue;
        if (erpp_plan_set_tile(p, cand[c].data()) != ERPP_OK) continue;   // does not fit these boxes
        float ms = 0.f;
        time_scatter(ms);
        if (status == ERPP_OK && ms < best_ms) {
            best_ms = ms;
            std::memcpy(best, cand[c].data(), sizeof best);
        }
    }
    if (status == ERPP_OK) status = erpp_plan_set_tile(p, best);
    for (int rows = erpp::kMinBand; rows <= erpp::kMaxBand && status == ERPP_OK; ++rows) {
        if (rows == erpp::kDefaultBand) continue;
        status = erpp_plan_set_rows_per_item(p, rows);
        float ms = 0.f;
        if (status == ERPP_OK) time_scatter(ms);
        if (status == ERPP_OK && ms < best_ms) {
            best_ms = ms;
            best_rows = rows;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    // leave the step counter where it was (each timed scatter advanced it)
    {
        const hipError_t e = erpp::set_step(p, n, st);
        if (e != hipSuccess && status == ERPP_OK) status = hip_fail(e, "erpp_plan_tune");
    }
    if (status != ERPP_OK) return status;
    status = erpp_plan_set_rows_per_item(p, best_rows);
    if (status == ERPP_OK) status = erpp_plan_set_tile(p, best);
    if (status == ERPP_OK && cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        if (o)
            o << k << "|" << best[0] << " " << best[1] << " " << best[2] << " " << best_rows
              << "\n";
    }
    return status;
}

erpp_status erpp_stage_times(erpp_plan *p, int64_t step0, int64_t nsteps, double ms[5],
                             void *stream) {
    if (!p || !ms) return fail(ERPP_EINVAL, "NULL argument");
    if (step0 < 0 || nsteps < 1) return fail(ERPP_EINVAL, "need step0 >= 0 and nsteps >= 1");
    hipStream_t st = as_stream(stream);
    hipEvent_t ev[6];
    for (int k = 0; k < 6; ++k) HIP_OR_RETURN(hipEventCreate(&ev[k]));
    double acc[5] = {0, 0, 0, 0, 0};
    erpp_status status = ERPP_OK;
    for (int64_t i = 0; i < nsteps && status == ERPP_OK; ++i) {
        hipError_t e = erpp::set_step(p, step0 + i, st);
        (void)hipEventRecord(ev[0], st);
        for (int k = 0; k < 5 && e == hipSuccess; ++k) {
            e = p->prec == ERPP_F32_FAST ? erpp::fast_stage(p, k, st) : erpp::plain_stage(p, k, st);
            if (e == hipSuccess) e = hipEventRecord(ev[k + 1], st);
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
        if (e != hipSuccess) {
            status = hip_fail(e, "erpp_stage_times");
            break;
        }
        for (int k = 0; k < 5; ++k) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ev[k], ev[k + 1]);
            acc[k] += t;
        }
    }
    for (int k = 0; k < 6; ++k) (void)hipEventDestroy(ev[k]);
    if (status != ERPP_OK) return status;
    for (int k = 0; k < 5; ++k) ms[k] = acc[k] / (double)nsteps;
    return ERPP_OK;
}

void erpp_plan_destroy(erpp_plan *p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    drop_graph(p);
    free_scratch(p);
    delete p;
}

}  // extern "C"
