// erpp_internal.hpp -- plan and per-box descriptors shared by the host API and
// the kernels of the MI355X ERPP coupling step.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/erpp.h"

namespace erpp {

constexpr int kMaxTileY = 64;        // scatter pencil: T1 x T2 nodes in (y, z), all of x
constexpr int kMaxTileZ = 8;
constexpr int kBlock = 256;          // threads per block of particle kernels
constexpr int kMinBand = 2;          // rows per work item of the scatter: the
constexpr int kMaxBand = 4;          //   instances built
constexpr int kDefaultBand = 3;
constexpr int kScanChunk = 4096;     // counters per block of the device-wide scan
constexpr int kXBlockShift = 4;      // step binning: x-blocks of 16 cells per cell row
constexpr int kAux = 6;              // record-order grid terms: lap, grad x3, u(x*), lap(x*)
constexpr int kBoundXChunk = 16;     // x-blocks per LDS pass of the pencil-scale kernel

// Everything a kernel needs to know about one box; lives in device memory as
// an array indexed by box.  Plain old data.
struct DevBox {
    int32_t n[3];        // nodes
    int32_t mlo[3];      // stencil offsets m in [mlo, mhi] around the base cell
    int32_t mhi[3];
    int32_t T[3];        // scatter pencil (nodes) of this box: T[0] = Nx, T[1], T[2] clipped
    int32_t ntile[3];    // pencils per dimension (ntile[0] = 1)
    int32_t pxa;         // words per unwrapped pencil row in LDS (Nx + mhi - mlo + 1)
    int32_t lds_tab;     // LDS word offset of the window's record-start table
    int64_t np;          // particles
    int64_t poff;        // first particle in the concatenated particle space
    int64_t cell_off;    // first cell of this box in the concatenated cell space (erpp_bin)
    int64_t key_off;     // first key of this box in the step's (row, x-block) key space
    int32_t nxb;         // x-blocks per cell row
    int32_t integ;       // particle integrator: 0 explicit Euler, 1 exponential, 2 Heun
    int64_t blk_p;       // first block of this box in particle launches
    int64_t blk_t;       // first block of this box in tile launches
    int64_t blk_b;       // first block of this box in (cell row, x-block) launches
    int64_t blk_r;       // first block of this box in (particle, row) launches
    int64_t rows;        // stencil rows (my, mz) per particle
    double L[3];
    double dx[3];        // L / N
    double dV;
    double R2;           // (cutoff * sigma)^2, FP64 sphere threshold
    double two_s2;       // 2 sigma^2
    double m_p, rho_f, shear;
    double gb[3];        // body acceleration of the particles, (m_p - m_f) g / m_p
    double fax;          // Faxen coefficient a_p^2 / 6 (0: no Faxen term)
    double am_mf;        // added mass: displaced fluid mass m_f (0: no added-mass terms)
    double am_fax;       // added mass: Faxen coefficient a^2 / 10 of its d/dt term
    double *am_hist;     // added mass: [6][np] u~ and u~ + am_fax lap u~ of the last step
    int32_t *am_valid;   // added mass: 0 until the first step with the terms has run
    double bs_k;         // Basset: 12 pi mu a_b^2 / sqrt(pi nu dt) (0: no Basset term)
    double bs_fax;       // Basset: Faxen coefficient a_b^2 / 6 of its bracket
    double *bs_hist;     // Basset: [3][np] w = u~ + bs_fax lap u~ - v of the last step
    int32_t *bs_valid;   // Basset: 0 until the first step with the term has run
    double s2s;          // sigma_s^2 = sigma^2 + 2 nu dt  (self-disturbance width)
    double pref;         // -(dt/rho_f) (2 pi sigma_s^2)^(-3/2)
    float dxf[3];
    float R2f;           // FP32 sphere threshold
    float guard;         // |d2 - R2f| <= guard: decide in FP64
    float cexp;          // 1 / (2 sigma^2 ln 2): raw weight = exp2(-d2 cexp)
    float s2sf, preff;
    float rhof_inv;
    float idxf0;         // 1 / dx (FP32), row-end estimates
    double *x, *v, *ring_x;
    void *ring_d;
    const float *tau;
    const void *u;
    void *f;
};

// Geometry of one exact cell binning (erpp_bin), passed to its kernels by value.
struct BinGeom {
    int32_t n[3];
    double L[3];
    double dx[3];        // L / N
    int64_t np;
};

struct Scratch {
    // ERPP_F32_FAST
    int32_t *count = nullptr;    // [ncell_total]   per-step cell histogram (kept zero at rest)
    int32_t *start = nullptr;    // [ncell_total+1] exclusive scan of count
    int32_t *part = nullptr;     // [nchunk+1]      scan partials
    int32_t *rank = nullptr;     // [np_total]      rank of a particle inside its cell
    float4 *rec = nullptr;       // [2*np_total]    cell-sorted injection records
    float *bsum = nullptr;       // [nkey_total]    max_c |amplitude| summed over x-blocks X-1..X+1
    float *pscale = nullptr;     // [sum Ny Nz]     fixed-point scale of each scatter pencil
    int32_t *pctr = nullptr;     // [8]             scatter: pencils handed out of each XCD's
                                 //                 run (cleared by the pencil-scale kernel)
    double4 *xs = nullptr;       // [np_total]      x^n in record order, particle index in w
    double4 *up = nullptr;       // [np_total]      carrier at x^n in particle order (FP64)
    // grid terms of the optional forces, in particle order (allocated when a box
    // turns on the Faxen term, the added mass or Heun): [kAux][np_total] of
    // lap u, grad u (3: d_x u, d_y u, d_z u), carrier and lap u at Heun's x*
    double4 *aux = nullptr;
    double4 *vrec = nullptr;     // [np_total]      v^n in record order (Heun)
    // ERPP_F64_PLAIN
    double *pamp = nullptr;      // [4][np_total] -D/rho_f (3 components) and Z
    double *pphi = nullptr;      // [3][np_total] offsets inside the base cell
    int32_t *pbase = nullptr;    // [3][np_total] base cell
    // both
    int32_t *am_valid = nullptr; // [2 nbox]        history present (per box): added mass,
                                 //                 then Basset
    int64_t *step = nullptr;     // [2] step index: [0] next step to run (set by the host,
                                 // advanced by the scan of the fast path or by a kernel
                                 // of its own in the plain path), [1] the step in progress
};

}  // namespace erpp

struct erpp_plan {
    int device = 0;
    int32_t nbox = 0;
    int32_t M = 1;
    double dt = 0;
    erpp_precision prec = ERPP_F32_FAST;
    int32_t self_correction = 1;
    int32_t tile[3] = {512, 4, 4};   // scatter: [0] threads per workgroup, pencil T1, T2
    std::vector<erpp_box> boxes;
    std::vector<erpp::DevBox> hbox;
    erpp::DevBox *dbox = nullptr;
    int64_t np_total = 0;
    int64_t ncell_total = 0;
    int64_t nkey_total = 0;
    int64_t pblocks = 0;         // blocks of particle launches (box aligned)
    int64_t tblocks = 0;         // blocks of tile launches
    int64_t bblocks = 0;         // blocks of (cell row, x-block) launches
    int64_t nrows_total = 0;     // cell rows (y, z) of all boxes: the most pencils possible
    int64_t pblocks_rows = 0;    // plain scatter: blocks over (particle,row)
    erpp::Scratch s;
    size_t lds_bytes = 0;
    int32_t band = erpp::kDefaultBand;  // scatter: stencil rows per work item (lane)
    size_t bound_lds = 0;        // dynamic LDS of the pencil-scale kernel
    // scatter: resident workgroups (compute units x workgroups per unit) of the
    // instance and LDS size they were computed for
    int64_t sgrid = 0;
    const void *sgrid_fn = nullptr;
    size_t sgrid_lds = 0;
    // graph of one step (step index read from s.step)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // graph of one coupled step (coupling step, then the fluid step of every box)
    // and the identities of the fluid steppers it was captured with
    hipGraph_t cgraph = nullptr;
    hipGraphExec_t cgraph_exec = nullptr;
    std::vector<uint64_t> cfluid_ids;
};

namespace erpp {
// error reporting shared by the ABI entry points: sets erpp_last_error()
erpp_status fail(erpp_status s, const char *fmt, ...);
erpp_status hip_fail(hipError_t e, const char *what);

// fluid stepper (fluid.hip): a unique id per created stepper, the check that it
// fits box `ibox` of a plan, and the launches of one step on a stream
uint64_t fluid_id(const erpp_fluid *fl);
erpp_status fluid_check(const erpp_fluid *fl, const erpp_box &b, double dt, erpp_precision prec,
                        int ibox);
erpp_status fluid_launch(erpp_fluid *fl, void *u, const void *f, hipStream_t st);

// kernel launchers (each returns hipSuccess or the launch error)
hipError_t fast_stage(erpp_plan *p, int k, hipStream_t st);      // k = 0 bin .. 4 update
hipError_t plain_stage(erpp_plan *p, int k, hipStream_t st);
hipError_t fast_scatter_stages(erpp_plan *p, hipStream_t st);   // bin, scan, eval, scatter
hipError_t fast_update_stage(erpp_plan *p, hipStream_t st);     // gather, self term, update
hipError_t fast_gather(erpp_plan *p, double *u_p, hipStream_t st);
hipError_t fast_bin_positions(erpp_plan *p, int ibox, const double *pos, int32_t *key,
                              int32_t *perm, int32_t *bin_start, hipStream_t st);
// exact cell binning with caller-provided scratch: count [ncell] (zero on entry
// unless clear), rank [np], part [ncell / kScanChunk + 2]; count is zero again on
// exit
hipError_t bin_positions(const BinGeom &G, const double *pos, int32_t *key, int32_t *perm,
                         int32_t *bin_start, int32_t *count, int32_t *rank, int32_t *part,
                         bool clear, hipStream_t st);
hipError_t plain_scatter_stages(erpp_plan *p, hipStream_t st);
hipError_t plain_update_stage(erpp_plan *p, hipStream_t st);
hipError_t set_step(erpp_plan *p, int64_t n, hipStream_t st);
hipError_t advance_step(erpp_plan *p, hipStream_t st);
// after an update: the added-mass and Basset histories of the boxes using them exist
hipError_t mark_memory_terms(erpp_plan *p, hipStream_t st);
bool fill_box_tiles(erpp_plan *p);      // tiles, blocks, LDS layout; false if it does not fit
erpp_status ensure_aux(erpp_plan *p);   // allocate Scratch::aux / vrec (FP32 path)
// start = exclusive scan of count, count = 0; with stepp, also step[1] = step[0]++
hipError_t scan_counts(int32_t *count, int64_t n, int32_t *start, int32_t *part, int64_t *stepp,
                       hipStream_t st);
hipError_t fast_prepare_lds(size_t bytes);         // opt the scatter into > 64 KB LDS
hipError_t fast_prepare_bound_lds(size_t bytes);   // same for the pencil-scale kernel
constexpr size_t kMaxScatterLds = 150 * 1024;
}  // namespace erpp
