// fast.hip -- ERPP_F32_FAST path of the coupling step for gfx950.
//
// Per step n (all boxes of a plan in one launch per stage):
//   k_bin_count   histogram of the delayed positions X^{n-M} by cell row and
//                 x-block; a particle's atomic ticket is its rank in its bin
//   k_scan_*      device-wide exclusive scan of the histogram (and its reset);
//                 publishes the step index for the kernels after it
//   k_eval        per particle: FP64 cell/offset of X^{n-M}, FP32 Gaussian
//                 normalisation over the 3-sigma sphere, record
//                 {offsets, amplitude} written at its cell-sorted slot, and x^n
//                 in record order
//   k_block_sums, k_pencil_scale  the fixed-point bound of every scatter pencil
//   k_scatter     pencils of nodes (full x extent), one per workgroup or, on
//                 large grids, taken in turn by resident workgroups: the stencil
//                 rows of every particle that reaches the pencil are accumulated
//                 into an LDS copy of it, which is then stored (each node written
//                 once, no global atomics)
//   k_gather_sorted  carrier at x^n by trilinear interpolation, particles
//                 visited in cell order (records of level n - M), results in
//                 particle order
//   k_update      per particle: closed-form self term, Stokes drag, history
//                 write, the step of the chosen integrator, wrap
#include <hip/hip_runtime.h>

#include <algorithm>

#include "erpp_device.hpp"
#include "erpp_internal.hpp"

namespace erpp {

namespace {

// Logical block of a launch whose grid is padded to a multiple of kXcds:
// physical block b runs on XCD b mod kXcds; XCD x takes logical blocks
// [x G/kXcds, (x + 1) G/kXcds).  A bijection on [0, grid).
constexpr int kXcds = 8;
// the scatter runs resident workgroups when its pencils exceed this many per
// resident workgroup (the 512^3 box: 46 per CU, 5.21 -> 4.76 ms per step; at 7 per
// CU, as on the 256^3 box, it measured 1% slower, at 2 the same)
constexpr int64_t kPersist = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t grid) {
    return (b % kXcds) * (grid / kXcds) + b / kXcds;
}

// Sort key of the step's binning: cell row (b1, b2), then x-block of
// 2^kXBlockShift cells.  Records of a cell row stay contiguous (the scatter's
// ranges) and in x-block order (the gather's locality), while the counters are
// few enough to stay in L2.
__device__ __forceinline__ int64_t step_key(const DevBox &B, int b0, int b1, int b2) {
    return B.key_off + ((int64_t)b2 * B.n[1] + b1) * B.nxb + (b0 >> kXBlockShift);
}

__global__ void __launch_bounds__(kBlock) k_bin_count(const DevBox *__restrict__ Bs, int nbox,
                                                      const int64_t *__restrict__ stepp, int M,
                                                      int32_t *__restrict__ count,
                                                      int32_t *__restrict__ rank) {
    const int64_t n = *stepp;
    if (n < M) return;
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int64_t p = (int64_t)(blockIdx.x - B.blk_p) * kBlock + threadIdx.x;
    if (p >= B.np) return;
    const int64_t np = B.np;
    const int64_t slot = (n - M) % (M + 1);
    const double *X = B.ring_x + slot * 3 * np;
    int b[3];
    double ph;
    for (int d = 0; d < 3; ++d) cell_of(X[d * np + p], B.L[d], B.dx[d], B.n[d], b[d], ph);
    rank[B.poff + p] = atomicAdd(&count[step_key(B, b[0], b[1], b[2])], 1);
}

// ------------------------------------------------------------------ scan ----
// start[0..n] = exclusive scan of count[0..n), count reset to zero.  Two
// launches: per-chunk sums, then the per-chunk scan, each workgroup adding the
// sum of the chunk sums before its own (integer sums: the order does not
// matter).  Chunks of kScanChunk counters, 256 threads.

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over the workgroup (nw waves); *total
// receives the sum.  sw: nw ints of LDS.  Contains barriers: call uniformly.
__device__ __forceinline__ int block_excl_scan(int v, int *sw, int nw, int *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = wave_incl_scan(v);
    if (lane == 63) sw[w] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        const int t = sw[k];
        pre += (k < w) ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

// Per-chunk sums into part[chunk].
__global__ void __launch_bounds__(256) k_scan_reduce(const int32_t *__restrict__ count,
                                                     int64_t n, int32_t *__restrict__ part) {
    __shared__ int sw[4];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int s = 0;
#pragma unroll
    for (int j = 0; j < kScanChunk / 256; ++j) {
        const int64_t i = base + j * 256 + threadIdx.x;
        s += (i < n) ? count[i] : 0;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sw[0] + sw[1] + sw[2] + sw[3];
}

// The last workgroup also writes start[n] (the total); workgroup 0 publishes
// the step index for the step's own binning: stepp[1] = stepp[0] (read by the
// kernels after the scan), stepp[0] += 1 (the next step).
__global__ void __launch_bounds__(256) k_scan_down(int32_t *__restrict__ count, int64_t n,
                                                   const int32_t *__restrict__ part,
                                                   int64_t nchunk, int32_t *__restrict__ start,
                                                   int64_t *__restrict__ stepp) {
    // chunk staged in LDS with one pad word per kRun (thread t owns kRun consecutive
    // counters; the odd stride kRun + 1 keeps the row reads off each other's banks)
    constexpr int kRun = kScanChunk / 256;
    static_assert(kScanChunk % 256 == 0 && (kRun & (kRun - 1)) == 0, "scan chunk: 256 x 2^k");
    __shared__ int buf[kScanChunk + kScanChunk / kRun];
    __shared__ int sw[4], sw2[4];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    const int t = threadIdx.x;
    int cv[kScanChunk / 256];
#pragma unroll
    for (int j = 0; j < kScanChunk / 256; ++j) {
        const int64_t i = base + j * 256 + t;
        cv[j] = (i < n) ? count[i] : 0;
    }
#pragma unroll
    for (int j = 0; j < kScanChunk / 256; ++j) {
        const int k = j * 256 + t;
        const int64_t i = base + k;
        if (i < n) count[i] = 0;
        buf[k + k / kRun] = cv[j];
    }
    // offset of the chunk: the sum of the chunk sums before it
    int pre = 0;
    for (int64_t c = t; c < (int64_t)blockIdx.x; c += 256) pre += part[c];
    for (int off = 32; off > 0; off >>= 1) pre += __shfl_xor(pre, off, 64);
    if ((t & 63) == 0) sw2[t >> 6] = pre;
    __syncthreads();
    const int off = sw2[0] + sw2[1] + sw2[2] + sw2[3];
    int s = 0;
    for (int j = 0; j < kRun; ++j) s += buf[t * (kRun + 1) + j];
    int total;
    int run = block_excl_scan(s, sw, 4, &total) + off;
    for (int j = 0; j < kRun; ++j) {
        const int c = buf[t * (kRun + 1) + j];
        buf[t * (kRun + 1) + j] = run;
        run += c;
    }
    __syncthreads();
    for (int j = 0; j < kScanChunk / 256; ++j) {
        const int k = j * 256 + t;
        const int64_t i = base + k;
        if (i < n) start[i] = buf[k + k / kRun];
    }
    if (blockIdx.x == nchunk - 1 && t == 0) start[n] = off + total;
    if (blockIdx.x == 0 && t == 0 && stepp) {
        const int64_t cur = stepp[0];
        stepp[1] = cur;
        stepp[0] = cur + 1;
    }
}

// ------------------------------------------------------------------ eval ----
constexpr int kMaxOff = 16;   // max stencil offsets per dimension (mhi - mlo + 1)

// six workgroups per CU: at most 80 VGPRs (66 used), 6 waves per SIMD to hide the
// latencies of the row loop (exp, sqrt, LDS), which at 5 waves showed as 23% idle
// VALU issue (53.0 -> 46.2 us on the shear box)
__global__ void __launch_bounds__(kBlock, 6) k_eval(const DevBox *__restrict__ Bs, int nbox,
                                                 const int64_t *__restrict__ stepp, int M,
                                                 const int32_t *__restrict__ start,
                                                 const int32_t *__restrict__ rank,
                                                 float4 *__restrict__ rec,
                                                 double4 *__restrict__ xs,
                                                 double4 *__restrict__ vrec) {
    __shared__ float sP[kMaxOff + 1][kBlock];   // prefix sums of the x factors
    __shared__ int s_rng[kMaxOff];               // per mz: reachable my in [lo, hi]
    const int64_t n = *stepp;
    if (n < M) return;
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)(blockIdx.x - B.blk_p) * kBlock + tid;
    const float cut = B.R2f + B.guard;
    // row classes (my, mz) whose row can meet the sphere for some offset in the
    // cell: for each mz the reachable my form one interval (the test is convex
    // in |my|); rows are summed in (mz, my) order, so the order of Z is fixed
    const int mlo1 = B.mlo[1], ny = B.mhi[1] - B.mlo[1] + 1;
    const int mlo2 = B.mlo[2], nz = B.mhi[2] - B.mlo[2] + 1;
    if (tid < nz) {
        const int dz = mlo2 + tid;
        const float az = (float)(dz >= 1 ? dz - 1 : -dz) * B.dxf[2];
        int lo = 1 << 20, hi = -(1 << 20);
        for (int k = 0; k < ny; ++k) {
            const int dy = mlo1 + k;
            const float ay = (float)(dy >= 1 ? dy - 1 : -dy) * B.dxf[1];
            if (fmaf(ay, ay, az * az) <= cut) {
                lo = min(lo, dy);
                hi = max(hi, dy);
            }
        }
        s_rng[tid] = lo <= hi ? ((lo + 512) | ((hi + 512) << 16)) : -1;
    }
    __syncthreads();
    if (p >= B.np) return;
    const int64_t np = B.np;
    const int64_t slot = (n - M) % (M + 1);
    const double *X = B.ring_x + slot * 3 * np;
    const float *Dd = (const float *)B.ring_d + slot * 3 * np;
    int b[3];
    double ph[3];
    for (int d = 0; d < 3; ++d) cell_of(X[d * np + p], B.L[d], B.dx[d], B.n[d], b[d], ph[d]);
    const float phx = (float)ph[0], phy = (float)ph[1], phz = (float)ph[2];
    // loads needed after the normalisation, issued now so that their latency
    // overlaps it
    const int32_t sk = start[step_key(B, b[0], b[1], b[2])];
    const int32_t rk = rank[B.poff + p];
    const float D0 = Dd[p], D1 = Dd[np + p], D2 = Dd[2 * np + p];
    const double x0 = B.x[p], x1 = B.x[np + p], x2 = B.x[2 * np + p];
    const int mlo0 = B.mlo[0], mhi0 = B.mhi[0];
    float hx = B.dxf[0], hy = B.dxf[1], hz = B.dxf[2], c = B.cexp;
    // box constants of the row loop, pinned in registers (a reload from the box
    // descriptor inside the loop would wait on the LDS counter)
    RowK K = row_consts(B);
    float cutv = cut;
    asm volatile("" : "+v"(K.R2f), "+v"(K.guard), "+v"(K.idx0), "+v"(K.dx0), "+v"(K.gs));
    asm volatile("" : "+v"(K.mlo0), "+v"(K.mhi0), "+v"(hx), "+v"(hy), "+v"(hz), "+v"(c),
                 "+v"(cutv));
    // prefix sums of the x factors (indexed by the row ends); raw v_exp_f32, the
    // arguments lie in [-(R + dx)^2 c, 0]
    sP[0][tid] = 0.0f;
    {
        float acc = 0.0f;
        for (int m = mlo0; m <= mhi0; ++m) {
            const float t = ((float)m - phx) * hx;
            acc += __builtin_amdgcn_exp2f(-(t * t) * c);
            sP[m - mlo0 + 1][tid] = acc;
        }
    }
    const int pid = (int)p;
    // y factor of row my by the ratio recurrence along y: gy(my + 1) = gy(my) r(my),
    // r(my + 1) = r(my) qy, with r(my) = exp2(-c hy^2 (2 (my - phy) + 1))
    const float qy = __builtin_amdgcn_exp2f(-2.0f * c * hy * hy);
    float Z = 0.0f;
    for (int iz = 0; iz < nz; ++iz) {
        const int rg = s_rng[iz];
        if (rg < 0) continue;
        const int mz = mlo2 + iz;
        const float tz = d1(mz, phz, hz);
        const float tz2 = tz * tz;
        const int ylo = (rg & 0xffff) - 512, yhi = (rg >> 16) - 512;
        const float ty0 = d1(ylo, phy, hy);
        float gyz = __builtin_amdgcn_exp2f(-fmaf(ty0, ty0, tz2) * c);
        float ry = __builtin_amdgcn_exp2f(-c * hy * fmaf(2.0f, ty0, hy));
        for (int my = ylo; my <= yhi; ++my) {
            const float ty = d1(my, phy, hy);
            const float ryz = fmaf(ty, ty, tz2);
            const float w = gyz;
            gyz *= ry;
            ry *= qy;
            if (ryz > cutv) continue;
            int lo, hi;
            row_range(phx, ryz, K, &B, slot, pid, my, mz, lo, hi);
            if (lo > hi) continue;
            Z = fmaf(w, sP[hi - mlo0 + 1][tid] - sP[lo - mlo0][tid], Z);
        }
    }
    const float Zv = Z * (float)B.dV;
    const float inv = -B.rhof_inv / Zv;
    const float ax = D0 * inv, ay = D1 * inv, az = D2 * inv;
    const int64_t slotr = (int64_t)sk + rk;
    const uint32_t ijk = (uint32_t)b[0] | ((uint32_t)b[1] << 11) | ((uint32_t)b[2] << 22);
    rec[2 * slotr] = make_float4(phx, phy, phz, __uint_as_float(ijk));
    rec[2 * slotr + 1] = make_float4(ax, ay, az, __int_as_float((int)p));
    // the current position x^n, in record order for the carrier gather, with the
    // particle index (exact in a double) for the gather's writes
    xs[slotr] = make_double4(x0, x1, x2, (double)p);
    // and v^n for Heun's second stage (x* = x^n + dt v^n), evaluated by the gather
    if (vrec && B.integ == 2) vrec[slotr] = make_double4(B.v[p], B.v[np + p], B.v[2 * np + p], 0.0);
}

__device__ __forceinline__ int wrap_index(int i, int N) {
    i %= N;
    return i < 0 ? i + N : i;
}

// --------------------------------------------------------- scatter bound ----
// Fixed-point range of each scatter pencil.  A node in x-block X receives only
// from particles whose base cell lies within the stencil's x offsets of the
// block, in the cell rows its row classes reach, each at most max_c |a| (the
// raw Gaussian is <= 1).  k_block_sums: for every cell row and x-block, the sum
// of max_c |a| over the records of the blocks holding those base cells
// (periodic; one or two runs of keys).  k_pencil_scale:
// for every pencil, the largest sum over (pencil row, X) of those entries over
// the reachable row classes bounds |f| on the pencil; its scale is 2^30 / bound.
__device__ __forceinline__ float rec_amax(const float4 *__restrict__ rec, int64_t r) {
    const float4 b = rec[2 * r + 1];
    return fmaxf(fabsf(b.x), fmaxf(fabsf(b.y), fabsf(b.z)));
}

__global__ void __launch_bounds__(kBlock) k_block_sums(const DevBox *__restrict__ Bs, int nbox,
                                                       const int64_t *__restrict__ stepp, int M,
                                                       const int32_t *__restrict__ start,
                                                       const float4 *__restrict__ rec,
                                                       float *__restrict__ bsum) {
    if (*stepp < M) return;
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_b; });
    const DevBox &B = Bs[bi];
    const int64_t e = (int64_t)(blockIdx.x - B.blk_b) * kBlock + threadIdx.x;
    const int nxb = B.nxb;
    if (e >= (int64_t)B.n[1] * B.n[2] * nxb) return;
    const int X = (int)(e % nxb);
    const int64_t row = B.key_off + (e - X);     // first key of the cell row
    // A node x of block X receives from base cells b0 = x - m, m in [mlo, mhi]:
    // the cells [16 X - mhi, min(16 X + 15, Nx - 1) - mlo] (periodic).  Their
    // blocks form one run of keys, or two when the cell range wraps (a short
    // last block can put cells of block nxb - 2 in the range of block 0).
    const int Nx = B.n[0];
    const int xhi = min((X << kXBlockShift) + (1 << kXBlockShift) - 1, Nx - 1);
    int clo = (X << kXBlockShift) - B.mhi[0];
    int chi = xhi - B.mlo[0];
    int k0a, k0b, k1a, k1b;                       // key runs [k0a, k0b), [k1a, k1b)
    if (chi - clo + 1 >= Nx) {
        k0a = 0, k0b = nxb, k1a = k1b = 0;
    } else {
        clo = wrap_index(clo, Nx);
        chi = wrap_index(chi, Nx);
        const int blo = clo >> kXBlockShift, bhi = chi >> kXBlockShift;
        if (clo <= chi) {
            k0a = blo, k0b = bhi + 1, k1a = k1b = 0;
        } else if (bhi >= blo) {                  // the two runs overlap: every block
            k0a = 0, k0b = nxb, k1a = k1b = 0;
        } else {
            k0a = blo, k0b = nxb, k1a = 0, k1b = bhi + 1;
        }
    }
    int g0[2], g1[2];
    g0[0] = start[row + k0a];
    g1[0] = start[row + k0b];
    g0[1] = (k1b > k1a) ? start[row + k1a] : 0;
    g1[1] = (k1b > k1a) ? start[row + k1b] : 0;
    // Records within a key sit in an arbitrary order (atomic ranks), so the sum
    // runs in FP64, exact for FP32 terms unless their exponents spread over
    // ~29 bits, and is rounded up to FP32: the bound, and with it the
    // fixed-point scale and the forcing, do not depend on that order.
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll 4
        for (int g = g0[k]; g < g1[k]; ++g) s += (double)rec_amax(rec, g);
    bsum[B.key_off + e] = __double2float_ru(s);
}

static_assert(kBlock % kBoundXChunk == 0 && (kBoundXChunk & (kBoundXChunk - 1)) == 0,
              "the window load maps a power-of-two chunk of x-blocks onto the block");

__global__ void __launch_bounds__(kBlock) k_pencil_scale(const DevBox *__restrict__ Bs, int nbox,
                                                         const int64_t *__restrict__ stepp, int M,
                                                         const float *__restrict__ bsum,
                                                         float *__restrict__ pscale,
                                                         int64_t npen, int32_t *__restrict__ pctr) {
    // the scatter that follows hands its pencils out from these counters
    if (blockIdx.x == 0 && threadIdx.x < kXcds) pctr[threadIdx.x] = 0;
    if (*stepp < M) return;
    // each XCD (its own L2) takes one contiguous run of pencils, whose windows of
    // block sums overlap
    const int64_t pen = xcd_block(blockIdx.x, gridDim.x);
    if (pen >= npen) return;
    extern __shared__ float win[];              // [WZ][WY][kBoundXChunk] of bsum
    __shared__ int s_off[256];                  // window row offset of each class
    __shared__ int s_wcnt[kBlock / 64];
    __shared__ float s_max[kBlock / 64];
    const int bi = box_of_block(Bs, nbox, pen, [](const DevBox &b) { return b.blk_t; });
    const DevBox &B = Bs[bi];
    const int t = (int)(pen - B.blk_t);
    const int T1 = B.T[1], T2 = B.T[2];
    const int o1 = (t % B.ntile[1]) * T1;
    const int o2 = (t / B.ntile[1]) * T2;
    const int Ny = B.n[1], Nz = B.n[2], nxb = B.nxb;
    const int e1 = min(T1, Ny - o1);
    const int e2 = min(T2, Nz - o2);
    const int mlo1 = B.mlo[1], mhi1 = B.mhi[1], mlo2 = B.mlo[2], mhi2 = B.mhi[2];
    const int ny = mhi1 - mlo1 + 1, nz = mhi2 - mlo2 + 1;
    const int WY = e1 + mhi1 - mlo1, WZ = e2 + mhi2 - mlo2;
    const int tid = threadIdx.x;
    // reachable row classes in (dz, dy) order: a deterministic compaction
    // (ballot ranks + wave counts), so the FP32 class sums below, the bound and
    // the pencil's fixed-point scale do not depend on wave timing
    int ncls = 0;
    for (int c0 = 0; c0 < ny * nz; c0 += kBlock) {
        const int k = c0 + tid;
        bool reach = false;
        if (k < ny * nz) {
            const int dy = mlo1 + k % ny, dz = mlo2 + k / ny;
            const float ay = (float)(dy >= 1 ? dy - 1 : -dy) * B.dxf[1];
            const float az = (float)(dz >= 1 ? dz - 1 : -dz) * B.dxf[2];
            reach = fmaf(ay, ay, az * az) <= B.R2f + B.guard;
        }
        const uint64_t mask = __ballot(reach);
        const int lane = tid & 63, w = tid >> 6;
        if (lane == 0) s_wcnt[w] = __popcll(mask);
        __syncthreads();
        int before = ncls, total = ncls;
        for (int q = 0; q < kBlock / 64; ++q) {
            before += (q < w) ? s_wcnt[q] : 0;
            total += s_wcnt[q];
        }
        if (reach) {
            const int i = before + __popcll(mask & ((1ull << lane) - 1ull));
            // class (dy, dz) = (mlo1 + k mod ny, mlo2 + k / ny): the window row of
            // pencil row (y, z) is (z + mhi2 - dz) WY + y + mhi1 - dy
            s_off[i] = (mhi2 - (mlo2 + k / ny)) * WY + mhi1 - (mlo1 + k % ny);
        }
        ncls = total;
        __syncthreads();
    }
    float bmax = 0.0f;
    for (int X0 = 0; X0 < nxb; X0 += kBoundXChunk) {
        const int nx = min(kBoundXChunk, nxb - X0);
        // window cell rows b1 = o1 - mhi1 + wy, b2 = o2 - mhi2 + wz (periodic): thread
        // t fills column X = t mod 16 of rows t/16, t/16 + 16, ... (entries past nx
        // are zero), its (wy, wz) advanced without a division per entry
        {
            constexpr int kRowStep = kBlock / kBoundXChunk;
            constexpr int kBatch = 32;
            const int X = tid & (kBoundXChunk - 1);
            const int Xc = min(X, nx - 1);
            const int total = WZ * WY;
            int r0 = tid / kBoundXChunk;
            int wz = r0 / WY, wy = r0 - wz * WY;
            const int sz = kRowStep / WY, sy = kRowStep - sz * WY;
            for (; r0 < total; r0 += kBatch * kRowStep) {
                // kBatch loads in flight: every address is valid (rows past the
                // window re-read its last plane, padding columns column nx - 1) and
                // the values are masked when stored
                float v[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    int b1 = o1 - mhi1 + wy, b2 = o2 - mhi2 + min(wz, WZ - 1);
                    b1 += (b1 < 0) ? Ny : 0;
                    b1 -= (b1 >= Ny) ? Ny : 0;
                    b2 += (b2 < 0) ? Nz : 0;
                    b2 -= (b2 >= Nz) ? Nz : 0;
                    v[u] = bsum[B.key_off + ((int64_t)b2 * Ny + b1) * nxb + X0 + Xc];
                    wy += sy;
                    wz += sz;
                    if (wy >= WY) {
                        wy -= WY;
                        ++wz;
                    }
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int r = r0 + u * kRowStep;
                    if (r < total) win[r * kBoundXChunk + X] = (X < nx) ? v[u] : 0.0f;
                }
            }
        }
        __syncthreads();
        // four x-blocks per output (128-bit LDS reads; entries past nx are zero); two
        // neighbouring lanes per output, each summing every other class (two
        // accumulators), combined in a fixed order
        const int nq = (nx + 3) / 4;
        for (int k2 = tid; k2 < 2 * e1 * e2 * nq; k2 += kBlock) {
            const int h = k2 & 1, k = k2 >> 1;
            const int Xq = k % nq, r = k / nq;
            const int y = r % e1, z = r / e1;
            const float *wp = win + (z * WY + y) * kBoundXChunk + 4 * Xq;
            float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
            int ci = h;
            for (; ci + 2 < ncls; ci += 4) {
                const float4 v0 = *(const float4 *)(wp + s_off[ci] * kBoundXChunk);
                const float4 v1 = *(const float4 *)(wp + s_off[ci + 2] * kBoundXChunk);
                a0.x += v0.x; a0.y += v0.y; a0.z += v0.z; a0.w += v0.w;
                a1.x += v1.x; a1.y += v1.y; a1.z += v1.z; a1.w += v1.w;
            }
            if (ci < ncls) {
                const float4 v0 = *(const float4 *)(wp + s_off[ci] * kBoundXChunk);
                a0.x += v0.x; a0.y += v0.y; a0.z += v0.z; a0.w += v0.w;
            }
            float4 sum = make_float4(a0.x + a1.x, a0.y + a1.y, a0.z + a1.z, a0.w + a1.w);
            sum.x += __shfl_xor(sum.x, 1, 64);
            sum.y += __shfl_xor(sum.y, 1, 64);
            sum.z += __shfl_xor(sum.z, 1, 64);
            sum.w += __shfl_xor(sum.w, 1, 64);
            bmax = fmaxf(bmax, fmaxf(fmaxf(sum.x, sum.y), fmaxf(sum.z, sum.w)));
        }
        __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) bmax = fmaxf(bmax, __shfl_xor(bmax, off, 64));
    if ((tid & 63) == 0) s_max[tid >> 6] = bmax;
    __syncthreads();
    if (tid == 0) {
        float bound = 0.0f;
        for (int w = 0; w < kBlock / 64; ++w) bound = fmaxf(bound, s_max[w]);
        bound *= 1.0001f;   // margin for the FP32 roundings of the sums
        pscale[pen] = (bound > 0.0f && bound < 3.0e38f) ? 1073741824.0f / bound : 1.0f;
    }
}

// --------------------------------------------------------------- scatter ----

// Rows of one work item of the scatter: a band of KB (kMinBand..kMaxBand, the
// plan's rows per item) consecutive stencil rows dy of one plane dz (all lanes of
// a pass take the same band).

// Fourth descriptor word of a raw (unformatted, unswizzled) gfx9 buffer resource.
constexpr int kBufferWord3 = 0x00020000;

// One 16-byte half of a record, at a byte offset from the record array.
__device__ __forceinline__ float4 rec_load(__amdgpu_buffer_rsrc_t r, int byteoff) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, byteoff, 0, 0));
}

// Makes the four values available in registers at this point (the compiler
// places the wait for their load here); emits no instruction.
__device__ __forceinline__ void pin4(float4 &v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
}

// Contribution to the integer tile: v_cvt_rpi_i32_f32 rounds to floor(v + 0.5)
// in one instruction (|v| < 2^30 by the choice of scale; the error of one term
// is at most half a unit; ties, which round up, have measure zero).
__device__ __forceinline__ uint32_t fixed32(float v) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return (uint32_t)r;
}


// Pencils of nodes: the whole x extent of the box times T1 x T2 nodes in (y, z),
// each taken by one workgroup.  Owner computes: every node of the pencil is
// written once, by that workgroup; no global atomics on the grid.
//
// Row classes.  Every stencil row of a particle is a relative offset (dy, dz)
// from its base cell (b0, b1, b2) -- its class.  For class (dy, dz) the
// particles whose row lies on pencil plane z are those with b2 = o2 + z - dz and
// b1 in [o1 - dy, o1 - dy + e1): since records are sorted by cell and a pencil
// spans all of x, that is one contiguous record range (two when it wraps in y).
// Classes are taken KB rows at a time (consecutive dy of one dz): a wave
// takes a band and runs one lane per (particle, band) over the ranges of all e2
// planes, so its 64 lanes walk rows of the same relative offsets, whose lengths
// differ by at most a node or two, no row is ever cut by the tile, and the
// record load and decode of an item serve KB rows.  Records are read straight
// from the cell-sorted array (L2) through a buffer resource, one item ahead of
// use, so the loads overlap the previous item's LDS atomics (they wait on a
// different counter).  Per row, the weight of the first node is one exp2; the
// ratio to the next node is the item's factor exp2(c hx^2 (2 phi_x - 1)) times a
// tabulated power exp2(-2 c hx^2 m) of the first node's offset m.
//
// The LDS tile keeps each pencil row unwrapped in x: a row's nodes b0 + m,
// m in [mlo, mhi], sit at index b0 + m - mlo of a row of Nx + (mhi - mlo) + 1
// words, and the store folds the ends back onto the periodic row.
//
// Accumulation is exact integer arithmetic: each contribution a*w is rounded to
// an int32 with the per-pencil scale 2^30 / A, where A bounds the sum of |a w|
// over the contributions to any node of the pencil (k_pencil_scale), and
// added with ds_add_u32 (the FP32 LDS atomic runs ~40x slower on gfx950).
// Integer additions commute, so the forcing does not depend on the order of the
// adds.
// TZ: the plan's pencil depth rounded up to a power of two (>= every box's T2);
// a row class has at most 2 TZ record ranges.  NT: threads per workgroup.  KB:
// rows per work item.  RES: resident workgroups taking pencils in turn (else one
// workgroup per pencil, the grid padded to a multiple of 8).
template <int TZ, int NT, int KB, bool RES>
__global__ void __launch_bounds__(NT) k_scatter(const DevBox *__restrict__ Bs,
                                                           int nbox,
                                                           const int64_t *__restrict__ stepp,
                                                           int M,
                                                           const int32_t *__restrict__ start,
                                                           const float4 *__restrict__ rec,
                                                           const float *__restrict__ pscale,
                                                           int64_t npen, int64_t npart,
                                                           int32_t *__restrict__ pctr,
                                                           int run, int lds_words) {
    extern __shared__ int32_t lds[];
    __shared__ int s_cls[256];            // row bands: dz, first dy, rows
    __shared__ int s_ncls;
    __shared__ int s_next;                // next class to hand out
    __shared__ float s_q[32];             // exp2(-2 c hx^2 m), m = mlo .. mhi in x
    __shared__ int s_pen;                 // the pencil in hand
    __shared__ int s_clsbox;              // the box whose bands s_cls, s_q hold
    const int tid = threadIdx.x, lane = tid & 63;
    // Workgroups take pencils until none is left.  Workgroups are dealt to the 8
    // XCDs round-robin, so the pencils are cut into 8 contiguous runs (their
    // record windows overlap, within one L2) and workgroup w drains run w mod 8
    // first: its first pencil by its index (the first gridDim/8 pencils of every
    // run), the rest from the run's counter, then the other runs in turn.  Every
    // workgroup ends once all runs are drained, whatever XCD it landed on.  With
    // one workgroup per pencil (RES false, gridDim/8 = run) no counter is touched.
    const int home = (int)(blockIdx.x % kXcds);
    const int first = (int)(gridDim.x / kXcds);
    constexpr bool again = RES;           // a workgroup may take more than one pencil
    int tries = again ? 0 : kXcds;        // runs found drained (thread 0)
    auto pencil_of = [&](int r, int i) -> int {
        const int64_t pn = (int64_t)r * run + first + i;
        return (first + i < run && pn < npen) ? (int)pn : -1;
    };
    auto claim_next = [&]() -> int {      // thread 0: next pencil, npen when none
        while (tries < kXcds) {
            const int r = (home + tries) % kXcds;
            const int pn = pencil_of(r, atomicAdd(&pctr[r], 1));
            if (pn >= 0) return pn;
            ++tries;
        }
        return (int)npen;
    };
    // the LDS starts undefined: clear it once; every pencil leaves it clear (the
    // barriers before its first use order the clearing)
    for (int i = tid; i < lds_words; i += NT) lds[i] = 0;
    // the first pencil from the workgroup's index: uniform, so the box constants
    // below are scalar loads issued at once (no LDS round trip); a resident
    // workgroup past the end of its run claims one instead
    const int j = (int)(blockIdx.x / kXcds);
    const int64_t p0 = (int64_t)home * run + j;
    int pen = (j < run && p0 < npen) ? (int)p0 : -1;
    if (again) {
        if (tid == 0) {
            s_clsbox = -1;
            if (pen < 0) s_pen = claim_next();
        }
        __syncthreads();
        if (pen < 0) pen = __builtin_amdgcn_readfirstlane(s_pen);
    } else if (pen < 0) {
        return;                           // past the last pencil
    }
    for (;;) {
        if (pen >= npen) break;
        // the next pencil of the home run is claimed now and checked after the
        // deposition, so the atomic's latency hides behind it
        int claim = 0;
        if (tid == 0 && tries < kXcds) claim = atomicAdd(&pctr[(home + tries) % kXcds], 1);
        const int64_t n = *stepp;
        const int bi = box_of_block(Bs, nbox, pen, [](const DevBox &b) { return b.blk_t; });
        const DevBox &B = Bs[bi];
        const int t = (int)(pen - B.blk_t);
        const int T1 = B.T[1], T2 = B.T[2];
        const int o1 = (t % B.ntile[1]) * T1;
        const int o2 = (t / B.ntile[1]) * T2;
        const int Nx = B.n[0], Ny = B.n[1], Nz = B.n[2];
        const int e1 = min(T1, Ny - o1);
        const int e2 = min(T2, Nz - o2);
        const int PXa = B.pxa;                 // words per unwrapped row (per component)
        int32_t *acc = lds;                    // [T2][T1][PXa][3]
        int *tab = lds + B.lds_tab;            // record-start table of the window
        const int mlo0 = B.mlo[0], mhi0 = B.mhi[0];
        const int mlo1 = B.mlo[1], mhi1 = B.mhi[1];
        const int mlo2 = B.mlo[2], mhi2 = B.mhi[2];
        float scale = 1.0f;
        if (n >= M) {
            const int WY = e1 + mhi1 - mlo1;      // window cell rows in y, z
            const int WZ = e2 + mhi2 - mlo2;
            const int TW = WY + 2;                // table row: WY + 1 row starts, then end of plane
            // tab[wz][j] = first record of cell row b1 = (o1 - mhi1 + j) mod Ny of window
            // plane b2 = (o2 - mhi2 + wz) mod Nz, j <= WY; tab[wz][WY + 1] = end of the plane
            for (int k = tid; k < WZ * TW; k += NT) {
                const int wz = k / TW, j = k - wz * TW;
                const int b2 = wrap_index(o2 - mhi2 + wz, Nz);
                const int64_t plane = B.key_off + (int64_t)b2 * Ny * B.nxb;
                const int b1 = (j <= WY) ? wrap_index(o1 - mhi1 + j, Ny) : Ny;
                tab[k] = start[plane + (int64_t)b1 * B.nxb];
            }
            // row classes that some particle can reach: nearest approach of the row to
            // a base-cell offset in [0, 1)^2 within the cut-off.  They depend on the box
            // only: kept from the previous pencil of the same box
            const float cut = B.R2f + B.guard;
            const int ny = mhi1 - mlo1 + 1, nz = mhi2 - mlo2 + 1;
            const bool fresh = !again || s_clsbox != bi;
            if (tid == 0) {
                if (fresh) s_ncls = 0;
                s_next = 0;
            }
            if (fresh && tid <= mhi0 - mlo0)
                s_q[tid] = exp2f(-2.0f * B.cexp * B.dxf[0] * B.dxf[0] * (float)(mlo0 + tid));
            __syncthreads();
            if (fresh && tid < nz) {
                // the rows dy of plane dz that some particle reaches form one interval
                // (the test is convex in |dy|); it is cut into bands of KB rows
                const int dz = mlo2 + tid;
                const float az = (float)(dz >= 1 ? dz - 1 : -dz) * B.dxf[2];
                int lo = 1 << 20, hi = -(1 << 20);
                for (int k = 0; k < ny; ++k) {
                    const int dy = mlo1 + k;
                    const float ay = (float)(dy >= 1 ? dy - 1 : -dy) * B.dxf[1];
                    if (fmaf(ay, ay, az * az) <= cut) {
                        lo = min(lo, dy);
                        hi = max(hi, dy);
                    }
                }
                for (int dy0 = lo; dy0 <= hi; dy0 += KB) {
                    const int nb = min(KB, hi - dy0 + 1);
                    s_cls[atomicAdd(&s_ncls, 1)] = (dz + 64) | ((dy0 + 64) << 8) | (nb << 16);
                }
            }
            __syncthreads();
            if (again && tid == 0) s_clsbox = bi;  // read again only after the pencil's last barrier
            // records of window plane wz, cell rows j in [ja, ja + len): [g0, g1) and,
            // when the rows wrap past Ny, [h0, h1)
            auto ranges = [&](int wz, int ja, int len, int &g0, int &g1, int &h0, int &h1) {
                const int *T = tab + wz * TW;
                const int b1a = wrap_index(o1 - mhi1 + ja, Ny);
                g0 = T[ja];
                if (b1a + len <= Ny) {
                    g1 = (b1a + len == Ny) ? T[WY + 1] : T[ja + len];
                    h0 = h1 = 0;
                } else {
                    g1 = T[WY + 1];
                    h0 = T[ja + (Ny - b1a)];
                    h1 = T[ja + len];
                }
            };
            // fixed-point scale of the pencil (k_pencil_scale)
            scale = pscale[pen];
            // the records through a buffer resource: 32-bit byte offsets
            const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
                (void *)rec, (short)0, (int)(32 * npart), kBufferWord3);
            const int64_t slot = (n - M) % (M + 1);
            float hx = B.dxf[0], hy = B.dxf[1], hz = B.dxf[2];
            float c = B.cexp;
            const float qx = exp2f(-2.0f * c * hx * hx);
            const float chx2 = c * hx * hx;
            // box constants of the row loop, pinned in registers: reloading them from
            // the box descriptor inside the loop would wait on the LDS counter, i.e.
            // on the previous row's atomics
            RowK K = row_consts(B);
            float cutv = cut;
            asm volatile("" : "+v"(K.R2f), "+v"(K.guard), "+v"(K.idx0), "+v"(K.dx0), "+v"(K.gs));
            asm volatile("" : "+v"(K.mlo0), "+v"(K.mhi0), "+v"(hx), "+v"(hy), "+v"(hz), "+v"(c),
                         "+v"(cutv));
            const int ncls = s_ncls;
            const int nr = 2 * e2;
            // classes are handed out to the waves as they finish the previous one (the
            // classes differ in size, so a fixed round-robin leaves waves idle at the end)
            for (;;) {
                int cn = 0;
                if (lane == 0) cn = atomicAdd(&s_next, 1);
                const int ci = __builtin_amdgcn_readfirstlane(cn);
                if (ci >= ncls) break;
                const int clw = s_cls[ci];
                const int dz = (clw & 255) - 64, dy0 = ((clw >> 8) & 255) - 64, nb = clw >> 16;
                // rows dy0 .. dy0 + nb - 1 of plane dz.  The records whose band reaches the
                // pencil: cell rows b1 in [o1 - dy0 - nb + 1, o1 - dy0 + e1), window rows
                // ja .. ja + len - 1.  Lane k < 2 e2: part (k & 1) of the records of plane
                // k >> 1; part 0 holds cell rows b1 in [b1a, ...), part 1 (wrapped past
                // Ny) b1 in [0, ...).  A record's window row is b1 + jo (jo uniform over
                // the range); its row dy0 + r lands on pencil row b1 + jo + r - nb + 1
                // and LDS node index b1 PXa + b0 + m + rowoff + r PXa.
                const int ja = mhi1 - dy0 - nb + 1, wlen = e1 + nb - 1;
                const int b1a = wrap_index(o1 - dy0 - nb + 1, Ny);
                int len = 0, gb = 0, rowoff = 0, jo = 0;
                if (lane < nr) {
                    int g0, g1, h0, h1;
                    ranges((lane >> 1) + mhi2 - dz, ja, wlen, g0, g1, h0, h1);
                    gb = (lane & 1) ? h0 : g0;
                    len = (lane & 1) ? h1 - h0 : g1 - g0;
                    jo = -b1a + ((lane & 1) ? Ny : 0);
                    rowoff = ((lane >> 1) * T1 + jo - nb + 1) * PXa - mlo0;
                }
                const int incl = wave_incl_scan(len);
                const int total = __shfl(incl, 63, 64);
                if (total == 0) continue;
                // item q of range k is record q + off_k (pre_k <= q < pre_k + len_k)
                const int pre = incl - len;
                const int off = gb - pre;
                constexpr int kMaxRanges = 2 * TZ;
                int pre_k[kMaxRanges], off_k[kMaxRanges], row_k[kMaxRanges], jo_k[kMaxRanges];
    #pragma unroll
                for (int k = 0; k < kMaxRanges; ++k) {
                    pre_k[k] = __builtin_amdgcn_readlane(pre, k);
                    off_k[k] = __builtin_amdgcn_readlane(off, k);
                    row_k[k] = __builtin_amdgcn_readlane(rowoff, k);
                    jo_k[k] = __builtin_amdgcn_readlane(jo, k);
                }
                // byte offset of item q's record, and the LDS row offset and window-row
                // offset of its range
                auto record_of = [&](int q, int &ro, int &jr) -> int {
                    int o = off_k[0];
                    ro = row_k[0];
                    jr = jo_k[0];
    #pragma unroll
                    for (int k = 1; k < kMaxRanges; ++k)
                        if (k < nr && q >= pre_k[k]) {
                            o = off_k[k];
                            ro = row_k[k];
                            jr = jo_k[k];
                        }
                    return (q + o) << 5;
                };
                // lane l takes the items [l P, l P + P): the lanes of one pass are spread
                // over the whole range, so fewer of them add into the same node or bank
                const int P = (total + 63) >> 6;
                int q = lane * P;
                const int qend = min(q + P, total);
                // one band of an item: per row the pencil test, the sphere test, the
                // range, the first weight, then the node walk
                const float tzc = (float)dz;
                auto band = [&](const float4 qa, const float4 qb, const int ro, const int jr) {
                    const uint32_t ijk = __float_as_uint(qa.w);
                    const int b0 = (int)(ijk & 2047u);
                    const int b1 = (int)((ijk >> 11) & 2047u);
                    const int rowx = (int)__umul24((unsigned)b1, (unsigned)PXa) + b0 + ro;
                    const int y0 = b1 + jr - nb + 1;          // pencil row of the band's first row
                    const float tzv = (tzc - qa.z) * hz;
                    const float tz2 = tzv * tzv;
                    // ratio w(m + 1) / w(m) along a row is exp2(c hx^2 (2 phi_x - 1)) times
                    // s_q[m - mlo] = exp2(-2 c hx^2 m); the amplitudes carry the scale
                    const float ra = __builtin_amdgcn_exp2f(chx2 * fmaf(2.0f, qa.x, -1.0f));
                    const float sax = qb.x * scale, say = qb.y * scale, saz = qb.z * scale;
    #pragma unroll
                    for (int r = 0; r < KB; ++r) {
                        if (r >= nb) break;
                        const int y = y0 + r;
                        if (y < 0 || y >= e1) continue;
                        const int dy = dy0 + r;
                        const float tyv = d1(dy, qa.y, hy);
                        const float ryz = fmaf(tyv, tyv, tz2);
                        if (ryz > cutv) continue;
                        int rlo, rhi;
                        row_range(qa.x, ryz, K, &B, slot, __float_as_int(qb.w), dy, dz, rlo, rhi);
                        if (rlo > rhi) continue;
                        // raw v_exp_f32: the argument lies in [-2 R^2 c, 0], far from underflow
                        const float t0 = ((float)rlo - qa.x) * hx;
                        const float w = __builtin_amdgcn_exp2f(-fmaf(t0, t0, ryz) * c);
                        // weight ratio of the first step along the row: the item's factor
                        // times the tabulated power of the first node
                        float rr = ra * s_q[rlo - K.mlo0];
                        // contributions a_c w of the row's first node, advanced along the row
                        // by the weight ratio rr (itself advanced by qx)
                        float cx = sax * w, cy = say * w, cz = saz * w;
                        int a = 3 * (rowx + rlo + r * PXa);
                        int cntn = rhi - rlo + 1;
                        do {
                            atomicAdd((uint32_t *)&lds[a], fixed32(cx));
                            atomicAdd((uint32_t *)&lds[a + 1], fixed32(cy));
                            atomicAdd((uint32_t *)&lds[a + 2], fixed32(cz));
                            cx *= rr;
                            cy *= rr;
                            cz *= rr;
                            rr *= qx;
                            a += 3;
                        } while (--cntn != 0);
                    }
                };
                // records are fetched one item ahead into two register sets used in
                // turn (no copies between them).  The fetch is unconditional (the last
                // item re-reads its own record) and each set is pinned before the next
                // fetch is issued, so the wait for a set never waits for the younger
                // fetch behind it.
                float4 ra0, rb0, ra1, rb1;
                int ro0 = 0, ro1 = 0, jr0 = 0, jr1 = 0;
                if (q < qend) {
                    const int g = record_of(q, ro0, jr0);
                    ra0 = rec_load(rsrc, g);
                    rb0 = rec_load(rsrc, g + 16);
                }
                while (q < qend) {
                    pin4(ra0);
                    pin4(rb0);
                    {
                        const int g = record_of(min(q + 1, qend - 1), ro1, jr1);
                        ra1 = rec_load(rsrc, g);
                        rb1 = rec_load(rsrc, g + 16);
                    }
                    band(ra0, rb0, ro0, jr0);
                    if (++q >= qend) break;
                    pin4(ra1);
                    pin4(rb1);
                    {
                        const int g = record_of(min(q + 1, qend - 1), ro0, jr0);
                        ra0 = rec_load(rsrc, g);
                        rb0 = rec_load(rsrc, g + 16);
                    }
                    band(ra1, rb1, ro1, jr1);
                    ++q;
                }
            }
        }
        __syncthreads();
        // store: node x of a pencil row = index x - mlo plus its periodic images
        // x + Nx - mlo (for x < mhi) and x - Nx - mlo (for x >= Nx + mlo).  Each wave
        // stores whole pencil rows, lanes along x, so the row and its place in the
        // box are wave-uniform and no lane divides.  When the workgroup may take
        // another pencil, every word it reads is cleared for it (the deposition
        // writes no other word)
        float *f = (float *)B.f;
        const float inv = 1.0f / scale;
        const int64_t ng = (int64_t)Nx * Ny * Nz;
        const int nw = NT >> 6;
        const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
        int ly = wv % e1, lz = wv / e1;
        for (int r = wv; r < e1 * e2; r += nw) {
            float *fr = f + ((int64_t)(o2 + lz) * Ny + (o1 + ly)) * Nx;
            const int base = 3 * ((lz * T1 + ly) * PXa - mlo0);
            for (int x = lane; x < Nx; x += 64) {
                const int a = base + 3 * x;
                int v0 = acc[a], v1 = acc[a + 1], v2 = acc[a + 2];
                if (again) acc[a] = acc[a + 1] = acc[a + 2] = 0;
                if (x < mhi0) {
                    const int a2 = a + 3 * Nx;
                    v0 += acc[a2];
                    v1 += acc[a2 + 1];
                    v2 += acc[a2 + 2];
                    if (again) acc[a2] = acc[a2 + 1] = acc[a2 + 2] = 0;
                }
                if (x >= Nx + mlo0) {
                    const int a2 = a - 3 * Nx;
                    v0 += acc[a2];
                    v1 += acc[a2 + 1];
                    v2 += acc[a2 + 2];
                    if (again) acc[a2] = acc[a2 + 1] = acc[a2 + 2] = 0;
                }
                fr[x] = (float)v0 * inv;
                fr[ng + x] = (float)v1 * inv;
                fr[2 * ng + x] = (float)v2 * inv;
            }
            // next row of this wave: r + nw = (lz, ly) advanced by nw rows of e1
            ly += nw;
            while (ly >= e1) {
                ly -= e1;
                ++lz;
            }
        }
        if (!again) break;
        // the record-start table too (another box's pencil may lay accumulators there)
        if (n >= M) {
            const int tw = (e2 + mhi2 - mlo2) * (e1 + mhi1 - mlo1 + 2);
            for (int k = tid; k < tw; k += NT) tab[k] = 0;
        }
        if (tid == 0) {
            int nxt = (int)npen;
            if (tries < kXcds) {
                nxt = pencil_of((home + tries) % kXcds, claim);
                if (nxt < 0) {
                    ++tries;
                    nxt = claim_next();
                }
            }
            s_pen = nxt;
        }
        __syncthreads();
        pen = __builtin_amdgcn_readfirstlane(s_pen);
    }
}

// Carrier at the particles, visited in the cell order of their delayed
// positions (record order of level n - M): particles move far less than a cell
// in M steps, so neighbouring threads read neighbouring carrier nodes and the
// field streams through L2 about once, instead of eight scattered rows per
// particle.  x^n arrives in record order from the evaluation kernel; the FP64
// trilinear value (plus the mean shear) is stored in particle order, where the
// update reads it.
// LAP: also lap u at x^n (Faxen term, added mass); GRAD: grad u at x^n (added
// mass); HEUN: the carrier (and, with LAP, lap u) at Heun's x* = x^n + dt v^n.
// These go to aux[k][particle], k = 0 lap, 1..3 grad (d_x u, d_y u, d_z u), 4 u(x*),
// 5 lap u(x*), for the boxes that use them.
template <bool LAP, bool GRAD, bool HEUN>
__global__ void __launch_bounds__(kBlock) k_gather_sorted(const DevBox *__restrict__ Bs, int nbox,
                                                          int64_t nblk,
                                                          const int64_t *__restrict__ stepp,
                                                          int M, const double4 *__restrict__ xs,
                                                          double4 *__restrict__ up,
                                                          double4 *__restrict__ aux, int64_t npt,
                                                          const double4 *__restrict__ vrec,
                                                          double dt) {
    const int64_t n = *stepp;
    if (n < M) return;
    // workgroups are dealt to the 8 XCDs round-robin; give each XCD (its own L2)
    // one contiguous eighth of the records, so that neighbouring particles share
    // the carrier lines they read
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblk) return;
    const int bi = box_of_block(Bs, nbox, blk, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int64_t r = (blk - B.blk_p) * kBlock + threadIdx.x;
    if (r >= B.np) return;
    // the records of a box are [poff, poff + np): its cells follow the cells of
    // the boxes before it in the scanned key space
    const double4 x4 = xs[B.poff + r];
    double xp[3] = {x4.x, x4.y, x4.z};
    double u[3];
    trilinear<float>(B, (const float *)B.u, xp, u);
    // results go to the particle's own slot, so that the update reads them in
    // particle order (one line per 2 particles rather than one per particle)
    const int64_t slot = B.poff + (int64_t)x4.w;
    up[slot] = make_double4(u[0], u[1], u[2], 0.0);
    const bool lap = LAP && (B.fax != 0.0 || B.am_mf != 0.0 || B.bs_k != 0.0);
    const bool grad = GRAD && B.am_mf != 0.0;
    double l[3], g[9];
    if (lap && grad)
        trilinear_stencils<float, true, true>(B, (const float *)B.u, xp, l, g);
    else if (lap)
        trilinear_stencils<float, true, false>(B, (const float *)B.u, xp, l, g);
    else if (grad)
        trilinear_stencils<float, false, true>(B, (const float *)B.u, xp, l, g);
    if (lap) aux[slot] = make_double4(l[0], l[1], l[2], 0.0);
    if (grad) {
        // column j of the gradient: (d_j u_x, d_j u_y, d_j u_z)
        for (int j = 0; j < 3; ++j)
            aux[(1 + j) * npt + slot] = make_double4(g[j], g[3 + j], g[6 + j], 0.0);
    }
    if (HEUN && B.integ == 2) {
        const double4 v4 = vrec[B.poff + r];
        const double x2[3] = {xp[0] + dt * v4.x, xp[1] + dt * v4.y, xp[2] + dt * v4.z};
        double u2[3];
        trilinear<float>(B, (const float *)B.u, x2, u2);
        aux[4 * npt + slot] = make_double4(u2[0], u2[1], u2[2], 0.0);
        if (lap) {
            double l2[3];
            trilinear_laplacian<float>(B, (const float *)B.u, x2, l2);
            aux[5 * npt + slot] = make_double4(l2[0], l2[1], l2[2], 0.0);
        }
    }
}

// Self term of particle p at position pos (the App. E disturbance of the last
// injection, level n-1-M) into vs and, when FAX, the Faxen terms: up gets
// fax lap u, vs gets fax lap v_self.
template <bool FAX>
__device__ __forceinline__ void self_terms(const DevBox &B, int64_t p, int64_t n, int M, int selfc,
                                           const double pos[3], double up[3], double vs[3],
                                           const double (&lu_pre)[3], bool use_pre) {
    const int64_t np = B.np;
    vs[0] = vs[1] = vs[2] = 0.0;
    const bool live = selfc && n >= M + 1;
    const int64_t ss = (n - 1 - M) % (M + 1);
    const double *Xs = B.ring_x + ss * 3 * np;
    const float *Ds = (const float *)B.ring_d + ss * 3 * np;
    if (live) {
        float r[3];
        for (int d = 0; d < 3; ++d) {
            double rd = pos[d] - Xs[d * np + p];
            rd -= B.L[d] * rint(rd / B.L[d]);
            r[d] = (float)rd;
        }
        float v0, v1, v2;
        self_disturbance32(r[0], r[1], r[2], Ds[p], Ds[np + p], Ds[2 * np + p], B.s2sf,
                           B.preff, v0, v1, v2);
        vs[0] = v0;
        vs[1] = v1;
        vs[2] = v2;
    }
    if (FAX && B.fax != 0.0) {
        // Faxen term (a_p^2/6) lap u~: grid Laplacian minus the self part
        double lu[3], ls[3] = {0.0, 0.0, 0.0};
        if (use_pre) {
            for (int d = 0; d < 3; ++d) lu[d] = lu_pre[d];
        } else {
            trilinear_laplacian<float>(B, (const float *)B.u, pos, lu);
        }
        if (live) {
            double r[3], D[3];
            for (int d = 0; d < 3; ++d) {
                double rd = pos[d] - Xs[d * np + p];
                rd -= B.L[d] * rint(rd / B.L[d]);
                r[d] = rd;
                D[d] = (double)Ds[d * np + p];
            }
            self_laplacian64(r, D, B.s2s, B.pref, ls);
        }
        for (int d = 0; d < 3; ++d) {
            up[d] += B.fax * lu[d];
            vs[d] += B.fax * ls[d];
        }
    }
}

// FAX: some box of the plan has a Faxen term; HEUN: some box uses the Heun
// integrator (second stage at x* = x^n + dt v^n).  Their extra work doubles the
// registers, so plans without them run the lean instance.
// Laplacian and gradient of u~ = u - v_self at pos for the added-mass terms:
// interpolated nodal stencils of the carrier (computed here unless pre, when
// the caller passes them in lap and grad) minus the closed forms of the
// self-disturbance of the last injection (FP64).
__device__ __forceinline__ void am_terms(const DevBox &B, int64_t p, int64_t n, int M, int selfc,
                                         const double pos[3], double lap[3], double grad[9],
                                         bool pre) {
    if (!pre) trilinear_stencils<float, true, true>(B, (const float *)B.u, pos, lap, grad);
    if (selfc && n >= M + 1) {
        const int64_t np = B.np;
        const int64_t ss = (n - 1 - M) % (M + 1);
        const double *Xs = B.ring_x + ss * 3 * np;
        const float *Ds = (const float *)B.ring_d + ss * 3 * np;
        double r[3], D[3], ls[3], gs[9];
        for (int d = 0; d < 3; ++d) {
            double rd = pos[d] - Xs[d * np + p];
            rd -= B.L[d] * rint(rd / B.L[d]);
            r[d] = rd;
            D[d] = (double)Ds[d * np + p];
        }
        self_laplacian64(r, D, B.s2s, B.pref, ls);
        self_gradient64(r, D, B.s2s, B.pref, gs);
        for (int d = 0; d < 3; ++d) lap[d] -= ls[d];
        for (int q = 0; q < 9; ++q) grad[q] -= gs[q];
    }
}

// AM: the added-mass terms are on for some box (explicit Euler only); boxes
// without them take the plain Euler step.
template <bool FAX, bool HEUN, bool AM>
__global__ void __launch_bounds__(kBlock) k_update(const DevBox *__restrict__ Bs, int nbox,
                                                   const int64_t *__restrict__ stepp, int M,
                                                   double dt, int selfc,
                                                   const double4 *__restrict__ upc,
                                                   const double4 *__restrict__ aux, int64_t npt) {
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int64_t p = (int64_t)(blockIdx.x - B.blk_p) * kBlock + threadIdx.x;
    if (p >= B.np) return;
    const int64_t n = *stepp;
    const int64_t np = B.np;
    double xp[3] = {B.x[p], B.x[np + p], B.x[2 * np + p]};
    double up[3];
    // grid terms gathered by k_gather_sorted (in particle order) once records exist;
    // the first M steps (no records yet) interpolate in place
    const bool rec = n >= M;
    const int64_t sr = B.poff + p;
    if (rec) {
        const double4 g = upc[sr];
        up[0] = g.x;
        up[1] = g.y;
        up[2] = g.z;
    } else {
        trilinear<float>(B, (const float *)B.u, xp, up);
    }
    const bool lpre = (FAX || AM) && rec && (B.fax != 0.0 || B.am_mf != 0.0 || B.bs_k != 0.0);
    double lu[3] = {0.0, 0.0, 0.0};
    if (lpre) {
        const double4 l = aux[sr];
        lu[0] = l.x;
        lu[1] = l.y;
        lu[2] = l.z;
    }
    const int64_t sw = n % (M + 1);
    if (AM && (B.am_mf != 0.0 || B.bs_k != 0.0)) {
        double vs[3], ut[3], lap[3], grad[9];
        self_terms<false>(B, p, n, M, selfc, xp, up, vs, lu, false);
        for (int d = 0; d < 3; ++d) ut[d] = up[d] - vs[d];
        if (rec) {
            // the gather wrote the gradient only for boxes with added mass, the
            // only ones that use it
            for (int d = 0; d < 3; ++d) lap[d] = lu[d];
            for (int j = 0; j < 3; ++j) {
                const double4 g = B.am_mf != 0.0 ? aux[(1 + j) * npt + sr]
                                                 : make_double4(0.0, 0.0, 0.0, 0.0);
                grad[j] = g.x;
                grad[3 + j] = g.y;
                grad[6 + j] = g.z;
            }
        }
        am_terms(B, p, n, M, selfc, xp, lap, grad, rec);
        update_particle_mem(B, p, dt, xp, ut, lap, grad, *B.am_valid, *B.bs_valid,
                            B.ring_x + sw * 3 * np, nullptr, (float *)B.ring_d + sw * 3 * np);
        return;
    }
    double vs[3];
    self_terms<FAX>(B, p, n, M, selfc, xp, up, vs, lu, lpre);
    double up2[3] = {0.0, 0.0, 0.0}, vs2[3] = {0.0, 0.0, 0.0};
    if (HEUN && B.integ == 2) {
        const double xs[3] = {xp[0] + dt * B.v[p], xp[1] + dt * B.v[np + p],
                              xp[2] + dt * B.v[2 * np + p]};
        double l2[3] = {0.0, 0.0, 0.0};
        if (rec) {
            const double4 g = aux[4 * npt + sr];
            up2[0] = g.x;
            up2[1] = g.y;
            up2[2] = g.z;
            if (lpre) {
                const double4 l = aux[5 * npt + sr];
                l2[0] = l.x;
                l2[1] = l.y;
                l2[2] = l.z;
            }
        } else {
            trilinear<float>(B, (const float *)B.u, xs, up2);
        }
        self_terms<FAX>(B, p, n, M, selfc, xs, up2, vs2, l2, lpre);
    }
    update_particle(B, p, dt, xp, up, vs, up2, vs2, B.ring_x + sw * 3 * np, nullptr,
                    (float *)B.ring_d + sw * 3 * np);
}

__global__ void __launch_bounds__(kBlock) k_gather(const DevBox *__restrict__ Bs, int nbox,
                                                   double *__restrict__ out, int f64) {
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int64_t p = (int64_t)(blockIdx.x - B.blk_p) * kBlock + threadIdx.x;
    if (p >= B.np) return;
    const int64_t np = B.np;
    double xp[3] = {B.x[p], B.x[np + p], B.x[2 * np + p]};
    double up[3];
    if (f64)
        trilinear<double>(B, (const double *)B.u, xp, up);
    else
        trilinear<float>(B, (const float *)B.u, xp, up);
    double *o = out + 3 * B.poff;
    o[p] = up[0];
    o[np + p] = up[1];
    o[2 * np + p] = up[2];
}

// ------------------------------------------------------------- erpp_bin ----
// Exact cell binning of any position array of one box; the geometry comes by
// value, the histogram and the ranks through pointers (plan scratch, or the
// static scratch of the allocation-free variant).
__global__ void __launch_bounds__(kBlock) k_bin_pos_count(BinGeom G,
                                                          const double *__restrict__ pos,
                                                          int32_t *__restrict__ key,
                                                          int32_t *__restrict__ count,
                                                          int32_t *__restrict__ rank) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= G.np) return;
    const int64_t np = G.np;
    int b[3];
    double ph;
    for (int d = 0; d < 3; ++d) cell_of(pos[d * np + p], G.L[d], G.dx[d], G.n[d], b[d], ph);
    const int64_t k = ((int64_t)b[2] * G.n[1] + b[1]) * G.n[0] + b[0];
    key[p] = (int32_t)k;
    rank[p] = atomicAdd(&count[k], 1);
}

__global__ void __launch_bounds__(kBlock) k_bin_pos_place(BinGeom G,
                                                          const int32_t *__restrict__ key,
                                                          const int32_t *__restrict__ start,
                                                          const int32_t *__restrict__ rank,
                                                          int32_t *__restrict__ perm) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= G.np) return;
    perm[start[key[p]] + rank[p]] = (int32_t)p;
}

// words[0..n) = 0 (a kernel rather than a memset node, so that a captured graph
// replays it faithfully)
__global__ void __launch_bounds__(kBlock) k_fill_zero(int32_t *__restrict__ words, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) words[i] = 0;
}

}  // namespace

hipError_t scan_counts(int32_t *count, int64_t n, int32_t *start, int32_t *part, int64_t *stepp,
                       hipStream_t st) {
    const int64_t nchunk = (n + kScanChunk - 1) / kScanChunk;
    if (nchunk == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nchunk), dim3(256), 0, st, count, n, part);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nchunk), dim3(256), 0, st, count, n, part,
                       nchunk, start, stepp);
    return hipGetLastError();
}

hipError_t fast_prepare_bound_lds(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_pencil_scale,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// The scatter instance of a plan: pencil depth TZ (rounded up to a power of
// two), workgroup size and rows per work item.
using ScatterFn = void (*)(const DevBox *, int, const int64_t *, int, const int32_t *,
                           const float4 *, const float *, int64_t, int64_t, int32_t *, int, int);

template <int NT, int KB, bool RES>
ScatterFn scatter_fn_tz(int tz) {
    return tz <= 1   ? k_scatter<1, NT, KB, RES>
         : tz <= 2 ? k_scatter<2, NT, KB, RES>
         : tz <= 4 ? k_scatter<4, NT, KB, RES>
                   : k_scatter<8, NT, KB, RES>;
}

template <int NT, bool RES>
ScatterFn scatter_fn_nt(int tz, int band) {
    static_assert(kMinBand == 2 && kMaxBand == 4, "instances below cover kMinBand..kMaxBand");
    return band <= 2 ? scatter_fn_tz<NT, 2, RES>(tz)
         : band == 3 ? scatter_fn_tz<NT, 3, RES>(tz)
                     : scatter_fn_tz<NT, 4, RES>(tz);
}

ScatterFn scatter_fn(int tz, bool big, int band, bool res) {
    if (res) return big ? scatter_fn_nt<1024, true>(tz, band) : scatter_fn_nt<512, true>(tz, band);
    return big ? scatter_fn_nt<1024, false>(tz, band) : scatter_fn_nt<512, false>(tz, band);
}

hipError_t fast_prepare_lds(size_t bytes) {
    for (int res = 0; res < 2; ++res)
        for (int big = 0; big < 2; ++big)
            for (int tz = 1; tz <= 8; tz *= 2)
                for (int band = kMinBand; band <= kMaxBand; ++band) {
                    hipError_t e = hipFuncSetAttribute(
                        (const void *)scatter_fn(tz, big != 0, band, res != 0),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                    if (e != hipSuccess) return e;
                }
    return hipSuccess;
}

hipError_t fast_stage(erpp_plan *P, int k, hipStream_t st) {
    switch (k) {
        case 0:
            if (P->np_total > 0)
                hipLaunchKernelGGL(k_bin_count, dim3((unsigned)P->pblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step, P->M, P->s.count, P->s.rank);
            break;
        case 1:
            return scan_counts(P->s.count, P->nkey_total, P->s.start, P->s.part,
                               P->s.step, st);
        case 2:
            if (P->np_total > 0)
                hipLaunchKernelGGL(k_eval, dim3((unsigned)P->pblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step + 1, P->M, P->s.start, P->s.rank,
                                   P->s.rec, P->s.xs, P->s.vrec);
            break;
        case 3:
            {
                const bool big = P->tile[0] == 1024;
                const ScatterFn rfn = scatter_fn(P->tile[2], big, P->band, true);
                hipLaunchKernelGGL(k_block_sums, dim3((unsigned)P->bblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step + 1, P->M, P->s.start, P->s.rec,
                                   P->s.bsum);
                const int64_t pgrid = (P->tblocks + kXcds - 1) / kXcds * kXcds;
                hipLaunchKernelGGL(k_pencil_scale, dim3((unsigned)pgrid), dim3(kBlock),
                                   P->bound_lds, st, P->dbox, P->nbox, P->s.step + 1, P->M,
                                   P->s.bsum, P->s.pscale, P->tblocks, P->s.pctr);
                // one workgroup per pencil, or, when the pencils outnumber the
                // workgroups the compute units hold at once more than kPersist
                // times, that many resident workgroups taking pencils in turn (a
                // multiple of the XCD count): the per-pencil prologue, clearing and
                // launch then repeat within a workgroup instead of across launches
                if (P->sgrid_fn != (const void *)rfn || P->sgrid_lds != P->lds_bytes) {
                    int dev = 0, ncu = 0, per = 0;
                    hipError_t e = hipGetDevice(&dev);
                    if (e == hipSuccess)
                        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
                    if (e == hipSuccess)
                        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &per, (const void *)rfn, big ? 1024 : 512, P->lds_bytes);
                    if (e != hipSuccess) return e;
                    P->sgrid = (int64_t)std::max(ncu, 1) * std::max(per, 1);
                    P->sgrid_fn = (const void *)rfn;
                    P->sgrid_lds = P->lds_bytes;
                }
                const int64_t res = std::max<int64_t>(kXcds, P->sgrid / kXcds * kXcds);
                const bool resident = pgrid > kPersist * res;
                const ScatterFn fn = resident ? rfn : scatter_fn(P->tile[2], big, P->band, false);
                const int64_t sgrid = resident ? res : pgrid;
                hipLaunchKernelGGL(fn, dim3((unsigned)sgrid), dim3(big ? 1024 : 512),
                                   P->lds_bytes, st, P->dbox, P->nbox, P->s.step + 1, P->M,
                                   P->s.start, P->s.rec, P->s.pscale, P->tblocks,
                                   P->np_total, P->s.pctr, (int)(pgrid / kXcds),
                                   (int)(P->lds_bytes / 4));
            }
            break;
        case 4:
            if (P->np_total > 0) {
                const int64_t grid = (P->pblocks + kXcds - 1) / kXcds * kXcds;
                bool fax = false, heun = false, am = false;
                for (const auto &B : P->hbox) {
                    fax = fax || B.fax != 0.0;
                    heun = heun || B.integ == 2;
                    am = am || B.am_mf != 0.0 || B.bs_k != 0.0;
                }
                const bool lap = fax || am;
                // the added-mass and Basset terms run with explicit Euler only (checked
                // by the setters)
                auto gat = am ? k_gather_sorted<true, true, false>
                         : lap ? (heun ? k_gather_sorted<true, false, true>
                                       : k_gather_sorted<true, false, false>)
                               : (heun ? k_gather_sorted<false, false, true>
                                       : k_gather_sorted<false, false, false>);
                hipLaunchKernelGGL(gat, dim3((unsigned)grid), dim3(kBlock), 0, st, P->dbox,
                                   P->nbox, P->pblocks, P->s.step + 1, P->M, P->s.xs, P->s.up,
                                   P->s.aux, P->np_total, P->s.vrec, P->dt);
                auto upd = am ? (fax ? k_update<true, false, true> : k_update<false, false, true>)
                         : fax ? (heun ? k_update<true, true, false> : k_update<true, false, false>)
                               : (heun ? k_update<false, true, false>
                                       : k_update<false, false, false>);
                hipLaunchKernelGGL(upd,
                                   dim3((unsigned)P->pblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step + 1, P->M, P->dt, P->self_correction,
                                   P->s.up, P->s.aux, P->np_total);
                if (am) return mark_memory_terms(P, st);
            }
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t fast_scatter_stages(erpp_plan *P, hipStream_t st) {
    for (int k = 0; k < 4; ++k) {
        hipError_t e = fast_stage(P, k, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fast_update_stage(erpp_plan *P, hipStream_t st) { return fast_stage(P, 4, st); }

hipError_t fast_gather(erpp_plan *P, double *u_p, hipStream_t st) {
    if (P->np_total > 0) {
        hipLaunchKernelGGL(k_gather, dim3((unsigned)P->pblocks), dim3(kBlock), 0, st, P->dbox,
                           P->nbox, u_p, (int)(P->prec == ERPP_F64_PLAIN));
    }
    return hipGetLastError();
}

hipError_t bin_positions(const BinGeom &G, const double *pos, int32_t *key, int32_t *perm,
                         int32_t *bin_start, int32_t *count, int32_t *rank, int32_t *part,
                         bool clear, hipStream_t st) {
    const int64_t nc = (int64_t)G.n[0] * G.n[1] * G.n[2];
    const unsigned blocks = (unsigned)((G.np + kBlock - 1) / kBlock);
    if (clear)
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((nc + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, count, nc);
    if (G.np > 0)
        hipLaunchKernelGGL(k_bin_pos_count, dim3(blocks), dim3(kBlock), 0, st, G, pos, key, count,
                           rank);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_counts(count, nc, bin_start, part, nullptr, st);
    if (e != hipSuccess) return e;
    if (G.np > 0)
        hipLaunchKernelGGL(k_bin_pos_place, dim3(blocks), dim3(kBlock), 0, st, G, key, bin_start,
                           rank, perm);
    return hipGetLastError();
}

hipError_t fast_bin_positions(erpp_plan *P, int ibox, const double *pos, int32_t *key,
                              int32_t *perm, int32_t *bin_start, hipStream_t st) {
    const DevBox &H = P->hbox[ibox];
    BinGeom G;
    for (int d = 0; d < 3; ++d) {
        G.n[d] = H.n[d];
        G.L[d] = H.L[d];
        G.dx[d] = H.dx[d];
    }
    G.np = H.np;
    return bin_positions(G, pos, key, perm, bin_start, P->s.count + H.cell_off,
                         P->s.rank + H.poff, P->s.part, false, st);
}

}  // namespace erpp
