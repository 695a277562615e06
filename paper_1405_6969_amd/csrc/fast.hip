// fast.hip -- ERPP_F32_FAST path of the coupling step for gfx950.
//
// Per step n (all boxes of a plan in one launch per stage):
//   k_bin_count   tile histogram of the delayed positions X^{n-M}; a particle's
//                 atomic ticket is its rank inside its tile
//   k_scan        exclusive scan of the histogram (and reset of it)
//   k_eval        per particle: FP64 cell/offset of X^{n-M}, FP32 Gaussian
//                 normalisation over the 3-sigma sphere, record
//                 {offsets, amplitude} written at its tile-sorted slot
//   k_scatter     one workgroup per tile: accumulate the stencils of every
//                 particle that reaches the tile into an LDS tile, then store
//                 the tile (each node written once, no global atomics)
//   k_update      per particle: trilinear carrier, closed-form self term,
//                 Stokes drag, history write, explicit Euler, wrap
#include <hip/hip_runtime.h>

#include "erpp_device.hpp"
#include "erpp_internal.hpp"

namespace erpp {

namespace {

__device__ __forceinline__ int tile_of(const DevBox &B, int b0, int b1, int b2) {
    return ((b2 / B.T[2]) * B.ntile[1] + (b1 / B.T[1])) * B.ntile[0] + (b0 / B.T[0]);
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
    const int t = tile_of(B, b[0], b[1], b[2]);
    rank[B.poff + p] = atomicAdd(&count[B.bin_off + t], 1);
}

// Exclusive scan of count[0..nb) into start[0..nb], count (and the per-bin
// amplitude bound, when given) reset to zero.  One workgroup of 1024 threads,
// each owning a contiguous chunk.
__global__ void __launch_bounds__(1024) k_scan(int32_t *__restrict__ count,
                                               int32_t *__restrict__ start, int64_t nb,
                                               uint32_t *__restrict__ binmax) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (nb + 1023) / 1024;
    const int64_t a = tid * chunk;
    const int64_t e = (a + chunk < nb) ? a + chunk : nb;
    int32_t s = 0;
    for (int64_t i = a; i < e; ++i) s += count[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = (tid >= off) ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - s;
    for (int64_t i = a; i < e; ++i) {
        int32_t c = count[i];
        start[i] = run;
        run += c;
        count[i] = 0;
        if (binmax) binmax[i] = 0u;
    }
    if (tid == 1023) start[nb] = part[1023];
}

constexpr int kMaxOff = 16;   // max stencil offsets per dimension (mhi - mlo + 1)

__global__ void __launch_bounds__(kBlock) k_eval(const DevBox *__restrict__ Bs, int nbox,
                                                 const int64_t *__restrict__ stepp, int M,
                                                 const int32_t *__restrict__ start,
                                                 const int32_t *__restrict__ rank,
                                                 float4 *__restrict__ rec,
                                                 uint32_t *__restrict__ binmax) {
    __shared__ float sP[kMaxOff + 1][kBlock];   // prefix sums of the x factors
    __shared__ float sGy[kMaxOff][kBlock];
    __shared__ float sTy[kMaxOff][kBlock];
    const int64_t n = *stepp;
    if (n < M) return;
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)(blockIdx.x - B.blk_p) * kBlock + tid;
    if (p >= B.np) return;
    const int64_t np = B.np;
    const int64_t slot = (n - M) % (M + 1);
    const double *X = B.ring_x + slot * 3 * np;
    const float *Dd = (const float *)B.ring_d + slot * 3 * np;
    int b[3];
    double ph[3];
    for (int d = 0; d < 3; ++d) cell_of(X[d * np + p], B.L[d], B.dx[d], B.n[d], b[d], ph[d]);
    const float phx = (float)ph[0], phy = (float)ph[1], phz = (float)ph[2];
    const int mlo0 = B.mlo[0], mhi0 = B.mhi[0];
    const int mlo1 = B.mlo[1], mhi1 = B.mhi[1];
    // x factors and their prefix sums, y factors
    sP[0][tid] = 0.0f;
    {
        float acc = 0.0f;
        for (int m = mlo0; m <= mhi0; ++m) {
            acc += g1(m, phx, B.dxf[0], B.cexp);
            sP[m - mlo0 + 1][tid] = acc;
        }
    }
    for (int m = mlo1; m <= mhi1; ++m) {
        sGy[m - mlo1][tid] = g1(m, phy, B.dxf[1], B.cexp);
        sTy[m - mlo1][tid] = d1(m, phy, B.dxf[1]);
    }
    const float cut = B.R2f + B.guard;
    const int pid = (int)p;
    float Z = 0.0f;
    for (int mz = B.mlo[2]; mz <= B.mhi[2]; ++mz) {
        const float tz = d1(mz, phz, B.dxf[2]);
        const float tz2 = tz * tz;
        if (tz2 > cut) continue;
        const float gz = g1(mz, phz, B.dxf[2], B.cexp);
        for (int my = mlo1; my <= mhi1; ++my) {
            const float ty = sTy[my - mlo1][tid];
            const float ryz = fmaf(ty, ty, tz2);
            if (ryz > cut) continue;
            int lo, hi;
            row_range(phx, ryz, B, &B, slot, pid, my, mz, lo, hi);
            if (lo > hi) continue;
            const float gyz = sGy[my - mlo1][tid] * gz;
            const float rs = sP[hi - mlo0 + 1][tid] - sP[lo - mlo0][tid];
            Z = fmaf(gyz, rs, Z);
        }
    }
    const float Zv = Z * (float)B.dV;
    const float inv = -B.rhof_inv / Zv;
    const float ax = Dd[p] * inv, ay = Dd[np + p] * inv, az = Dd[2 * np + p] * inv;
    const int t = tile_of(B, b[0], b[1], b[2]);
    const int64_t slotr = (int64_t)start[B.bin_off + t] + rank[B.poff + p];
    const uint32_t ijk = (uint32_t)b[0] | ((uint32_t)b[1] << 11) | ((uint32_t)b[2] << 22);
    rec[2 * slotr] = make_float4(phx, phy, phz, __uint_as_float(ijk));
    rec[2 * slotr + 1] = make_float4(ax, ay, az, __int_as_float((int)p));
    // per-bin bound of the largest amplitude (non-negative floats order as uints)
    const float amax = fmaxf(fabsf(ax), fmaxf(fabsf(ay), fabsf(az)));
    atomicMax(&binmax[B.bin_off + t], __float_as_uint(amax));
}

constexpr int kMaxTileList = 24;

// |v| <= 2^30 by construction of the scale: round to int32, sign-extend to the
// 64-bit two's-complement word added into the LDS accumulator.
__device__ __forceinline__ unsigned long long to_fixed(float v) {
    return (unsigned long long)(long long)__float2int_rn(v);
}

// Tiles of one dimension holding base cells in [a, c] (unwrapped, c - a < N),
// written to list[0..*cnt) without duplicates.
__device__ void tiles_for_range(int a, int c, int N, int T, int *list, int *cnt) {
    int n = 0;
    auto add_interval = [&](int u, int v) {
        for (int t = u / T; t <= v / T; ++t) {
            bool dup = false;
            for (int q = 0; q < n; ++q) dup |= (list[q] == t);
            if (!dup && n < kMaxTileList) list[n++] = t;
        }
    };
    int aw = a % N;
    if (aw < 0) aw += N;
    const int len = c - a;
    if (aw + len < N) {
        add_interval(aw, aw + len);
    } else {
        add_interval(aw, N - 1);
        add_interval(0, aw + len - N);
    }
    *cnt = n;
}

// A particle whose stencil reaches the tile, as staged in LDS.
struct Visit {
    float phx, phy, phz;   // FP32 offsets of the delayed position in its cell
    float ax, ay, az;      // amplitude / Z, already multiplied by the tile scale
    int dl;                // base cell relative to the tile origin, 3 x 10 bits (+512)
    int pid;               // particle index (FP64 fallback of the sphere test)
};

constexpr int kVisCap = 640;    // visits staged per round (2 workgroups per CU fit in LDS)
constexpr int kVisBuckets = 24; // work classes (clipped stencil-box volume, ratio sqrt 2)

__device__ __forceinline__ int work_bucket(int vol) {
    // floor(2 log2(vol)) from the exponent and the top mantissa bit
    const float fv = (float)vol;
    const uint32_t u = __float_as_uint(fv);
    const int e = (int)((u >> 23) & 255u) - 127;
    const int half = (u >> 22) & 1u;    // mantissa >= 1.5 ~ sqrt(2)
    const int b = 2 * e + half;
    return b < 0 ? 0 : (b >= kVisBuckets ? kVisBuckets - 1 : b);
}

// Contribution to the integer tile: round to the nearest int32 (|v| < 2^30 by
// the choice of scale; the error of one term is at most half a unit).
__device__ __forceinline__ uint32_t fixed32(float v) { return (uint32_t)__float2int_rn(v); }

__device__ __forceinline__ int pack_dl(int a, int b, int c) {
    return (a + 512) | ((b + 512) << 10) | ((c + 512) << 20);
}

// One workgroup per tile of nodes (owner computes: every node of the tile is
// written once, by this workgroup; no global atomics).  Every particle whose
// stencil reaches the tile -- found in the bins of the tile and its neighbours --
// is a "visit": it adds the part of its stencil inside the tile to an LDS copy
// of the tile.
//
// Accumulation is exact integer arithmetic: each contribution a*w is rounded to
// an int32 with the per-tile scale 2^30 / A, where A = sum over the tile's
// visits of max_c |amplitude| bounds |f| at every node of the tile, and added
// with ds_add_u32 (the FP32 LDS atomic runs ~40x slower on gfx950).  Integer
// additions commute, so the forcing does not depend on the order of the adds.
//
// Work split: one lane per visit.  A lane walks its clipped stencil plane by
// plane (z), over the y-range of each plane's disk, and along each row (x) over
// the exact in-sphere range; along a row the Gaussian weight advances by a
// multiplicative recurrence (two multiplies per node).
__global__ void __launch_bounds__(kScatterBlock) k_scatter(const DevBox *__restrict__ Bs,
                                                           int nbox,
                                                           const int64_t *__restrict__ stepp,
                                                           int M,
                                                           const int32_t *__restrict__ start,
                                                           const float4 *__restrict__ rec) {
    extern __shared__ int32_t acc[];
    __shared__ int s_list[3][kMaxTileList];
    __shared__ int s_cnt[3];
    __shared__ float s_part[kScatterBlock / 64];
    __shared__ float s_scale;
    __shared__ int s_nvis;
    __shared__ int s_bcnt[kVisBuckets];
    __shared__ int s_boff[kVisBuckets];
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_t; });
    const DevBox &B = Bs[bi];
    const int t = (int)(blockIdx.x - B.blk_t);
    const int tx = t % B.ntile[0];
    const int ty = (t / B.ntile[0]) % B.ntile[1];
    const int tz = t / (B.ntile[0] * B.ntile[1]);
    const int o0 = tx * B.T[0], o1 = ty * B.T[1], o2 = tz * B.T[2];
    const int e0 = min(B.T[0], B.n[0] - o0);
    const int e1 = min(B.T[1], B.n[1] - o1);
    const int e2 = min(B.T[2], B.n[2] - o2);
    const int PX = B.T[0] + 1;
    const int PL = B.T[1] * PX;
    const int CS = B.T[2] * PL;        // nodes of the padded tile; component c of node a at 3a+c
    Visit *vis = (Visit *)(acc + 3 * CS + ((3 * CS) & 1));   // 8-byte aligned after the tile
    int *vkey = (int *)(vis + kVisCap);                         // bucket << 16 | rank in bucket
    int *vperm = vkey + kVisCap;                                // visits in work order
    const int tid = threadIdx.x;
    for (int i = tid; i < 3 * CS; i += kScatterBlock) acc[i] = 0;
    const int64_t n = *stepp;
    const bool live = n >= M;
    // base cells whose stencil reaches the tile, per dimension
    const int lo0 = o0 - B.mhi[0], hi0 = o0 + e0 - 1 - B.mlo[0];
    const int lo1 = o1 - B.mhi[1], hi1 = o1 + e1 - 1 - B.mlo[1];
    const int lo2 = o2 - B.mhi[2], hi2 = o2 + e2 - 1 - B.mlo[2];
    if (tid < kVisBuckets) s_bcnt[tid] = 0;
    if (tid == 0) {
        tiles_for_range(lo0, hi0, B.n[0], B.T[0], s_list[0], &s_cnt[0]);
        tiles_for_range(lo1, hi1, B.n[1], B.T[1], s_list[1], &s_cnt[1]);
        tiles_for_range(lo2, hi2, B.n[2], B.T[2], s_list[2], &s_cnt[2]);
        s_nvis = 0;
    }
    __syncthreads();
    const int nlx = s_cnt[0], nly = s_cnt[1], nlz = s_cnt[2];
    const int ncb = live ? nlx * nly * nlz : 0;
    // unwrapped base of record r relative to the tile range; false if it misses
    auto locate = [&](const float4 &qa, int &d0, int &d1, int &d2) -> bool {
        const uint32_t ijk = __float_as_uint(qa.w);
        int bu0 = (int)(ijk & 2047u), bu1 = (int)((ijk >> 11) & 2047u), bu2 = (int)(ijk >> 22);
        if (bu0 > hi0) bu0 -= B.n[0];
        if (bu0 < lo0) bu0 += B.n[0];
        if (bu1 > hi1) bu1 -= B.n[1];
        if (bu1 < lo1) bu1 += B.n[1];
        if (bu2 > hi2) bu2 -= B.n[2];
        if (bu2 < lo2) bu2 += B.n[2];
        d0 = bu0 - o0;
        d1 = bu1 - o1;
        d2 = bu2 - o2;
        return bu0 >= lo0 && bu0 <= hi0 && bu1 >= lo1 && bu1 <= hi1 && bu2 >= lo2 && bu2 <= hi2;
    };
    auto bin_of = [&](int k) -> int64_t {
        const int ix = k % nlx, iy = (k / nlx) % nly, iz = k / (nlx * nly);
        return B.bin_off + ((int64_t)s_list[2][iz] * B.ntile[1] + s_list[1][iy]) * B.ntile[0] +
               s_list[0][ix];
    };
    // ---- pass A: amplitude bound of the tile (fixed-order reduction)
    float part = 0.0f;
    for (int k = 0; k < ncb; ++k) {
        const int64_t gb = bin_of(k);
        const int rs = start[gb], re = start[gb + 1];
        for (int r = rs + tid; r < re; r += kScatterBlock) {
            const float4 qa = rec[2 * (int64_t)r];
            int d0, d1, d2;
            if (locate(qa, d0, d1, d2)) {
                const float4 qb = rec[2 * (int64_t)r + 1];
                part += fmaxf(fabsf(qb.x), fmaxf(fabsf(qb.y), fabsf(qb.z)));
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if ((tid & 63) == 0) s_part[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
        float bound = 0.0f;
        for (int w = 0; w < kScatterBlock / 64; ++w) bound += s_part[w];
        s_scale = (bound > 0.0f && bound < 3.0e38f) ? 1073741824.0f / bound : 1.0f;
    }
    __syncthreads();
    const float scale = s_scale;
    if (ncb > 0) {
        const int64_t slot = (n - M) % (M + 1);
        const float cut = B.R2f + B.guard;
        const float hx = B.dxf[0];
        const float c = B.cexp;
        const float qx = exp2f(-2.0f * c * hx * hx);
        // ---- pass B: stage visits in rounds, one lane per visit.  The cursor
        // (k = bin, r = record) is uniform across the block; s_nvis is read by
        // every thread before any thread appends (barrier in between).
        int k = 0;
        int64_t gb0 = bin_of(0);
        int r = start[gb0], re = start[gb0 + 1];
        while (true) {
            while (k < ncb) {
                if (r >= re) {
                    if (++k >= ncb) break;
                    const int64_t gb = bin_of(k);
                    r = start[gb];
                    re = start[gb + 1];
                    continue;
                }
                const int nv0 = s_nvis;
                __syncthreads();
                // a chunk of c records adds at most c visits
                const int room = kVisCap - nv0;
                if (room < 64) break;
                const int chunk = min(min(re - r, kScatterBlock), room);
                if (tid < chunk) {
                    const int rr = r + tid;
                    const float4 qa = rec[2 * (int64_t)rr];
                    int d0, d1, d2;
                    if (locate(qa, d0, d1, d2)) {
                        const float4 qb = rec[2 * (int64_t)rr + 1];
                        const int slotv = atomicAdd(&s_nvis, 1);
                        Visit v;
                        v.phx = qa.x;
                        v.phy = qa.y;
                        v.phz = qa.z;
                        v.ax = qb.x * scale;
                        v.ay = qb.y * scale;
                        v.az = qb.z * scale;
                        v.dl = pack_dl(d0, d1, d2);
                        v.pid = __float_as_int(qb.w);
                        vis[slotv] = v;
                        const int vol = (min(B.mhi[0], e0 - 1 - d0) - max(B.mlo[0], -d0) + 1) *
                                        (min(B.mhi[1], e1 - 1 - d1) - max(B.mlo[1], -d1) + 1) *
                                        (min(B.mhi[2], e2 - 1 - d2) - max(B.mlo[2], -d2) + 1);
                        const int bk = work_bucket(vol);
                        vkey[slotv] = (bk << 16) | atomicAdd(&s_bcnt[bk], 1);
                    }
                }
                r += chunk;
                __syncthreads();
            }
            __syncthreads();
            const int nv = s_nvis;
            if (nv == 0) break;
            // order the staged visits by work, largest first, so that the 64 lanes of
            // a wave walk stencils of similar size
            if (tid == 0) {
                int run = 0;
                for (int b = kVisBuckets - 1; b >= 0; --b) {
                    s_boff[b] = run;
                    run += s_bcnt[b];
                }
            }
            __syncthreads();
            for (int vi = tid; vi < nv; vi += kScatterBlock) {
                const int key = vkey[vi];
                vperm[s_boff[key >> 16] + (key & 0xffff)] = vi;
            }
            __syncthreads();
            if (tid < kVisBuckets) s_bcnt[tid] = 0;
            for (int vs = tid; vs < nv; vs += kScatterBlock) {
                const Visit v = vis[vperm[vs]];
                const int dl0 = (v.dl & 1023) - 512, dl1 = ((v.dl >> 10) & 1023) - 512,
                          dl2 = ((v.dl >> 20) & 1023) - 512;
                const int c0lo = max(B.mlo[0], -dl0), c0hi = min(B.mhi[0], e0 - 1 - dl0);
                const int c1lo = max(B.mlo[1], -dl1), c1hi = min(B.mhi[1], e1 - 1 - dl1);
                const int c2lo = max(B.mlo[2], -dl2), c2hi = min(B.mhi[2], e2 - 1 - dl2);
                for (int mz = c2lo; mz <= c2hi; ++mz) {
                    const float tzv = d1(mz, v.phz, B.dxf[2]);
                    const float tz2 = tzv * tzv;
                    if (tz2 > cut) continue;
                    const float gz = exp2f(-tz2 * c);
                    // y-range of this plane's disk (superset; rows are settled exactly below)
                    const float sy = sqrtf(fmaxf(cut - tz2, 0.0f)) / B.dxf[1];
                    const int ylo = max(c1lo, (int)ceilf(v.phy - sy) - 1);
                    const int yhi = min(c1hi, (int)floorf(v.phy + sy) + 1);
                    for (int my = ylo; my <= yhi; ++my) {
                        const float tyv = d1(my, v.phy, B.dxf[1]);
                        const float ryz = fmaf(tyv, tyv, tz2);
                        if (ryz > cut) continue;
                        int lo, hi;
                        row_range(v.phx, ryz, B, &B, slot, v.pid, my, mz, lo, hi);
                        lo = max(lo, c0lo);
                        hi = min(hi, c0hi);
                        if (lo > hi) continue;
                        const float gyz = exp2f(-(tyv * tyv) * c) * gz;
                        const float t0 = ((float)lo - v.phx) * hx;
                        float w = exp2f(-(t0 * t0) * c) * gyz;
                        float rr = exp2f(-c * hx * fmaf(2.0f, t0, hx));
                        uint32_t *ap =
                            (uint32_t *)&acc[3 * ((mz + dl2) * PL + (my + dl1) * PX + dl0 + lo)];
                        for (int m = lo; m <= hi; ++m) {
                            atomicAdd(ap, fixed32(v.ax * w));
                            atomicAdd(ap + 1, fixed32(v.ay * w));
                            atomicAdd(ap + 2, fixed32(v.az * w));
                            w *= rr;
                            rr *= qx;
                            ap += 3;
                        }
                    }
                }
            }
            __syncthreads();
            if (tid == 0) s_nvis = 0;
            __syncthreads();
            if (k >= ncb) break;
        }
    }
    __syncthreads();
    float *f = (float *)B.f;
    const float inv = 1.0f / scale;
    const int64_t Nx = B.n[0], Ny = B.n[1];
    const int64_t ng = Nx * Ny * B.n[2];
    const int cnt = e0 * e1 * e2;
    for (int i = tid; i < cnt; i += kScatterBlock) {
        const int lx = i % e0;
        const int ly = (i / e0) % e1;
        const int lz = i / (e0 * e1);
        const int64_t g = ((int64_t)(o2 + lz) * Ny + (o1 + ly)) * Nx + (o0 + lx);
        const int a = 3 * (lz * PL + ly * PX + lx);
        f[g] = (float)acc[a] * inv;
        f[ng + g] = (float)acc[a + 1] * inv;
        f[2 * ng + g] = (float)acc[a + 2] * inv;
    }
}

__global__ void __launch_bounds__(kBlock) k_update(const DevBox *__restrict__ Bs, int nbox,
                                                   const int64_t *__restrict__ stepp, int M,
                                                   double dt, int selfc) {
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int64_t p = (int64_t)(blockIdx.x - B.blk_p) * kBlock + threadIdx.x;
    if (p >= B.np) return;
    const int64_t n = *stepp;
    const int64_t np = B.np;
    double xp[3] = {B.x[p], B.x[np + p], B.x[2 * np + p]};
    double up[3];
    trilinear<float>(B, (const float *)B.u, xp, up);
    double vs[3] = {0.0, 0.0, 0.0};
    if (selfc && n >= M + 1) {
        const int64_t ss = (n - 1 - M) % (M + 1);
        const double *Xs = B.ring_x + ss * 3 * np;
        const float *Ds = (const float *)B.ring_d + ss * 3 * np;
        float r[3];
        for (int d = 0; d < 3; ++d) {
            double rd = xp[d] - Xs[d * np + p];
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
    const int64_t sw = n % (M + 1);
    update_particle(B, p, dt, xp, up, vs, B.ring_x + sw * 3 * np, nullptr,
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
__global__ void __launch_bounds__(kBlock) k_bin_pos_count(const DevBox *__restrict__ Bs, int ibox,
                                                          const double *__restrict__ pos,
                                                          int32_t *__restrict__ key,
                                                          int32_t *__restrict__ count,
                                                          int32_t *__restrict__ rank) {
    const DevBox &B = Bs[ibox];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= B.np) return;
    const int64_t np = B.np;
    int b[3];
    double ph;
    for (int d = 0; d < 3; ++d) cell_of(pos[d * np + p], B.L[d], B.dx[d], B.n[d], b[d], ph);
    key[p] = (int32_t)(((int64_t)b[2] * B.n[1] + b[1]) * B.n[0] + b[0]);
    rank[B.poff + p] = atomicAdd(&count[B.bin_off + tile_of(B, b[0], b[1], b[2])], 1);
}

__global__ void __launch_bounds__(kBlock) k_bin_pos_place(const DevBox *__restrict__ Bs, int ibox,
                                                          const int32_t *__restrict__ key,
                                                          const int32_t *__restrict__ start,
                                                          const int32_t *__restrict__ rank,
                                                          int32_t *__restrict__ perm) {
    const DevBox &B = Bs[ibox];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= B.np) return;
    const int32_t k = key[p];
    const int b0 = k % B.n[0];
    const int b1 = (k / B.n[0]) % B.n[1];
    const int b2 = k / (B.n[0] * B.n[1]);
    perm[start[tile_of(B, b0, b1, b2)] + rank[B.poff + p]] = (int32_t)p;
}

}  // namespace

hipError_t fast_prepare_lds(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_scatter, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

size_t scatter_lds_bytes(const int32_t tile[3]) {
    const size_t cs = 3 * (size_t)tile[2] * tile[1] * (tile[0] + 1);
    return sizeof(int32_t) * (cs + (cs & 1)) + (sizeof(Visit) + 2 * sizeof(int)) * kVisCap;
}

hipError_t fast_stage(erpp_plan *P, int k, hipStream_t st) {
    switch (k) {
        case 0:
            if (P->np_total > 0)
                hipLaunchKernelGGL(k_bin_count, dim3((unsigned)P->pblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step, P->M, P->s.count, P->s.rank);
            break;
        case 1:
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, P->s.count, P->s.start,
                               P->nbins_total, P->s.binmax);
            break;
        case 2:
            if (P->np_total > 0)
                hipLaunchKernelGGL(k_eval, dim3((unsigned)P->pblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step, P->M, P->s.start, P->s.rank,
                                   P->s.rec, P->s.binmax);
            break;
        case 3:
            hipLaunchKernelGGL(k_scatter, dim3((unsigned)P->tblocks), dim3(kScatterBlock),
                               P->lds_bytes, st, P->dbox, P->nbox, P->s.step, P->M, P->s.start,
                               P->s.rec);
            break;
        case 4:
            if (P->np_total > 0)
                hipLaunchKernelGGL(k_update, dim3((unsigned)P->pblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step, P->M, P->dt, P->self_correction);
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

hipError_t fast_bin_positions(erpp_plan *P, int ibox, const double *pos, int32_t *key,
                              int32_t *perm, int32_t *bin_start, hipStream_t st) {
    const DevBox &H = P->hbox[ibox];
    const int64_t nb = (int64_t)H.ntile[0] * H.ntile[1] * H.ntile[2];
    const unsigned blocks = (unsigned)((H.np + kBlock - 1) / kBlock);
    if (H.np > 0)
        hipLaunchKernelGGL(k_bin_pos_count, dim3(blocks), dim3(kBlock), 0, st, P->dbox, ibox, pos,
                           key, P->s.count, P->s.rank);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, P->s.count + H.bin_off, bin_start, nb,
                       (uint32_t *)nullptr);
    if (H.np > 0)
        hipLaunchKernelGGL(k_bin_pos_place, dim3(blocks), dim3(kBlock), 0, st, P->dbox, ibox, key,
                           bin_start, P->s.rank, perm);
    return hipGetLastError();
}

}  // namespace erpp
