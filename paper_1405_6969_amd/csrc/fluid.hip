// fluid.hip -- periodic unsteady-Stokes step of the disturbance field
// (Sec. 2.3, eq. velo_reg_eq) by the forcing / diffusion / projection
// splitting of App. E, pseudo-spectral with hipFFT.
//
// Grids whose three sizes are powers of two (Nx >= 4) use this file's own
// transforms, five passes over the half spectrum U [3][Nz][Ny][Nx/2+1]:
//   k_fx_r2c     u + dt f (eq. forcing_step) and its real FFT along x
//   k_fy         FFT along y (forward)
//   k_fz_spec    FFT along z, then exp(-nu k^2 dt) (I - k_d k_d^T / k_d^2) / N
//                (exact heat semigroup, eq. diffusion_step; the projection
//                lap(phi) = -div(u*), u = u* + grad(phi)), inverse FFT along z
//   k_fy         inverse FFT along y
//   k_fx_c2r     inverse real FFT along x into u
// Each pass stages its lines in LDS and runs a Stockham transform there (radix 8
// and 4 passes, natural order in and out).  Other
// sizes use hipFFT, four launches:
//   k_fluid_force     u += dt f
//   forward R2C       U = FFT(u), three components batched (may overwrite u)
//   k_fluid_spectral  the same Fourier multiplier
//   inverse C2R       u = IFFT(U)
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "erpp_internal.hpp"

struct erpp_fluid {
    uint64_t id;        // unique per created stepper (graph bookkeeping)
    int32_t n[3];
    double L[3];
    double nu, dt;
    erpp_precision prec;
    int64_t nodes;      // Nx Ny Nz
    int64_t modes;      // Nz Ny (Nx/2+1), per component
    hipfftHandle fwd = 0, inv = 0;
    bool have_fwd = false, have_inv = false;
    void *spec = nullptr;   // [3][Nz][Ny][Nx/2+1] complex
    // own transforms (all sizes powers of two): twiddles e^{-2 pi i j / lt},
    // j = 0 .. lt/2, lt = the largest size
    bool own = false;
    void *tw = nullptr;
    int32_t lt = 0;
    int32_t rs = 0;         // row stride of U in complex values (Nx/2+1 padded to 16)
};

namespace {

constexpr int kFluidBlock = 256;

// u += dt f over `count` values; V values per thread through a vector type when
// both pointers are 16-byte aligned (the host picks V).
template <typename T, int V>
__global__ __launch_bounds__(kFluidBlock) void k_fluid_force(T *__restrict__ u,
                                                             const T *__restrict__ f, T dt,
                                                             int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (V > 1) {
        struct alignas(sizeof(T) * V) vec { T a[V]; };
        const int64_t nvec = count / V;
        vec *uv = reinterpret_cast<vec *>(u);
        const vec *fv = reinterpret_cast<const vec *>(f);
        for (int64_t i = i0; i < nvec; i += stride) {
            vec a = uv[i];
            const vec b = fv[i];
#pragma unroll
            for (int j = 0; j < V; ++j) a.a[j] += dt * b.a[j];
            uv[i] = a;
        }
        for (int64_t i = nvec * V + i0; i < count; i += stride) u[i] += dt * f[i];
    } else {
        for (int64_t i = i0; i < count; i += stride) u[i] += dt * f[i];
    }
}

template <typename T> struct cplx { T re, im; };

// Per Fourier mode of the half spectrum: exact diffusion over dt, projection
// onto fields of zero grid divergence, and the 1/(Nx Ny Nz) of the
// unnormalised inverse transform.  Mode index: x fastest over Nx/2+1, then y,
// then z.  The diffusion uses the full |k|^2; the projection's derivatives use
// k_d, whose component at the Nyquist index of an even N is zero (the grid
// derivative of (-1)^j vanishes at every node), which also makes the result
// independent of the sign of that index.
template <typename T>
__global__ __launch_bounds__(kFluidBlock) void k_fluid_spectral(
    cplx<T> *__restrict__ U, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t modes,
    T kx0, T ky0, T kz0, T nudt, T scale) {
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= modes) return;
    const uint32_t nh = nx / 2 + 1;
    const uint32_t ix = idx % nh;
    const uint32_t r = idx / nh;
    const uint32_t iy = r % ny;
    const uint32_t iz = r / ny;
    const int my = iy <= ny / 2 ? (int)iy : (int)iy - (int)ny;
    const int mz = iz <= nz / 2 ? (int)iz : (int)iz - (int)nz;
    const T kx = kx0 * (T)(int)ix, ky = ky0 * (T)my, kz = kz0 * (T)mz;
    const T k2 = kx * kx + ky * ky + kz * kz;
    const T dkx = (2 * ix == nx) ? (T)0 : kx;
    const T dky = (2 * iy == ny) ? (T)0 : ky;
    const T dkz = (2 * iz == nz) ? (T)0 : kz;
    const T kd2 = dkx * dkx + dky * dky + dkz * dkz;
    cplx<T> a = U[idx], b = U[idx + modes], c = U[idx + 2 * (size_t)modes];
    const T e = exp(-nudt * k2) * scale;
    if (kd2 > (T)0) {
        const T ik2 = (T)1 / kd2;
        // (k_d . U) / k_d^2, real and imaginary parts
        const T pr = (dkx * a.re + dky * b.re + dkz * c.re) * ik2;
        const T pi = (dkx * a.im + dky * b.im + dkz * c.im) * ik2;
        a.re -= dkx * pr; a.im -= dkx * pi;
        b.re -= dky * pr; b.im -= dky * pi;
        c.re -= dkz * pr; c.im -= dkz * pi;
    }
    a.re *= e; a.im *= e;
    b.re *= e; b.im *= e;
    c.re *= e; c.im *= e;
    U[idx] = a;
    U[idx + modes] = b;
    U[idx + 2 * (size_t)modes] = c;
}

// ------------------------------------------------------ own transforms ----

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// ---- Stockham transforms: natural order in and out, radix 8/4 (2 for n = 2),
// each pass reads a thread's butterflies into registers, waits, writes them
// back permuted, waits.  Twiddles e^{-2 pi i m / lt}, m in [0, lt).

template <typename T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a, int sign) {   // a * (sign i)
    return sign < 0 ? cplx<T>{a.im, -a.re} : cplx<T>{-a.im, a.re};
}

template <typename T>
__device__ __forceinline__ void dft2(cplx<T> &a, cplx<T> &b) {
    const cplx<T> t = a;
    a = {t.re + b.re, t.im + b.im};
    b = {t.re - b.re, t.im - b.im};
}

// 4-point DFT in place, w = e^{sign 2 pi i / 4} = sign i
template <typename T>
__device__ __forceinline__ void dft4(cplx<T> *v, int sign) {
    dft2(v[0], v[2]);                       // v0 + v2, v0 - v2
    dft2(v[1], v[3]);                       // v1 + v3, v1 - v3
    v[3] = mul_i(v[3], sign);
    const cplx<T> x0 = {v[0].re + v[1].re, v[0].im + v[1].im};
    const cplx<T> x2 = {v[0].re - v[1].re, v[0].im - v[1].im};
    const cplx<T> x1 = {v[2].re + v[3].re, v[2].im + v[3].im};
    const cplx<T> x3 = {v[2].re - v[3].re, v[2].im - v[3].im};
    v[0] = x0; v[1] = x1; v[2] = x2; v[3] = x3;
}

// 8-point DFT: two 4-point DFTs of the even and odd samples, combined with
// e^{sign 2 pi i k / 8}
template <typename T>
__device__ __forceinline__ void dft8(cplx<T> *v, int sign) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e, sign);
    dft4(o, sign);
    const T c = (T)0.70710678118654752440;
    const T sg = (T)sign;
    o[1] = cmul(o[1], cplx<T>{c, sg * c});
    o[2] = mul_i(o[2], sign);
    o[3] = cmul(o[3], cplx<T>{-c, sg * c});
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = {e[k].re + o[k].re, e[k].im + o[k].im};
        v[k + 4] = {e[k].re - o[k].re, e[k].im - o[k].im};
    }
}

template <typename T, int R>
__device__ __forceinline__ void dftr(cplx<T> *v, int sign) {
    if constexpr (R == 2) dft2(v[0], v[1]);
    else if constexpr (R == 4) dft4(v, sign);
    else dft8(v, sign);
}

// One radix-R pass over nb transforms of length 2^logn (LDS s[b * ld + i]),
// Ns = 2^logNs being the product of the earlier radices.  At most MAXB
// butterflies per thread (the host sizes the batches for it).
template <typename T, int R, int MAXB>
__device__ __forceinline__ void stockham_pass(cplx<T> *s, int ld, int logn, int logNs, int nb,
                                              int sign, const cplx<T> *__restrict__ tw, int loglt) {
    constexpr int LR = R == 2 ? 1 : (R == 4 ? 2 : 3);
    const int lognb = logn - LR;                 // log2 of butterflies per transform
    const int total = nb << lognb;
    const int Ns = 1 << logNs;
    const int tsh = loglt - logNs - LR;
    cplx<T> v[MAXB][R];
#pragma unroll
    for (int c = 0; c < MAXB; ++c) {
        const int t = threadIdx.x + c * blockDim.x;
        if (t < total) {
            const int b = t >> lognb, j = t & ((1 << lognb) - 1);
            const int jm = j & (Ns - 1);
            const cplx<T> *src = s + b * ld + j;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cplx<T> x = src[r << lognb];
                if (r > 0) {
                    cplx<T> w = tw[(r * jm) << tsh];
                    if (sign > 0) w.im = -w.im;
                    x = cmul(x, w);
                }
                v[c][r] = x;
            }
            dftr<T, R>(v[c], sign);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MAXB; ++c) {
        const int t = threadIdx.x + c * blockDim.x;
        if (t < total) {
            const int b = t >> lognb, j = t & ((1 << lognb) - 1);
            const int jm = j & (Ns - 1);
            cplx<T> *dst = s + b * ld + ((j >> logNs) << (logNs + LR)) + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r << logNs] = v[c][r];
        }
    }
    __syncthreads();
}

// nb transforms of length 2^logn in LDS, natural order in and out; sign -1
// forward, +1 inverse (unnormalised).  At most VPT values per thread of the
// workgroup (nb * 2^logn <= VPT blockDim): a pass holds that many complex
// values per thread in registers.  Ends with a barrier.
template <typename T, int VPT = 8>
__device__ void lds_fft_st(cplx<T> *s, int ld, int logn, int nb, int sign,
                           const cplx<T> *__restrict__ tw, int loglt) {
    int logNs = 0;
    if (logn == 1) {
        stockham_pass<T, 2, (VPT + 1) / 2>(s, ld, logn, 0, nb, sign, tw, loglt);
        return;
    }
    if (logn & 1) {
        stockham_pass<T, 8, (VPT + 7) / 8>(s, ld, logn, 0, nb, sign, tw, loglt);
        logNs = 3;
    }
    for (; logNs < logn; logNs += 2)
        stockham_pass<T, 4, (VPT + 3) / 4>(s, ld, logn, logNs, nb, sign, tw, loglt);
}

// Pass 1: rows (component, z, y) of nx reals, R rows per workgroup.  Loads
// u + dt f as nx/2 complex pairs z_m = x_2m + i x_2m+1, transforms them and
// unpacks X_k = E_k + e^{-2 pi i k/nx} O_k, k = 0 .. nx/2, with
// E_k = (Z_k + conj Z_{nh-k})/2 and O_k = (Z_k - conj Z_{nh-k})/(2i).
template <typename T>
__global__ __launch_bounds__(256) void k_fx_r2c(const T *__restrict__ u, const T *__restrict__ f,
                                                T dt, cplx<T> *__restrict__ U, int rows, int lognx,
                                                int rs, int R, const cplx<T> *__restrict__ tw,
                                                int loglt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *s = reinterpret_cast<cplx<T> *>(smem_raw);
    const int nx = 1 << lognx, lognh = lognx - 1, nh = nx >> 1;
    const int row0 = blockIdx.x * R;
    for (int e = threadIdx.x; e < R * nh; e += blockDim.x) {
        const int r = e >> lognh, m = e & (nh - 1);
        const int row = row0 + r;
        cplx<T> z = {(T)0, (T)0};
        if (row < rows) {
            const int64_t o = (int64_t)row * nx + 2 * m;
            z.re = u[o] + dt * f[o];
            z.im = u[o + 1] + dt * f[o + 1];
        }
        s[r * nh + m] = z;
    }
    __syncthreads();
    lds_fft_st(s, nh, lognh, R, -1, tw, loglt);
    for (int e = threadIdx.x; e < R * (nh + 1); e += blockDim.x) {
        const int r = e / (nh + 1), k = e - r * (nh + 1);
        const int row = row0 + r;
        if (row >= rows) continue;
        const cplx<T> zk = s[r * nh + (k & (nh - 1))];
        const cplx<T> zc = s[r * nh + ((nh - k) & (nh - 1))];
        // E = (zk + conj zc)/2, O = (zk - conj zc)/(2i)
        const cplx<T> E = {(zk.re + zc.re) * (T)0.5, (zk.im - zc.im) * (T)0.5};
        const cplx<T> O = {(zk.im + zc.im) * (T)0.5, -(zk.re - zc.re) * (T)0.5};
        const cplx<T> W = tw[k << (loglt - lognx)];
        const cplx<T> WO = cmul(W, O);
        U[(int64_t)row * rs + k] = {E.re + WO.re, E.im + WO.im};
    }
}

// Pass 5: the inverse of pass 1 (unnormalised): Z'_k = E'_k + i O'_k with
// E'_k = X_k + conj X_{nh-k}, O'_k = (X_k - conj X_{nh-k}) e^{2 pi i k/nx},
// inverse transform, x_2m = Re z_m, x_2m+1 = Im z_m.
template <typename T>
__global__ __launch_bounds__(256) void k_fx_c2r(const cplx<T> *__restrict__ U, T *__restrict__ u,
                                                int rows, int lognx, int rs, int R,
                                                const cplx<T> *__restrict__ tw, int loglt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *s = reinterpret_cast<cplx<T> *>(smem_raw);
    const int nx = 1 << lognx, lognh = lognx - 1, nh = nx >> 1;
    const int row0 = blockIdx.x * R;
    for (int e = threadIdx.x; e < R * nh; e += blockDim.x) {
        const int r = e >> lognh, k = e & (nh - 1);
        const int row = row0 + r;
        cplx<T> z = {(T)0, (T)0};
        if (row < rows) {
            const cplx<T> xk = U[(int64_t)row * rs + k];
            const cplx<T> xc = U[(int64_t)row * rs + (nh - k)];
            const cplx<T> E = {xk.re + xc.re, xk.im - xc.im};
            cplx<T> W = tw[k << (loglt - lognx)];
            W.im = -W.im;                                   // e^{+2 pi i k/nx}
            const cplx<T> O = cmul({xk.re - xc.re, xk.im + xc.im}, W);
            z = {E.re - O.im, E.im + O.re};
        }
        s[r * nh + k] = z;
    }
    __syncthreads();
    lds_fft_st(s, nh, lognh, R, +1, tw, loglt);
    for (int e = threadIdx.x; e < R * nh; e += blockDim.x) {
        const int r = e >> lognh, m = e & (nh - 1);
        const int row = row0 + r;
        if (row >= rows) continue;
        const cplx<T> z = s[r * nh + m];
        const int64_t o = (int64_t)row * nx + 2 * m;
        u[o] = z.re;
        u[o + 1] = z.im;
    }
}

// Passes 2 and 4: transform along y of every column (slab, kx); a workgroup
// owns TX consecutive kx columns of one slab (component, z).
template <typename T>
__global__ __launch_bounds__(256) void k_fy(cplx<T> *__restrict__ U, int nslab, int logny,
                                            int nkx, int rs, int logtx, int sign,
                                            const cplx<T> *__restrict__ tw, int loglt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *s = reinterpret_cast<cplx<T> *>(smem_raw);
    const int ny = 1 << logny, tx = 1 << logtx, ld = ny + 1;
    const int ntile = (nkx + tx - 1) >> logtx;
    const int slab = blockIdx.x / ntile, tile = blockIdx.x - slab * ntile;
    const int kx0 = tile << logtx;
    const int w = min(tx, nkx - kx0);
    cplx<T> *base = U + (int64_t)slab * ny * rs + kx0;
    for (int e = threadIdx.x; e < ny * tx; e += blockDim.x) {
        const int y = e >> logtx, c = e & (tx - 1);
        cplx<T> v = {(T)0, (T)0};
        if (c < w) v = base[(int64_t)y * rs + c];
        s[c * ld + y] = v;
    }
    __syncthreads();
    lds_fft_st(s, ld, logny, tx, sign, tw, loglt);
    for (int e = threadIdx.x; e < ny * tx; e += blockDim.x) {
        const int y = e >> logtx, c = e & (tx - 1);
        if (c < w) base[(int64_t)y * rs + c] = s[c * ld + y];
    }
}

// Logical block of a launch whose grid is padded to a multiple of kXcds:
// physical block b runs on XCD b mod kXcds; XCD x takes logical blocks
// [x G/kXcds, (x + 1) G/kXcds), in order.  A bijection on [0, grid).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int grid) {
    return (b % kXcds) * (grid / kXcds) + b / kXcds;
}

// Pass 3: for one ky and TX consecutive kx, the z lines of all three
// components: forward transform along z, the Fourier multiplier of the step
// (as in k_fluid_spectral, which holds the Nyquist rule), inverse transform.
// A tile narrower than a cache line shares each line with the next tile, so
// consecutive tiles are kept on one XCD (its own L2), one after the other.
constexpr int kZThreads = 512;
constexpr int kZVpt = 8;       // values per thread of the z pass

template <typename T>
__global__ __launch_bounds__(kZThreads) void k_fz_spec(cplx<T> *__restrict__ U, int lognx, int logny,
                                                 int lognz, int rs, int logtx, T kx0w, T ky0w,
                                                 T kz0w,
                                                 T nudt, T scale,
                                                 const cplx<T> *__restrict__ tw, int loglt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *s = reinterpret_cast<cplx<T> *>(smem_raw);
    const int nx = 1 << lognx, ny = 1 << logny, nz = 1 << lognz, tx = 1 << logtx;
    const int nkx = nx / 2 + 1, ld = nz + 1;
    const int ntile = (nkx + tx - 1) >> logtx;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= ny * ntile) return;       // grid padding
    const int iy = blk / ntile, tile = blk - iy * ntile;
    const int kx0 = tile << logtx;
    const int w = min(tx, nkx - kx0);
    const int64_t zstride = (int64_t)ny * rs, cstride = (int64_t)nz * zstride;
    cplx<T> *base = U + (int64_t)iy * rs + kx0;
    for (int e = threadIdx.x; e < 3 * nz * tx; e += blockDim.x) {
        const int c = e & (tx - 1), rz = e >> logtx;
        const int z = rz & (nz - 1), comp = rz >> lognz;
        cplx<T> v = {(T)0, (T)0};
        if (c < w) v = base[comp * cstride + z * zstride + c];
        s[(comp * tx + c) * ld + z] = v;
    }
    __syncthreads();
    lds_fft_st<T, kZVpt>(s, ld, lognz, 3 * tx, -1, tw, loglt);
    const int my = iy <= ny / 2 ? iy : iy - ny;
    const T ky = ky0w * (T)my;
    const T dky = (2 * iy == ny) ? (T)0 : ky;
    for (int e = threadIdx.x; e < nz * tx; e += blockDim.x) {
        const int c = e & (tx - 1), iz = e >> logtx;
        if (c >= w) continue;
        const int ix = kx0 + c;
        const int mz = iz <= nz / 2 ? iz : iz - nz;
        const T kx = kx0w * (T)ix, kz = kz0w * (T)mz;
        const T k2 = kx * kx + ky * ky + kz * kz;
        const T dkx = (2 * ix == nx) ? (T)0 : kx;
        const T dkz = (2 * iz == nz) ? (T)0 : kz;
        const T kd2 = dkx * dkx + dky * dky + dkz * dkz;
        cplx<T> &a = s[(0 * tx + c) * ld + iz];
        cplx<T> &b = s[(1 * tx + c) * ld + iz];
        cplx<T> &d = s[(2 * tx + c) * ld + iz];
        const T g = exp(-nudt * k2) * scale;
        cplx<T> A = a, B = b, D = d;
        if (kd2 > (T)0) {
            const T ik2 = (T)1 / kd2;
            const T pr = (dkx * A.re + dky * B.re + dkz * D.re) * ik2;
            const T pi = (dkx * A.im + dky * B.im + dkz * D.im) * ik2;
            A.re -= dkx * pr; A.im -= dkx * pi;
            B.re -= dky * pr; B.im -= dky * pi;
            D.re -= dkz * pr; D.im -= dkz * pi;
        }
        a = {A.re * g, A.im * g};
        b = {B.re * g, B.im * g};
        d = {D.re * g, D.im * g};
    }
    __syncthreads();
    lds_fft_st<T, kZVpt>(s, ld, lognz, 3 * tx, +1, tw, loglt);
    for (int e = threadIdx.x; e < 3 * nz * tx; e += blockDim.x) {
        const int c = e & (tx - 1), rz = e >> logtx;
        const int z = rz & (nz - 1), comp = rz >> lognz;
        if (c < w) base[comp * cstride + z * zstride + c] = s[(comp * tx + c) * ld + z];
    }
}

const char *fft_error(hipfftResult r) {
    switch (r) {
    case HIPFFT_SUCCESS: return "success";
    case HIPFFT_INVALID_PLAN: return "invalid plan";
    case HIPFFT_ALLOC_FAILED: return "allocation failed";
    case HIPFFT_INVALID_VALUE: return "invalid value";
    case HIPFFT_INTERNAL_ERROR: return "internal error";
    case HIPFFT_EXEC_FAILED: return "exec failed";
    case HIPFFT_SETUP_FAILED: return "setup failed";
    case HIPFFT_INVALID_SIZE: return "invalid size";
    default: return "hipFFT error";
    }
}

void release(erpp_fluid *fl) {
    if (fl->tw) (void)hipFree(fl->tw);
    if (fl->have_fwd) (void)hipfftDestroy(fl->fwd);
    if (fl->have_inv) (void)hipfftDestroy(fl->inv);
    if (fl->spec) (void)hipFree(fl->spec);
    delete fl;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

template <typename T>
hipError_t launch_force(erpp_fluid *fl, T *u, const T *f, hipStream_t st) {
    const int64_t count = 3 * fl->nodes;
    const bool vec = ((uintptr_t)u % 16 == 0) && ((uintptr_t)f % 16 == 0);
    constexpr int V = 16 / sizeof(T);
    const int64_t work = vec ? (count + V - 1) / V : count;
    // enough waves to fill every CU several times, grid-stride beyond that
    const int64_t blocks = std::min<int64_t>((work + kFluidBlock - 1) / kFluidBlock, 8192);
    if (vec)
        hipLaunchKernelGGL((k_fluid_force<T, V>), dim3((unsigned)blocks), dim3(kFluidBlock), 0,
                           st, u, f, (T)fl->dt, count);
    else
        hipLaunchKernelGGL((k_fluid_force<T, 1>), dim3((unsigned)blocks), dim3(kFluidBlock), 0,
                           st, u, f, (T)fl->dt, count);
    return hipGetLastError();
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// largest power of two <= 16 whose tile of columns fits `budget` bytes of LDS
// and at most `maxvals` values (eight per thread of the workgroup)
int tile_width(size_t bytes_per_column, size_t budget, size_t vals_per_column, size_t maxvals) {
    int tx = 16;
    while (tx > 1 && ((size_t)tx * bytes_per_column > budget || (size_t)tx * vals_per_column > maxvals))
        tx >>= 1;
    return tx;
}

constexpr size_t kFftLds = 64 * 1024;

template <typename T>
hipError_t launch_own(erpp_fluid *fl, T *u, const T *f, hipStream_t st) {
    const int nx = fl->n[0], ny = fl->n[1], nz = fl->n[2];
    const int lognx = ilog2(nx), logny = ilog2(ny), lognz = ilog2(nz), loglt = ilog2(fl->lt);
    const int nh = nx / 2, nkx = nh + 1, rs = fl->rs;
    const int rows = 3 * ny * nz;
    const cplx<T> *tw = (const cplx<T> *)fl->tw;
    cplx<T> *U = (cplx<T> *)fl->spec;
    const size_t cs = sizeof(cplx<T>);
    // pass 1: force + real FFT along x
    const int R = std::max(1, 512 / nh);
    const unsigned gx = (unsigned)((rows + R - 1) / R);
    hipLaunchKernelGGL(k_fx_r2c<T>, dim3(gx), dim3(256), (size_t)R * nh * cs, st, u, f,
                       (T)fl->dt, U, rows, lognx, rs, R, tw, loglt);
    // pass 2: forward FFT along y
    const int txy = tile_width((size_t)(ny + 1) * cs, kFftLds, (size_t)ny, 8 * 256);
    const int logtxy = ilog2(txy);
    const unsigned gy = (unsigned)(3 * nz * ((nkx + txy - 1) / txy));
    hipLaunchKernelGGL(k_fy<T>, dim3(gy), dim3(256), (size_t)txy * (ny + 1) * cs, st, U, 3 * nz,
                       logny, nkx, rs, logtxy, -1, tw, loglt);
    // pass 3: along z, the Fourier multiplier, back along z
    const int txz = tile_width((size_t)3 * (nz + 1) * cs, kFftLds, (size_t)3 * nz, (size_t)kZVpt * kZThreads);
    const int logtxz = ilog2(txz);
    const unsigned gz = (unsigned)((ny * ((nkx + txz - 1) / txz) + kXcds - 1) / kXcds * kXcds);
    const double tp = 2.0 * M_PI;
    hipLaunchKernelGGL(k_fz_spec<T>, dim3(gz), dim3(kZThreads), (size_t)3 * txz * (nz + 1) * cs, st, U,
                       lognx, logny, lognz, rs, logtxz, (T)(tp / fl->L[0]), (T)(tp / fl->L[1]),
                       (T)(tp / fl->L[2]), (T)(fl->nu * fl->dt), (T)(1.0 / (double)fl->nodes), tw,
                       loglt);
    // pass 4: inverse FFT along y
    hipLaunchKernelGGL(k_fy<T>, dim3(gy), dim3(256), (size_t)txy * (ny + 1) * cs, st, U, 3 * nz,
                       logny, nkx, rs, logtxy, +1, tw, loglt);
    // pass 5: inverse real FFT along x into u
    hipLaunchKernelGGL(k_fx_c2r<T>, dim3(gx), dim3(256), (size_t)R * nh * cs, st, U, u, rows,
                       lognx, rs, R, tw, loglt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spectral(erpp_fluid *fl, hipStream_t st) {
    const uint32_t modes = (uint32_t)fl->modes;
    const double tp = 2.0 * M_PI;
    const unsigned blocks = (modes + kFluidBlock - 1) / kFluidBlock;
    hipLaunchKernelGGL(k_fluid_spectral<T>, dim3(blocks), dim3(kFluidBlock), 0, st,
                       (cplx<T> *)fl->spec, (uint32_t)fl->n[0], (uint32_t)fl->n[1], (uint32_t)fl->n[2], modes,
                       (T)(tp / fl->L[0]), (T)(tp / fl->L[1]), (T)(tp / fl->L[2]),
                       (T)(fl->nu * fl->dt), (T)(1.0 / (double)fl->nodes));
    return hipGetLastError();
}

std::atomic<uint64_t> g_fluid_serial{1};

}  // namespace

namespace erpp {

uint64_t fluid_id(const erpp_fluid *fl) { return fl->id; }

erpp_status fluid_check(const erpp_fluid *fl, const erpp_box &b, double dt, erpp_precision prec,
                        int ibox) {
    for (int d = 0; d < 3; ++d) {
        if (fl->n[d] != b.n[d])
            return fail(ERPP_EINVAL, "box %d: fluid grid n[%d]=%d differs from the box's %d", ibox,
                        d, fl->n[d], b.n[d]);
        if (std::fabs(fl->L[d] - b.L[d]) > 1e-12 * b.L[d])
            return fail(ERPP_EINVAL, "box %d: fluid L[%d] differs from the box's", ibox, d);
    }
    if (fl->prec != prec) return fail(ERPP_EINVAL, "box %d: fluid precision differs", ibox);
    if (std::fabs(fl->dt - dt) > 1e-12 * dt)
        return fail(ERPP_EINVAL, "box %d: fluid dt differs from the plan's", ibox);
    // the self-disturbance removed by the update is what this fluid step makes
    // of one forcing step (App. E), so both must use the same viscosity
    if (std::fabs(fl->nu - b.nu) > 1e-12 * std::fabs(b.nu))
        return fail(ERPP_EINVAL, "box %d: fluid nu differs from the box's", ibox);
    if (b.shear != 0.0)
        return fail(ERPP_EINVAL, "box %d: the fluid step needs shear = 0", ibox);
    return ERPP_OK;
}

erpp_status fluid_launch(erpp_fluid *fl, void *u, const void *f, hipStream_t st) {
    if (fl->own) {
        hipError_t e = fl->prec == ERPP_F32_FAST
                           ? launch_own(fl, (float *)u, (const float *)f, st)
                           : launch_own(fl, (double *)u, (const double *)f, st);
        if (e != hipSuccess) return hip_fail(e, "fluid transform launch");
        return ERPP_OK;
    }
    hipfftResult r = hipfftSetStream(fl->fwd, st);
    if (r == HIPFFT_SUCCESS) r = hipfftSetStream(fl->inv, st);
    if (r != HIPFFT_SUCCESS) return fail(ERPP_EHIP, "hipfftSetStream: %s", fft_error(r));
    hipError_t e;
    if (fl->prec == ERPP_F32_FAST) {
        e = launch_force(fl, (float *)u, (const float *)f, st);
        if (e != hipSuccess) return hip_fail(e, "k_fluid_force launch");
        r = hipfftExecR2C(fl->fwd, (hipfftReal *)u, (hipfftComplex *)fl->spec);
        if (r != HIPFFT_SUCCESS) return fail(ERPP_EHIP, "hipfftExecR2C: %s", fft_error(r));
        e = launch_spectral<float>(fl, st);
        if (e != hipSuccess) return hip_fail(e, "k_fluid_spectral launch");
        r = hipfftExecC2R(fl->inv, (hipfftComplex *)fl->spec, (hipfftReal *)u);
        if (r != HIPFFT_SUCCESS) return fail(ERPP_EHIP, "hipfftExecC2R: %s", fft_error(r));
    } else {
        e = launch_force(fl, (double *)u, (const double *)f, st);
        if (e != hipSuccess) return hip_fail(e, "k_fluid_force launch");
        r = hipfftExecD2Z(fl->fwd, (hipfftDoubleReal *)u, (hipfftDoubleComplex *)fl->spec);
        if (r != HIPFFT_SUCCESS) return fail(ERPP_EHIP, "hipfftExecD2Z: %s", fft_error(r));
        e = launch_spectral<double>(fl, st);
        if (e != hipSuccess) return hip_fail(e, "k_fluid_spectral launch");
        r = hipfftExecZ2D(fl->inv, (hipfftDoubleComplex *)fl->spec, (hipfftDoubleReal *)u);
        if (r != HIPFFT_SUCCESS) return fail(ERPP_EHIP, "hipfftExecZ2D: %s", fft_error(r));
    }
    return ERPP_OK;
}

}  // namespace erpp

extern "C" {

erpp_status erpp_fluid_create(erpp_fluid **out, const int32_t n[3], const double L[3], double nu,
                              double dt, erpp_precision prec, void *stream) {
    using erpp::fail;
    if (!out) return fail(ERPP_EINVAL, "fluid pointer is NULL");
    *out = nullptr;
    if (!n || !L) return fail(ERPP_EINVAL, "n or L is NULL");
    if (prec != ERPP_F32_FAST && prec != ERPP_F64_PLAIN)
        return fail(ERPP_EINVAL, "unknown precision %d", (int)prec);
    if (!std::isfinite(nu) || nu < 0.0) return fail(ERPP_EINVAL, "nu must be finite and >= 0");
    if (!finite_pos(dt)) return fail(ERPP_EINVAL, "dt must be finite and > 0");
    int64_t nodes = 1;
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1) return fail(ERPP_EGEOM, "n[%d]=%d < 1", d, n[d]);
        if (!finite_pos(L[d])) return fail(ERPP_EGEOM, "L[%d] must be > 0", d);
        if (n[d] > 4096) return fail(ERPP_EUNSUPPORTED, "n[%d]=%d > 4096", d, n[d]);
        nodes *= n[d];
    }
    if (3 * nodes > INT32_MAX) return fail(ERPP_EUNSUPPORTED, "3 Nx Ny Nz > 2^31-1");
    erpp_fluid *fl = new (std::nothrow) erpp_fluid();
    if (!fl) return fail(ERPP_ENOMEM, "host allocation of the fluid stepper");
    for (int d = 0; d < 3; ++d) {
        fl->n[d] = n[d];
        fl->L[d] = L[d];
    }
    fl->id = g_fluid_serial.fetch_add(1);
    fl->nu = nu;
    fl->dt = dt;
    fl->prec = prec;
    fl->nodes = nodes;
    fl->modes = (int64_t)n[2] * n[1] * (n[0] / 2 + 1);
    const size_t csize = prec == ERPP_F32_FAST ? 2 * sizeof(float) : 2 * sizeof(double);
    // powers of two up to 1024 (a z tile of one column then fits 64 KiB of LDS
    // in FP64) take this file's transforms; their spectrum rows are padded to
    // 16 complex values so that every column tile starts a cache line
    const bool own = pow2(n[0]) && pow2(n[1]) && pow2(n[2]) && n[0] >= 4 && n[1] >= 2 &&
                     n[2] >= 2 && n[0] <= 1024 && n[1] <= 1024 && n[2] <= 1024;
    fl->rs = own ? ((n[0] / 2 + 1 + 15) / 16) * 16 : n[0] / 2 + 1;
    const size_t nspec = 3 * (size_t)n[2] * n[1] * fl->rs;
    hipError_t e = hipMalloc(&fl->spec, nspec * csize);
    if (e != hipSuccess) {
        fl->spec = nullptr;
        release(fl);
        return fail(ERPP_ENOMEM, "spectral buffer: %s", hipGetErrorString(e));
    }
    // own transforms: a twiddle table e^{-2 pi i j / lt}, j in [0, lt), for the
    // largest size lt, computed in FP64
    if (own) {
        const int lt = std::max(n[0], std::max(n[1], n[2]));
        const size_t ntw = (size_t)lt;
        std::vector<double> h(2 * ntw);
        for (size_t j = 0; j < ntw; ++j) {
            const double a = 2.0 * M_PI * (double)j / (double)lt;
            h[2 * j] = std::cos(a);
            h[2 * j + 1] = -std::sin(a);
        }
        const size_t esz = prec == ERPP_F32_FAST ? sizeof(float) : sizeof(double);
        e = hipMalloc(&fl->tw, 2 * ntw * esz);
        if (e != hipSuccess) {
            fl->tw = nullptr;
            release(fl);
            return fail(ERPP_ENOMEM, "twiddle table: %s", hipGetErrorString(e));
        }
        if (prec == ERPP_F32_FAST) {
            std::vector<float> hf(h.begin(), h.end());
            e = hipMemcpy(fl->tw, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(fl->tw, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            release(fl);
            return erpp::hip_fail(e, "twiddle upload");
        }
        fl->lt = lt;
        fl->own = true;
        *out = fl;
        return ERPP_OK;
    }
    // [Nz][Ny][Nx] real <-> [Nz][Ny][Nx/2+1] complex, three components batched
    int dims[3] = {n[2], n[1], n[0]};
    int rembed[3] = {n[2], n[1], n[0]};
    int cembed[3] = {n[2], n[1], n[0] / 2 + 1};
    const bool f32 = prec == ERPP_F32_FAST;
    hipfftResult r = hipfftPlanMany(&fl->fwd, 3, dims, rembed, 1, (int)nodes, cembed, 1,
                                    (int)fl->modes, f32 ? HIPFFT_R2C : HIPFFT_D2Z, 3);
    if (r != HIPFFT_SUCCESS) {
        release(fl);
        return fail(r == HIPFFT_ALLOC_FAILED ? ERPP_ENOMEM : ERPP_EHIP,
                    "hipfftPlanMany (forward): %s", fft_error(r));
    }
    fl->have_fwd = true;
    r = hipfftPlanMany(&fl->inv, 3, dims, cembed, 1, (int)fl->modes, rembed, 1, (int)nodes,
                       f32 ? HIPFFT_C2R : HIPFFT_Z2D, 3);
    if (r != HIPFFT_SUCCESS) {
        release(fl);
        return fail(r == HIPFFT_ALLOC_FAILED ? ERPP_ENOMEM : ERPP_EHIP,
                    "hipfftPlanMany (inverse): %s", fft_error(r));
    }
    fl->have_inv = true;
    (void)stream;
    *out = fl;
    return ERPP_OK;
}

erpp_status erpp_fluid_step(erpp_fluid *fl, void *u, const void *f, void *stream) {
    using erpp::fail;
    if (!fl) return fail(ERPP_EINVAL, "fluid is NULL");
    if (!u || !f) return fail(ERPP_EINVAL, "u or f is NULL");
    if (u == f) return fail(ERPP_EINVAL, "u and f alias");
    return erpp::fluid_launch(fl, u, f, (hipStream_t)stream);
}

void erpp_fluid_destroy(erpp_fluid *fl) {
    if (!fl) return;
    (void)hipDeviceSynchronize();
    release(fl);
}

}  // extern "C"
