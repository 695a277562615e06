// fluid.hip -- periodic unsteady-Stokes step of the disturbance field
// (Sec. 2.3, eq. velo_reg_eq) by the forcing / diffusion / projection
// splitting of App. E, pseudo-spectral with hipFFT.
//
// One step is four launches on the caller's stream:
//   k_fluid_force     u += dt f                      (eq. forcing_step)
//   forward R2C       U = FFT(u), three components batched
//   k_fluid_spectral  U <- exp(-nu k^2 dt) (I - k k^T / k^2) U / (Nx Ny Nz)
//                     (exact heat semigroup, eq. diffusion_step, then the
//                     projection lap(phi) = -div(u*), u = u* + grad(phi))
//   inverse C2R       u = IFFT(U)
// The forward transform may overwrite u; the inverse rewrites all of it.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <new>

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
    hipError_t e = hipMalloc(&fl->spec, 3 * (size_t)fl->modes * csize);
    if (e != hipSuccess) {
        fl->spec = nullptr;
        release(fl);
        return fail(ERPP_ENOMEM, "spectral buffer: %s", hipGetErrorString(e));
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
