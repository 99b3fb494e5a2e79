// Measurement kernels for fitting the hit-rate functions on the GPU itself
// (Sec. 4.5, Capacity Misses: the fit functions are fitted to observed hit
// rates of the redundant volumes against the oversubscription O).
//
// star25 is the range-4 3D 25-point star stencil of Sec. 5.2 in fp64 on
// x-fastest arrays with 4 ghost layers per side, with thread folding in y and
// z (each thread updates FY x FZ points; loads of one point it needs more
// than once are loaded once).  copy1 streams n doubles once (a transfer of
// known size, to scale request counters to bytes).  The launchers take
// device pointers and a stream and return a hipError_t.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int R = 4;  // stencil range

template <int FY, int FZ>
__global__ void star25(const double* __restrict__ src, double* __restrict__ dst, int nx, int ny, int nz)
{
    const int gx = blockIdx.x * blockDim.x + threadIdx.x;
    const int gy = (blockIdx.y * blockDim.y + threadIdx.y) * FY;
    const int gz = (blockIdx.z * blockDim.z + threadIdx.z) * FZ;
    if (gx >= nx || gy >= ny || gz >= nz) return;
    const int64_t sy = nx + 2 * R, sz = sy * (ny + 2 * R);
#pragma unroll
    for (int k = 0; k < FZ; k++)
#pragma unroll
        for (int j = 0; j < FY; j++) {
            const int64_t c = (gx + R) + sy * (gy + j + R) + sz * (gz + k + R);
            double v = 0.5 * src[c];
#pragma unroll
            for (int q = 1; q <= R; q++) {
                const double w = 1.0 / (q + 1);
                v += w * (src[c - q] + src[c + q] + src[c - q * sy] + src[c + q * sy] + src[c - q * sz] +
                          src[c + q * sz]);
            }
            dst[c] = v;
        }
}

// A lattice kernel given by its access table: every thread of the
// nx x ny x nz lattice (x fastest, no ghost layers: fields carry margins of
// their own) sums its n_ld loads in[ld_field[a]][c + ld_off[a]] and writes
// the sum to each of its n_st store fields at its own point.  The table is
// uniform across the wave, so its entries come through scalar loads and the
// vector memory traffic is the kernel's own.
__global__ void gather(const double* const* __restrict__ in, double* const* __restrict__ out,
                       const int32_t* __restrict__ ld_field, const int64_t* __restrict__ ld_off, int n_ld,
                       int n_st, int nx, int ny, int nz)
{
    const int gx = blockIdx.x * blockDim.x + threadIdx.x;
    const int gy = blockIdx.y * blockDim.y + threadIdx.y;
    const int gz = blockIdx.z * blockDim.z + threadIdx.z;
    if (gx >= nx || gy >= ny || gz >= nz) return;
    const int64_t c = gx + (int64_t)nx * (gy + (int64_t)ny * gz);
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int a = 0;
    for (; a + 4 <= n_ld; a += 4) {
        v0 += in[ld_field[a]][c + ld_off[a]];
        v1 += in[ld_field[a + 1]][c + ld_off[a + 1]];
        v2 += in[ld_field[a + 2]][c + ld_off[a + 2]];
        v3 += in[ld_field[a + 3]][c + ld_off[a + 3]];
    }
    for (; a < n_ld; a++) v0 += in[ld_field[a]][c + ld_off[a]];
    const double v = (v0 + v1) + (v2 + v3);
    for (int j = 0; j < n_st; j++) out[j][c] = v + j;
}

__global__ void copy1(const double* __restrict__ src, double* __restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

template <int FY, int FZ>
hipError_t launch(const double* src, double* dst, int nx, int ny, int nz, int bx, int by, int bz, hipStream_t s)
{
    const int ty = ny / FY, tz = nz / FZ;
    dim3 grid((nx + bx - 1) / bx, (ty + by - 1) / by, (tz + bz - 1) / bz);
    hipLaunchKernelGGL((star25<FY, FZ>), grid, dim3(bx, by, bz), 0, s, src, dst, nx, ny, nz);
    return hipGetLastError();
}

}  // namespace

extern "C" {

// dst = stencil(src) over the nx x ny x nz interior; arrays of
// (nx + 8)(ny + 8)(nz + 8) doubles.  fy, fz in {1, 2, 4, 8}, dividing ny, nz.
int32_t probe_star25(const double* src, double* dst, int32_t nx, int32_t ny, int32_t nz, int32_t bx, int32_t by,
                     int32_t bz, int32_t fy, int32_t fz, void* stream)
{
    if (nx < 1 || ny < 1 || nz < 1 || bx < 1 || by < 1 || bz < 1 || (int64_t)bx * by * bz > 1024) return -1;
    if (ny % fy || nz % fz) return -1;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipErrorInvalidValue;
#define WSE_PROBE_CASE(A, B) \
    if (fy == A && fz == B) e = launch<A, B>(src, dst, nx, ny, nz, bx, by, bz, s);
    WSE_PROBE_CASE(1, 1) WSE_PROBE_CASE(1, 2) WSE_PROBE_CASE(1, 4) WSE_PROBE_CASE(1, 8)
    WSE_PROBE_CASE(2, 1) WSE_PROBE_CASE(2, 2) WSE_PROBE_CASE(2, 4) WSE_PROBE_CASE(2, 8)
    WSE_PROBE_CASE(4, 1) WSE_PROBE_CASE(4, 2) WSE_PROBE_CASE(4, 4) WSE_PROBE_CASE(4, 8)
    WSE_PROBE_CASE(8, 1) WSE_PROBE_CASE(8, 2) WSE_PROBE_CASE(8, 4) WSE_PROBE_CASE(8, 8)
#undef WSE_PROBE_CASE
    return e == hipSuccess ? 0 : -4;
}

// The access-table lattice kernel (gather) over nx x ny x nz with blocks
// bx x by x bz: in/out are device arrays of field pointers, ld_field/ld_off
// device arrays of n_ld entries (field index into in, offset in elements).
// Every field must hold the lattice plus a margin of the largest |offset| on
// both sides.
int32_t probe_lattice(const double* const* in, double* const* out, const int32_t* ld_field, const int64_t* ld_off,
                      int32_t n_ld, int32_t n_st, int32_t nx, int32_t ny, int32_t nz, int32_t bx, int32_t by,
                      int32_t bz, void* stream)
{
    if (nx < 1 || ny < 1 || nz < 1 || bx < 1 || by < 1 || bz < 1 || (int64_t)bx * by * bz > 1024) return -1;
    if (n_ld < 0 || n_st < 0 || !in || !out || !ld_field || !ld_off) return -1;
    dim3 grid((nx + bx - 1) / bx, (ny + by - 1) / by, (nz + bz - 1) / bz);
    hipLaunchKernelGGL(gather, grid, dim3(bx, by, bz), 0, (hipStream_t)stream, in, out, ld_field, ld_off, n_ld,
                       n_st, nx, ny, nz);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// dst[i] = src[i] for i < n (one read and one write of 8 bytes each)
int32_t probe_copy(const double* src, double* dst, int64_t n, void* stream)
{
    if (n < 1) return -1;
    hipLaunchKernelGGL(copy1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, src, dst, n);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
