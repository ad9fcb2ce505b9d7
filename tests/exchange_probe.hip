// exchange_probe.hip -- a measurement probe, not part of the library: one
// radix-pass exchange of the segment transform done through LDS (as the
// kernels do) and with the gfx950 cross-lane swaps, to weigh the two.
//
// The exchange is the one between the last two passes of a 1024-point
// segment transform held by one wave (16 complex values per lane): lane
// (k1, p) = (lane % 16, lane / 16) holds v[r], r < 16, and afterwards holds
// in v[4 pp + g] the value lane (k1, pp) held in v[4 p + g] (g, pp < 4).  For
// each g that is a transpose of a 4 x 4 block of (register, row of 16 lanes)
// and applying it twice gives the input back.
//   method 0: through LDS, each lane writing its 16 values and reading 16,
//             laid out as the segment transform lays out this exchange
//             (slot k1 * 65 + r * 4 + p); the workgroup is one wave, so the
//             barriers compile to waits on its own LDS accesses;
//   method 1: v_permlane32_swap then v_permlane16_swap on register pairs,
//             four swaps per g and component (32 per exchange), no LDS.
// Each wave runs `reps` exchanges, adding 1 to v[0] after each, and writes
// its values back.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

struct cf {
    float re, im;
};

constexpr int kRow = 65;            // 64 lanes + 1 pad (complex slots)

__device__ __forceinline__ void exchange_lds(cf (&v)[16], cf *lds, int k1, int p)
{
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[k1 * kRow + r * 4 + p] = v[r];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) v[4 * pp + g] = lds[k1 * kRow + (4 * p + g) * 4 + pp];
    __syncthreads();
}

// transpose of (register i, row q) for four registers: x[i] row q <- x[q] row i
__device__ __forceinline__ void transpose4(float &x0, float &x1, float &x2, float &x3)
{
    auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(x0), __float_as_uint(x2), false, false);
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x1), __float_as_uint(x3), false, false);
    auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
    auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
    x0 = __uint_as_float(c[0]);
    x1 = __uint_as_float(c[1]);
    x2 = __uint_as_float(d[0]);
    x3 = __uint_as_float(d[1]);
}

__device__ __forceinline__ void exchange_swap(cf (&v)[16])
{
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        transpose4(v[g].re, v[4 + g].re, v[8 + g].re, v[12 + g].re);
        transpose4(v[g].im, v[4 + g].im, v[8 + g].im, v[12 + g].im);
    }
}

template <int METHOD>
__global__ __launch_bounds__(64) void exchange_kernel(const cf *__restrict__ in, cf *__restrict__ out, int reps)
{
    __shared__ cf lds[16 * kRow];
    const int lane = threadIdx.x, k1 = lane & 15, p = lane >> 4;
    const int64_t base = (int64_t)blockIdx.x * 64 * 16;
    cf v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = in[base + r * 64 + lane];
    for (int it = 0; it < reps; ++it) {
        if constexpr (METHOD == 0) exchange_lds(v, lds, k1, p);
        else exchange_swap(v);
        v[0].re += 1.0f;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) out[base + r * 64 + lane] = v[r];
}

}  // namespace

// in/out: device float pairs [waves][16][64]; method 0 (LDS) or 1 (swaps).
// Returns 0, or -1 for a bad argument, or the HIP error code of the launch.
extern "C" int exchange_probe(int method, const void *d_in, void *d_out, int waves, int reps, void *stream)
{
    if (!d_in || !d_out || waves <= 0 || reps < 0 || (method != 0 && method != 1)) return -1;
    const hipStream_t st = (hipStream_t)stream;
    if (method == 0)
        hipLaunchKernelGGL(exchange_kernel<0>, dim3(waves), dim3(64), 0, st, (const cf *)d_in, (cf *)d_out, reps);
    else
        hipLaunchKernelGGL(exchange_kernel<1>, dim3(waves), dim3(64), 0, st, (const cf *)d_in, (cf *)d_out, reps);
    return (int)hipGetLastError();
}
