// Storage codecs: spinor precision changes (FP64 <-> FP32, FP16 with a per-site scale) and
// link narrowing / 12-real compression / FP64 reunitarisation.
//
// Section 2.4 describes a Compressor that may change the precision of communicated fields; the
// same idea sets the storage precision of the sloppy solver's fields here.
#include "device.h"
#include "launch.h"

namespace gridmi {

// Read a site's 24 reals as float or double (F16S decodes with its scale).
template <typename T>
__device__ __forceinline__ void read_site(const void *src, int prec, const float *scale, size_t site, T v[24]) {
    if (prec == GRID_F64) {
        const double2 *q = reinterpret_cast<const double2 *>(src) + site * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            double2 d = q[k];
            v[2 * k] = static_cast<T>(d.x);
            v[2 * k + 1] = static_cast<T>(d.y);
        }
    } else if (prec == GRID_F32) {
        const float4 *q = reinterpret_cast<const float4 *>(src) + site * 6;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float4 f = q[k];
            v[4 * k] = f.x;
            v[4 * k + 1] = f.y;
            v[4 * k + 2] = f.z;
            v[4 * k + 3] = f.w;
        }
    } else {
        const uint4 *q = reinterpret_cast<const uint4 *>(src) + site * 3;
        const float s = scale[site];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint4 w = q[k];
            const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[8 * k + 2 * j] = static_cast<T>(half_bits_to_float(ww[j] & 0xffffu) * s);
                v[8 * k + 2 * j + 1] = static_cast<T>(half_bits_to_float(ww[j] >> 16) * s);
            }
        }
    }
}

__global__ void __launch_bounds__(256)
k_convert_spinor(const void *__restrict__ src, int src_prec, const float *__restrict__ src_scale, void *__restrict__ dst,
                 int dst_prec, float *__restrict__ dst_scale, long n_sites) {
    const long site = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
    if (site >= n_sites) return;
    if (dst_prec == GRID_F64) {
        double v[24];
        read_site<double>(src, src_prec, src_scale, site, v);
        double2 *q = reinterpret_cast<double2 *>(dst) + site * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = make_double2(v[2 * k], v[2 * k + 1]);
        return;
    }
    float v[24];
    read_site<float>(src, src_prec, src_scale, site, v);   // F64 -> float rounds to nearest even
    if (dst_prec == GRID_F32) {
        float4 *q = reinterpret_cast<float4 *>(dst) + site * 6;
#pragma unroll
        for (int k = 0; k < 6; ++k) q[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
        return;
    }
    // FP16 storage: s = max |v|, code = half(v * (1/s)), zeros for s = 0
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf(v[k]));
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    uint32_t w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = scaled_half_bits(v[2 * k], inv) | (scaled_half_bits(v[2 * k + 1], inv) << 16);
    uint4 *q = reinterpret_cast<uint4 *>(dst) + site * 3;
    q[0] = make_uint4(w[0], w[1], w[2], w[3]);
    q[1] = make_uint4(w[4], w[5], w[6], w[7]);
    q[2] = make_uint4(w[8], w[9], w[10], w[11]);
    dst_scale[site] = m;
}

hipError_t launch_convert_spinor(const void *src, int src_prec, const float *src_scale, void *dst, int dst_prec,
                                 float *dst_scale, long n_sites, hipStream_t stream) {
    if (n_sites == 0) return hipSuccess;
    const long blocks = (n_sites + 255) / 256;
    hipLaunchKernelGGL(k_convert_spinor, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, src, src_prec,
                       src_scale, dst, dst_prec, dst_scale, n_sites);
    return hipGetLastError();
}

// One thread per link: FP64 L18 in; optional FP64 reunitarisation; narrowed rows out.
__global__ void __launch_bounds__(256)
k_convert_links(const double2 *__restrict__ src, void *__restrict__ dst, int dst_prec, int rows, int reunit,
                long n_links) {
    const long l = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
    if (l >= n_links) return;
    Cx<double> u[3][3];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double2 d = src[l * 9 + k];
        u[k / 3][k % 3] = {d.x, d.y};
    }
    if (reunit) {
        // row0 /= |row0|; row1 -= (row0^dagger row1) row0; row1 /= |row1|; row2 = conj(row0 x row1)
        double n0 = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) n0 += u[0][b].r * u[0][b].r + u[0][b].i * u[0][b].i;
        n0 = 1.0 / sqrt(n0);
#pragma unroll
        for (int b = 0; b < 3; ++b) u[0][b] = cscale(n0, u[0][b]);
        Cx<double> d = {0, 0};
#pragma unroll
        for (int b = 0; b < 3; ++b) d = cmacc(d, u[0][b], u[1][b]);
#pragma unroll
        for (int b = 0; b < 3; ++b) u[1][b] = csub(u[1][b], cmul(d, u[0][b]));
        double n1 = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) n1 += u[1][b].r * u[1][b].r + u[1][b].i * u[1][b].i;
        n1 = 1.0 / sqrt(n1);
#pragma unroll
        for (int b = 0; b < 3; ++b) u[1][b] = cscale(n1, u[1][b]);
        rebuild_row2(u);
    }
    const int n = rows * 3;
    if (dst_prec == GRID_F64) {
        double2 *q = reinterpret_cast<double2 *>(dst) + l * n;
        for (int k = 0; k < n; ++k) q[k] = make_double2(u[k / 3][k % 3].r, u[k / 3][k % 3].i);
    } else if (dst_prec == GRID_F32) {
        float2 *q = reinterpret_cast<float2 *>(dst) + l * n;
        for (int k = 0; k < n; ++k)
            q[k] = make_float2(static_cast<float>(u[k / 3][k % 3].r), static_cast<float>(u[k / 3][k % 3].i));
    } else {
        uint32_t *q = reinterpret_cast<uint32_t *>(dst) + l * n;
        for (int k = 0; k < n; ++k)
            q[k] = float_to_half_bits(static_cast<float>(u[k / 3][k % 3].r)) |
                   (float_to_half_bits(static_cast<float>(u[k / 3][k % 3].i)) << 16);
    }
}

hipError_t launch_convert_links(const void *src, void *dst, int dst_prec, int dst_fmt, int reunitarise, long n_links,
                                hipStream_t stream) {
    if (n_links == 0) return hipSuccess;
    const long blocks = (n_links + 255) / 256;
    hipLaunchKernelGGL(k_convert_links, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       reinterpret_cast<const double2 *>(src), dst, dst_prec, dst_fmt == GRID_L12 ? 2 : 3,
                       reunitarise ? 1 : 0, n_links);
    return hipGetLastError();
}

}  // namespace gridmi
