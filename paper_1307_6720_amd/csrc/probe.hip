// Access-pattern reference for the roofline of the level-0 smoother: a
// kernel that moves the smoother's compulsory bytes in the smoother's own
// memory order, with no LDS, barrier or arithmetic worth the name.  Its
// rate is the ceiling the z-marching tile pattern itself allows on this
// memory system; the smoother's rate is judged against it and against a
// plain copy.  Measurement aid only: no solve uses it.
#include "internal.h"
#include "plan.h"

namespace mhs {
namespace {

__device__ __forceinline__ int probe_xcd_tile()
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int x = b % 8, q = b / 8;
    const int per = nb / 8, rem = nb % 8;
    return x * per + min(x, rem) + q;
}

// Per workgroup: an x-y tile of TX x TY interior nodes of one request,
// marching kz planes.  Like the smoother it reads, for every plane from two
// below the chunk to one above it, the tile plus a two-node ring of u_in
// (clamped at the array edge) two planes ahead of their use, f at the
// tile's nodes of the chunk's planes, and writes u_out at those nodes.
template <int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_pattern(const float *__restrict__ u, const float *__restrict__ f,
                                                float *__restrict__ o, int nx, int ny, int nz, int ntx, int nty,
                                                int ntz, int kz)
{
    constexpr int WX = TX + 4, WY = TY + 4, WC = WX * WY;
    constexpr int WPER = (WC + NT - 1) / NT;
    static_assert((TX * TY) % NT == 0, "tile must be a multiple of the block");
    constexpr int TPER = TX * TY / NT;
    constexpr int D = 2;
    const int tid = threadIdx.x;
    int t = probe_xcd_tile();
    const int per = ntx * nty * ntz;
    const int req = t / per;
    t -= req * per;
    const int tx = t % ntx;
    t /= ntx;
    const int ty = t % nty;
    const int tz = t / nty;
    const size_t sxy = (size_t)nx * ny;
    const size_t base = (size_t)req * sxy * (size_t)nz;
    const int i0 = 1 + tx * TX, j0 = 1 + ty * TY;
    const int kb = 1 + tz * kz, ke = min(kb + kz, nz - 1);
    const int ptop = min(ke + 1, nz - 1);
    int wo[WPER];
#pragma unroll
    for (int r = 0; r < WPER; ++r) {
        const int e = min(tid + r * NT, WC - 1);
        const int w = e / WX, c = e - w * WX;
        wo[r] = min(max(i0 - 2 + c, 0), nx - 1) + nx * min(max(j0 - 2 + w, 0), ny - 1);
    }
    int to[TPER];
    uint32_t tok = 0;
#pragma unroll
    for (int r = 0; r < TPER; ++r) {
        const int e = tid + r * NT;
        const int w = e / TX, c = e - w * TX;
        const int i = i0 + c, j = j0 + w;
        to[r] = min(i, nx - 1) + nx * min(j, ny - 1);
        if (i <= nx - 2 && j <= ny - 2) tok |= 1u << r;
    }
    const float *ub = u + base;
    const float *fb = f + base;
    float *ob = o + base;
    float ru[D][WPER], rf[D][TPER];
    const int p0 = max(kb - 2, 0);
    // f only on the planes the chunk writes (the workgroup-uniform branch
    // skips it on the halo planes below and above)
    auto load = [&](int p, float(&du)[WPER], float(&df)[TPER]) {
#pragma unroll
        for (int r = 0; r < WPER; ++r) du[r] = ub[sxy * p + wo[r]];
        if (p >= kb && p < ke) {
#pragma unroll
            for (int r = 0; r < TPER; ++r) df[r] = fb[sxy * p + to[r]];
        }
    };
#pragma unroll
    for (int q = 0; q < D; ++q) {
#pragma unroll
        for (int r = 0; r < TPER; ++r) rf[q][r] = 0.0f;
        load(min(p0 + q, ptop), ru[q], rf[q]);
    }
    float acc = 0.0f;
    for (int s0 = p0; s0 <= ptop; s0 += D) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const int p = s0 + q;
#pragma unroll
            for (int r = 0; r < WPER; ++r) acc += ru[q][r];
            if (p >= kb && p < ke) {
#pragma unroll
                for (int r = 0; r < TPER; ++r)
                    if ((tok >> r) & 1) ob[sxy * p + to[r]] = rf[q][r] + 1e-30f * acc;
            }
            load(min(p + D, ptop), ru[q], rf[q]);
        }
    }
}

} // namespace
} // namespace mhs

extern "C" int mhs_probe_smoother_pattern(const float *d_u, const float *d_f, float *d_out, int32_t nx, int32_t ny,
                                          int32_t nz, int32_t nreq, int32_t tile, int32_t kz, void *stream)
{
    using namespace mhs;
    if (!d_u || !d_f || !d_out) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    if (nx < 3 || ny < 3 || nz < 3 || nreq < 1 || kz < 1 || (tile != 0 && tile != 1))
        return fail(MHS_ERR_INVALID_ARG, "probe: bad sizes (nx %d ny %d nz %d nreq %d kz %d tile %d)", nx, ny, nz,
                    nreq, kz, tile);
    const int TX = tile ? 256 : 64, TY = tile ? 8 : 16;
    const long ntx = ceil_div(nx - 2, TX), nty = ceil_div(ny - 2, TY), ntz = ceil_div(nz - 2, kz);
    const long groups = ntx * nty * ntz * (long)nreq;
    if (groups > (1L << 30)) return fail(MHS_ERR_INVALID_ARG, "probe: too many workgroups");
    hipStream_t s = (hipStream_t)stream;
    if (tile)
        hipLaunchKernelGGL((k_pattern<256, 8, 1024>), dim3((unsigned)groups), dim3(1024), 0, s, d_u, d_f, d_out, nx,
                           ny, nz, (int)ntx, (int)nty, (int)ntz, kz);
    else
        hipLaunchKernelGGL((k_pattern<64, 16, 512>), dim3((unsigned)groups), dim3(512), 0, s, d_u, d_f, d_out, nx,
                           ny, nz, (int)ntx, (int)nty, (int)ntz, kz);
    HIPCHK(hipGetLastError());
    return MHS_OK;
}
