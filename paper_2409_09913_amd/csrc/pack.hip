// Packing of B-bit codes into the tile layout read by the int8 matrix-core
// scan.  A B-bit code is split into power-of-two parts (Sec. 3.3 and
// Sec. 4.2 describe splitting y_u into parts whose sizes are powers of two),
// e.g. 7 = 4 + 2 + 1 with the 1-bit part being the most significant bit
// (RaBitQ's sign code).  Inside a K-block of 64 dimensions, lane L of the
// wave covers vector L%32 and, for s in {0,1}, the 16 dimensions
// kb*64 + s*32 + (L/32)*16 + j.  Those 32 values of one part of width w are
// stored in w dwords so that one shift and one mask per output dword unpack
// them into bytes: output dword c = 4s + d (byte b <-> j = 4d + b) is slice c
// of the part, found in dword c*w/8 at bit offset (c % (8/w)) * w of every
// byte.
#include "erq_common.h"

namespace erq {

namespace {

__device__ inline int find_list(const int64_t* off, int64_t nlist, int64_t x) {
    // largest l with off[l] <= x (off non-decreasing, off[0] = 0)
    int64_t lo = 0, hi = nlist;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid;
    }
    return (int)lo;
}

}  // namespace

__global__ void pack_kernel(const uint8_t* __restrict__ codes, const int64_t* __restrict__ list_off,
                            const int64_t* __restrict__ tile_off, int64_t nlist, int dp, int bits,
                            int64_t ntiles, uint8_t* __restrict__ packed)
{
    const int nkb = dp / 64;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = ntiles * nkb * 64;
    if (gid >= total) return;
    const int L = (int)(gid & 63);
    const int64_t tk = gid >> 6;
    const int kb = (int)(tk % nkb);
    const int64_t T = tk / nkb;
    // tile_off is non-decreasing; empty lists repeat offsets: find the list owning T
    int l = find_list(tile_off, nlist, T);
    while (l + 1 <= nlist && tile_off[l + 1] <= T) ++l;
    const int64_t t = T - tile_off[l];
    const int64_t nl = list_off[l + 1] - list_off[l];
    const int64_t vloc = t * 32 + (L & 31);
    const bool valid = vloc < nl;
    const uint8_t* src = codes + (list_off[l] + vloc) * (int64_t)dp;
    const int xr = (bits == 8) ? 0x80 : 0;
    // the 32 byte values of this lane: index c*4 + b (c = 4s + d) <-> dim s*32 + h*16 + 4d + b
    uint32_t vals[32];
    const int h = L >> 5;
    for (int s = 0; s < 2; ++s)
        for (int jj = 0; jj < 16; ++jj) {
            int dim = kb * 64 + s * 32 + h * 16 + jj;
            vals[s * 16 + jj] = valid ? (uint32_t)(src[dim] ^ xr) : (uint32_t)xr;
        }
    Parts P = parts_of(bits);
    uint8_t* dst = packed + T * (int64_t)(4 * dp * bits) + (int64_t)kb * 256 * bits;
    int wsum = 0;
    for (int p = 0; p < P.n; ++p) {
        const int w = P.w[p], pos = P.pos[p];
        const int per = 8 / w;              // slices per dword
        uint32_t out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int c = 0; c < 8; ++c) {
            int m = c / per;
            int sh = (c % per) * w;
            for (int b = 0; b < 4; ++b) {
                uint32_t v = (vals[c * 4 + b] >> pos) & ((1u << w) - 1u);
                out[m] |= v << (8 * b + sh);
            }
        }
        uint32_t* d32 = (uint32_t*)(dst + wsum * 256 + L * 4 * w);
        for (int m = 0; m < w; ++m) d32[m] = out[m];
        wsum += w;
    }
}

__global__ void unpack_kernel(const uint8_t* __restrict__ packed, const int64_t* __restrict__ list_off,
                              const int64_t* __restrict__ tile_off, int64_t nlist, int dp, int bits,
                              int64_t ntiles, uint8_t* __restrict__ codes)
{
    const int nkb = dp / 64;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = ntiles * nkb * 64;
    if (gid >= total) return;
    const int L = (int)(gid & 63);
    const int64_t tk = gid >> 6;
    const int kb = (int)(tk % nkb);
    const int64_t T = tk / nkb;
    int l = find_list(tile_off, nlist, T);
    while (l + 1 <= nlist && tile_off[l + 1] <= T) ++l;
    const int64_t t = T - tile_off[l];
    const int64_t nl = list_off[l + 1] - list_off[l];
    const int64_t vloc = t * 32 + (L & 31);
    if (vloc >= nl) return;
    Parts P = parts_of(bits);
    const uint8_t* src = packed + T * (int64_t)(4 * dp * bits) + (int64_t)kb * 256 * bits;
    uint32_t U[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int wsum = 0;
    for (int p = 0; p < P.n; ++p) {
        const int w = P.w[p], pos = P.pos[p];
        const int per = 8 / w;
        const uint32_t mask = 0x01010101u * ((1u << w) - 1u);
        const uint32_t* s32 = (const uint32_t*)(src + wsum * 256 + L * 4 * w);
        for (int c = 0; c < 8; ++c) U[c] |= ((s32[c / per] >> ((c % per) * w)) & mask) << pos;
        wsum += w;
    }
    const int xr = (bits == 8) ? 0x80 : 0;
    const int h = L >> 5;
    uint8_t* dst = codes + (list_off[l] + vloc) * (int64_t)dp;
    for (int s = 0; s < 2; ++s)
        for (int jj = 0; jj < 16; ++jj) {
            int c = s * 4 + jj / 4, b = jj % 4;
            dst[kb * 64 + s * 32 + h * 16 + jj] = (uint8_t)(((U[c] >> (8 * b)) & 0xFF) ^ xr);
        }
}

hipError_t launch_pack_n(const uint8_t* codes, const int64_t* list_off, const int64_t* tile_off,
                         int64_t nlist, int dp, int bits, int64_t ntiles, uint8_t* packed, hipStream_t st)
{
    int64_t total = ntiles * (dp / 64) * 64;
    if (total == 0) return hipSuccess;
    int th = 256;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((total + th - 1) / th)), dim3(th), 0, st,
                       codes, list_off, tile_off, nlist, dp, bits, ntiles, packed);
    return hipGetLastError();
}

hipError_t launch_unpack_n(const uint8_t* packed, const int64_t* list_off, const int64_t* tile_off,
                           int64_t nlist, int dp, int bits, int64_t ntiles, uint8_t* codes, hipStream_t st)
{
    int64_t total = ntiles * (dp / 64) * 64;
    if (total == 0) return hipSuccess;
    int th = 256;
    hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((total + th - 1) / th)), dim3(th), 0, st,
                       packed, list_off, tile_off, nlist, dp, bits, ntiles, codes);
    return hipGetLastError();
}

}  // namespace erq
