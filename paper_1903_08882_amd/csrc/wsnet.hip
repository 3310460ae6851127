// wsnet.hip -- the learned warm start (include/lws.h): bfloat16 matrix-core
// 3-D convolutions (forward, data gradient, weight gradient), FiLM + SiLU,
// grid-level maps, loss, Adam, and the encoder-decoder that chains them.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16: rows are
// voxels (or, for the weight gradient, (tap, channel) pairs), the reduction
// runs over (tap, input channel) (or over voxels), columns are output
// channels.  A wave owns two 16-row tiles, so every B fragment feeds two
// MFMAs.  Activations are channels-last, so the 8 consecutive reduction
// indices a lane feeds to one MFMA are 8 adjacent channels of one tap: one
// 16-byte load.  The FP32 accumulator tile of a 16x16 MFMA sits in lane l as
// column l % 16, rows 4 (l / 16) + s, s = 0..3; the A and B operands are fed
// with the same (lane, slot) -> k assignment, so the sum over k does not
// depend on the order in which the hardware visits it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lws.h"

namespace lwsk {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) unsigned short u16x8;

constexpr int kThreads = 256;
constexpr int kMaxCout = 64;    // output channels of a forward convolution / weight gradient
constexpr int kMaxCin = 128;    // output channels of a data gradient

// Round to the nearest bfloat16, ties to even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

struct Grid {
    int B, D, H, W;
    uint32_t V;       // D H W
    uint64_t total;   // B V
};

Grid make_grid(lws_grid g) {
    Grid r{g.B, g.D, g.H, g.W, 0, 0};
    r.V = static_cast<uint32_t>(g.D) * g.H * g.W;
    r.total = static_cast<uint64_t>(g.B) * r.V;
    return r;
}

bool grid_ok(lws_grid g) {
    return g.B >= 1 && g.D >= 1 && g.H >= 1 && g.W >= 1 &&
           static_cast<uint64_t>(g.B) * g.D * g.H * g.W < (uint64_t{1} << 40) &&
           static_cast<uint64_t>(g.D) * g.H * g.W < (uint64_t{1} << 31);
}

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }
inline unsigned blocks_for(uint64_t n, unsigned per = kThreads) {
    return static_cast<unsigned>((n + per - 1) / per);
}

// ---------------------------------------------------------------------------
// Convolution forward (also the data gradient, with mirrored packed weights)
// ---------------------------------------------------------------------------
template <int NT, int MT>
__global__ __launch_bounds__(kThreads) void k_conv_fwd(const uint16_t *__restrict__ x, int x_shared, int cin,
                                                       const uint16_t *__restrict__ wp, int kpad, int cout,
                                                       float *__restrict__ z, Grid g) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t tile0 = (static_cast<uint64_t>(blockIdx.x) * 4 + wave) * 16 * MT;
    if (tile0 >= g.total) return;                     // whole wave
    const int r = lane & 15, grp = lane >> 4;
    bool valid[MT];
    uint64_t xbase[MT];
    int px[MT], py[MT], pz[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const uint64_t u = tile0 + 16 * m + r;
        valid[m] = u < g.total;
        xbase[m] = 0;
        px[m] = py[m] = pz[m] = 0;
        if (valid[m]) {
            const uint64_t b = u / g.V;
            const uint32_t v = static_cast<uint32_t>(u - b * g.V);
            px[m] = static_cast<int>(v % g.W);
            const uint32_t q = v / g.W;
            py[m] = static_cast<int>(q % g.H);
            pz[m] = static_cast<int>(q / g.H);
            xbase[m] = x_shared ? 0 : b * g.V;
        }
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    int t = (8 * grp) / cin, ci = 8 * grp - t * cin;
#pragma unroll 4
    for (int k0 = 0; k0 < kpad; k0 += 32) {
        const int k = k0 + 8 * grp;
        bf16x8 a[MT];
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            uint4 av = {0u, 0u, 0u, 0u};
            if (valid[m] && t < 27) {
                const int nz = pz[m] + dz, ny = py[m] + dy, nx = px[m] + dx;
                if (nz >= 0 && nz < g.D && ny >= 0 && ny < g.H && nx >= 0 && nx < g.W) {
                    const uint64_t idx = (xbase[m] + (static_cast<uint64_t>(nz) * g.H + ny) * g.W + nx) * cin + ci;
                    av = *reinterpret_cast<const uint4 *>(x + idx);
                }
            }
            a[m] = __builtin_bit_cast(bf16x8, av);
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const uint4 bv = *reinterpret_cast<const uint4 *>(wp + static_cast<uint64_t>(16 * j + r) * kpad + k);
            const bf16x8 b = __builtin_bit_cast(bf16x8, bv);
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][j], 0, 0, 0);
        }
        ci += 32;
        while (ci >= cin) {
            ci -= cin;
            ++t;
        }
    }
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int co = 16 * j + r;
            if (co >= cout) continue;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const uint64_t uo = tile0 + 16 * m + 4 * grp + s;
                if (uo < g.total) z[uo * cout + co] = acc[m][j][s];
            }
        }
}

// ---------------------------------------------------------------------------
// Convolution forward from an LDS brick (thin inputs): a block computes an
// 8 x 8 x 4 brick of output voxels of one sample.  It first stages the
// 10 x 10 x 6 input brick with its one-voxel halo (zeros outside the grid,
// channels-last, cin <= kBrickCin) in LDS, so every tap of every output voxel
// is a 16-byte LDS read: one global load per input voxel and channel group
// instead of 27 gathers.  Wave w owns output layer z0 + w: four MFMA row
// tiles of 16 voxels (8 along x by 2 along y).
// ---------------------------------------------------------------------------
constexpr int kBrickX = 8, kBrickY = 8, kBrickZ = 4;
constexpr int kHaloX = kBrickX + 2, kHaloY = kBrickY + 2, kHaloZ = kBrickZ + 2;
constexpr int kHaloVox = kHaloX * kHaloY * kHaloZ;
constexpr int kBrickCin = 48;   // 600 voxels x 48 channels x 2 bytes = 57.6 KB of LDS

template <int NT>
__global__ __launch_bounds__(kThreads) void k_conv_fwd_brick(const uint16_t *__restrict__ x, int x_shared, int cin,
                                                             const uint16_t *__restrict__ wp, int kpad, int cout,
                                                             float *__restrict__ z, Grid g, int nbx, int nby) {
    static_assert(kBrickZ * 64 == kThreads, "one wave per output layer");
    extern __shared__ uint4 lds_raw[];
    uint16_t *lx = reinterpret_cast<uint16_t *>(lds_raw);   // [kHaloVox][cin]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int bb = blockIdx.x;
    const int bxi = bb % nbx, byi = (bb / nbx) % nby, bzi = bb / (nbx * nby);
    const int x0 = bxi * kBrickX, y0 = byi * kBrickY, z0 = bzi * kBrickZ;
    const uint32_t b = blockIdx.y;
    const uint64_t xb = x_shared ? 0 : static_cast<uint64_t>(b) * g.V;
    const int cg = cin / 8;
    for (int e = threadIdx.x; e < kHaloVox * cg; e += kThreads) {
        const int hv = e / cg, c8 = e - hv * cg;
        const int hx = hv % kHaloX, hy = (hv / kHaloX) % kHaloY, hz = hv / (kHaloX * kHaloY);
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
        uint4 val = {0u, 0u, 0u, 0u};
        if (gx >= 0 && gx < g.W && gy >= 0 && gy < g.H && gz >= 0 && gz < g.D)
            val = *reinterpret_cast<const uint4 *>(
                x + (xb + (static_cast<uint64_t>(gz) * g.H + gy) * g.W + gx) * cin + 8 * c8);
        *reinterpret_cast<uint4 *>(lx + hv * cin + 8 * c8) = val;
    }
    __syncthreads();
    const int r = lane & 15, grp = lane >> 4;
    // halo index of this lane's output voxel in tile m, before the tap offset
    int hbase[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
        hbase[m] = ((wave + 1) * kHaloY + (2 * m + r / 8 + 1)) * kHaloX + (r % 8 + 1);
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    int t = (8 * grp) / cin, ci = 8 * grp - t * cin;
#pragma unroll 4
    for (int k0 = 0; k0 < kpad; k0 += 32) {
        const int k = k0 + 8 * grp;
        const int off = ((t / 9 - 1) * kHaloY + ((t / 3) % 3 - 1)) * kHaloX + (t % 3 - 1);
        bf16x8 a[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            uint4 av = {0u, 0u, 0u, 0u};
            if (t < 27) av = *reinterpret_cast<const uint4 *>(lx + (hbase[m] + off) * cin + ci);
            a[m] = __builtin_bit_cast(bf16x8, av);
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const uint4 bv = *reinterpret_cast<const uint4 *>(wp + static_cast<uint64_t>(16 * j + r) * kpad + k);
            const bf16x8 bw = __builtin_bit_cast(bf16x8, bv);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bw, acc[m][j], 0, 0, 0);
        }
        ci += 32;
        while (ci >= cin) {
            ci -= cin;
            ++t;
        }
    }
    const int oz = z0 + wave;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int row = 4 * grp + s4;
            const int ox = x0 + row % 8, oy = y0 + 2 * m + row / 8;
            if (ox >= g.W || oy >= g.H || oz >= g.D) continue;
            const uint64_t vo = static_cast<uint64_t>(b) * g.V + (static_cast<uint64_t>(oz) * g.H + oy) * g.W + ox;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int co = 16 * j + r;
                if (co < cout) z[vo * cout + co] = acc[m][j][s4];
            }
        }
}

// ---------------------------------------------------------------------------
// Weight gradient: rows m = t cin + ci, columns co, reduction over voxels in
// chunks (blockIdx.y); partial tiles go to work[chunk][m][co].  A wave owns MT
// row tiles, so each dz fragment feeds MT MFMAs; voxel coordinates advance
// incrementally (no divisions in the loop).
// ---------------------------------------------------------------------------
template <int NT, int MT>
__global__ __launch_bounds__(kThreads) void k_conv_wgrad(const uint16_t *__restrict__ x, int x_shared, int cin,
                                                         const uint16_t *__restrict__ dz, int cout,
                                                         float *__restrict__ work, Grid g, uint64_t chunk) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mrows = 27 * cin;
    const int m0 = (blockIdx.x * 4 + wave) * 16 * MT;
    if (m0 >= mrows) return;                          // whole wave
    const int r = lane & 15, grp = lane >> 4;
    int ci[MT], oz[MT], oy[MT], ox[MT];
    bool mv[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int m = m0 + 16 * t + r;
        mv[t] = m < mrows;
        const int tap = mv[t] ? m / cin : 13;
        ci[t] = mv[t] ? m - tap * cin : 0;
        oz[t] = tap / 9 - 1;
        oy[t] = (tap / 3) % 3 - 1;
        ox[t] = tap % 3 - 1;
    }
    const uint64_t u0 = static_cast<uint64_t>(blockIdx.y) * chunk;
    const uint64_t u1 = u0 + chunk < g.total ? u0 + chunk : g.total;
    // coordinates of this lane's first voxel, u0 + 8 grp
    int px, py, pz;
    uint32_t pb;
    {
        const uint64_t ul = u0 + 8 * grp;
        pb = static_cast<uint32_t>(ul / g.V);
        const uint32_t v = static_cast<uint32_t>(ul - static_cast<uint64_t>(pb) * g.V);
        px = static_cast<int>(v % g.W);
        const uint32_t q = v / g.W;
        py = static_cast<int>(q % g.H);
        pz = static_cast<int>(q / g.H);
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (uint64_t ub = u0; ub < u1; ub += 32) {
        u16x8 av[MT], bv[NT];
        int xs = px, ys = py, zs = pz;
        uint32_t bs = pb;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const uint64_t u = ub + 8 * grp + s;
            const bool valid = u < u1;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int co = 16 * j + r;
                bv[j][s] = (valid && co < cout) ? dz[u * cout + co] : uint16_t(0);
            }
            const uint64_t xb = x_shared ? 0 : static_cast<uint64_t>(bs) * g.V;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const int nz = zs + oz[t], ny = ys + oy[t], nx = xs + ox[t];
                uint16_t val = 0;
                if (valid && mv[t] && nz >= 0 && nz < g.D && ny >= 0 && ny < g.H && nx >= 0 && nx < g.W)
                    val = x[(xb + (static_cast<uint64_t>(nz) * g.H + ny) * g.W + nx) * cin + ci[t]];
                av[t][s] = val;
            }
            if (++xs == g.W) {
                xs = 0;
                if (++ys == g.H) {
                    ys = 0;
                    if (++zs == g.D) {
                        zs = 0;
                        ++bs;
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[t]),
                                                                     __builtin_bit_cast(bf16x8, bv[j]), acc[t][j],
                                                                     0, 0, 0);
        // the lane's first voxel moves on by 32
        px += 32;
        while (px >= g.W) {
            px -= g.W;
            if (++py == g.H) {
                py = 0;
                if (++pz == g.D) {
                    pz = 0;
                    ++pb;
                }
            }
        }
    }
    float *out = work + static_cast<uint64_t>(blockIdx.y) * mrows * cout;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int co = 16 * j + r;
            if (co >= cout) continue;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int mo = m0 + 16 * t + 4 * grp + s;
                if (mo < mrows) out[static_cast<uint64_t>(mo) * cout + co] = acc[t][j][s];
            }
        }
}

// Weight gradient with LDS staging (cin a multiple of 8).  A block owns
// kWgRows rows (4 waves x 2 tiles of 16) and one voxel chunk.  For each group
// of 32 voxels it stages, transposed so that 8 consecutive voxels of one
// channel are 16 contiguous bytes, the dz tile as [co][32] and, for every tap
// its rows touch, the shifted input x[v + off_t] as [tap][cin][32] (zero where
// the neighbour leaves the grid); every MFMA operand is then one 16-byte LDS
// read, and the global traffic is coalesced 16-byte loads.
constexpr int kWgRows = 128;
constexpr int kWgVox = 32;   // voxels staged per barrier (whole MFMA k-steps of 32; 64 was slower for wide layers)

int wg_taps(int cin) { return std::min(27, (kWgRows + cin - 1) / cin + 1); }

// Four consecutive voxels' 16-byte loads (8 channels each) written to LDS as
// eight channel rows of four voxels: one 8-byte store per channel instead of
// four 2-byte ones.
__device__ __forceinline__ void store_quad_transposed(uint16_t *dst, int ld, const uint4 (&val)[4]) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t w0 = val[0][d], w1 = val[1][d], w2 = val[2][d], w3 = val[3][d];
        uint2 lo, hi;   // channels 2d and 2d + 1
        lo.x = (w0 & 0xffffu) | (w1 << 16);
        lo.y = (w2 & 0xffffu) | (w3 << 16);
        hi.x = (w0 >> 16) | (w1 & 0xffff0000u);
        hi.y = (w2 >> 16) | (w3 & 0xffff0000u);
        *reinterpret_cast<uint2 *>(dst + (2 * d) * ld) = lo;
        *reinterpret_cast<uint2 *>(dst + (2 * d + 1) * ld) = hi;
    }
}

// Voxel coordinates, advanced one voxel at a time in the order of the
// channels-last index (x fastest, then y, z, batch).
struct Vox {
    int x, y, z;
    uint32_t b;
};
__device__ __forceinline__ Vox vox_of(uint32_t u, const Grid &g) {
    Vox p;
    p.b = u / g.V;
    const uint32_t v = u - p.b * g.V, q = v / g.W;
    p.x = static_cast<int>(v - q * g.W);
    p.y = static_cast<int>(q % g.H);
    p.z = static_cast<int>(q / g.H);
    return p;
}
__device__ __forceinline__ Vox vox_next(Vox p, const Grid &g) {
    if (++p.x == g.W) {
        p.x = 0;
        if (++p.y == g.H) {
            p.y = 0;
            if (++p.z == g.D) {
                p.z = 0;
                ++p.b;
            }
        }
    }
    return p;
}

template <int NT, int GV>
__global__ __launch_bounds__(kThreads) void k_conv_wgrad_lds(const uint16_t *__restrict__ x, int x_shared, int cin,
                                                             const uint16_t *__restrict__ dz, int cout,
                                                             float *__restrict__ work, Grid g, uint64_t chunk) {
    constexpr int NQ = GV / 4;   // voxel quads per group
    static_assert(GV % 32 == 0 && kThreads % NQ == 0, "voxel groups are whole MFMA k-steps");
    extern __shared__ uint4 lds_raw[];
    uint16_t *ldz = reinterpret_cast<uint16_t *>(lds_raw);   // [16 NT][GV]
    uint16_t *lx = ldz + 16 * NT * GV;                       // [taps][cin][GV]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mrows = 27 * cin;
    const int m0 = blockIdx.x * kWgRows;
    const int t_lo = m0 / cin;
    const int t_hi = min(26, (min(m0 + kWgRows, mrows) - 1) / cin);
    const int ntap = t_hi - t_lo + 1;
    const int cgroups = cin / 8;
    const int r = lane & 15, grp = lane >> 4;
    bool mv[2];
    int lrow[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int m = m0 + (wave * 2 + q) * 16 + r;
        mv[q] = m < mrows;
        const int t = mv[q] ? m / cin : t_lo;
        lrow[q] = (t - t_lo) * cin + (mv[q] ? m - t * cin : 0);
    }
    f32x4 acc[2][NT];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[q][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint32_t u0 = blockIdx.y * static_cast<uint32_t>(chunk);
    const uint32_t u1 = u0 + chunk < g.total ? static_cast<uint32_t>(u0 + chunk) : static_cast<uint32_t>(g.total);
    // every element this thread stages belongs to voxel quad vq of the group
    const int vq = threadIdx.x % NQ;
    for (uint32_t ub = u0; ub < u1; ub += GV) {
        const uint32_t uq = ub + 4 * vq;
        Vox p[4];
        p[0] = vox_of(uq, g);
#pragma unroll
        for (int k = 1; k < 4; ++k) p[k] = vox_next(p[k - 1], g);
        __syncthreads();                                  // the previous group's reads are done
        for (int e = threadIdx.x; e < 2 * NT * NQ; e += kThreads) {
            const int cg = e / NQ;
            uint4 val[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                val[k] = uint4{0u, 0u, 0u, 0u};
                if (uq + k < u1 && 8 * cg < cout)
                    val[k] = *reinterpret_cast<const uint4 *>(dz + static_cast<uint64_t>(uq + k) * cout + 8 * cg);
            }
            store_quad_transposed(ldz + (8 * cg) * GV + 4 * vq, GV, val);
        }
        for (int e = threadIdx.x; e < ntap * cgroups * NQ; e += kThreads) {
            const int rest = e / NQ;
            const int cg = rest % cgroups, tt = rest / cgroups;
            const int t = t_lo + tt;
            const int oz = t / 9 - 1, oy = (t / 3) % 3 - 1, ox = t % 3 - 1;
            uint4 val[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                val[k] = uint4{0u, 0u, 0u, 0u};
                const int nz = p[k].z + oz, ny = p[k].y + oy, nx = p[k].x + ox;
                if (uq + k < u1 && nz >= 0 && nz < g.D && ny >= 0 && ny < g.H && nx >= 0 && nx < g.W) {
                    const uint64_t xb = x_shared ? 0 : static_cast<uint64_t>(p[k].b) * g.V;
                    val[k] = *reinterpret_cast<const uint4 *>(
                        x + (xb + (static_cast<uint64_t>(nz) * g.H + ny) * g.W + nx) * cin + 8 * cg);
                }
            }
            store_quad_transposed(lx + (tt * cin + 8 * cg) * GV + 4 * vq, GV, val);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GV / 32; ++ks) {
            bf16x8 bfr[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j)
                bfr[j] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(ldz + (16 * j + r) * GV + 32 * ks + 8 * grp));
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                uint4 av = {0u, 0u, 0u, 0u};
                if (mv[q]) av = *reinterpret_cast<const uint4 *>(lx + lrow[q] * GV + 32 * ks + 8 * grp);
                const bf16x8 a = __builtin_bit_cast(bf16x8, av);
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[j], acc[q][j], 0, 0, 0);
            }
        }
    }
    float *out = work + static_cast<uint64_t>(blockIdx.y) * mrows * cout;
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int co = 16 * j + r;
            if (co >= cout) continue;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int mo = m0 + (wave * 2 + q) * 16 + 4 * grp + s4;
                if (mo < mrows) out[static_cast<uint64_t>(mo) * cout + co] = acc[q][j][s4];
            }
        }
}

// Sum of the per-chunk partial weight gradients, in a fixed order: a block
// takes 32 outputs, its 8 slices of 32 threads add every 8th chunk in FP64,
// and the 8 slice sums are added in slice order.
constexpr int kSumOut = 32, kSumSlices = kThreads / kSumOut;
__global__ __launch_bounds__(kThreads) void k_sum_chunks(const float *__restrict__ work, int nchunks, uint64_t n,
                                                         float *__restrict__ out) {
    __shared__ double part[kSumSlices][kSumOut];
    const int o = threadIdx.x % kSumOut, sl = threadIdx.x / kSumOut;
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kSumOut + o;
    double s = 0.0;
    if (i < n)
        for (int c = sl; c < nchunks; c += kSumSlices) s += work[static_cast<uint64_t>(c) * n + i];
    part[sl][o] = s;
    __syncthreads();
    if (sl == 0 && i < n) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kSumSlices; ++k) t += part[k][o];
        out[i] = static_cast<float>(t);
    }
}

// Voxels per chunk of the weight gradient: enough chunks that the launch has
// about kWgBlocks blocks (each block waits on a gather per voxel group, so
// occupancy is what hides the latency; 4096 ran the training shapes 1.1-1.9x
// faster than 512, 8192 no better), at least kWgVox * 16 voxels each.
constexpr uint64_t kWgBlocks = 4096;
uint64_t wgrad_chunk(uint64_t total, int cin) {
    const uint64_t rowblocks = (27 * static_cast<uint64_t>(cin) + kWgRows - 1) / kWgRows;
    const uint64_t want = std::max<uint64_t>(1, kWgBlocks / rowblocks);
    uint64_t c = (total + want - 1) / want;
    c = (c + kWgVox - 1) / kWgVox * kWgVox;
    return std::max<uint64_t>(c, 16 * kWgVox);
}

// ---------------------------------------------------------------------------
// Weight packing
// ---------------------------------------------------------------------------
__global__ void k_pack(const float *__restrict__ w, int cin, int cout, int dgrad, int rows, int kpad,
                       uint16_t *__restrict__ out) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<uint64_t>(rows) * kpad) return;
    const int row = static_cast<int>(i / kpad), k = static_cast<int>(i - static_cast<uint64_t>(row) * kpad);
    float v = 0.f;
    if (!dgrad) {   // row co, column t cin + ci: w[t][ci][co] = w[k cout + co]
        if (row < cout && k < 27 * cin) v = w[static_cast<uint64_t>(k) * cout + row];
    } else {        // row ci, column t cout + co: w[26 - t][ci][co]
        if (row < cin && k < 27 * cout) {
            const int t = k / cout, co = k - t * cout;
            v = w[(static_cast<uint64_t>(26 - t) * cin + row) * cout + co];
        }
    }
    out[i] = to_bf16(v);
}

void pack_dims(int cin, int cout, int dgrad, int *rows, int *kpad) {
    if (!dgrad) {
        *rows = round_up(cout, 16);
        *kpad = round_up(27 * cin, 32);
    } else {
        *rows = round_up(cin, 16);
        *kpad = round_up(27 * cout, 32);
    }
}

// ---------------------------------------------------------------------------
// Pointwise and level maps
// ---------------------------------------------------------------------------
__global__ void k_features(int M, uint16_t *__restrict__ out) {
    const uint32_t n = static_cast<uint32_t>(M) * M * M;
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int ix = v % M, iy = (v / M) % M, iz = v / (M * M);
    const float x = (ix + 0.5f) / M, y = (iy + 0.5f) / M, z = (iz + 0.5f) / M;
    const float d = fminf(fminf(fminf(x, 1.f - x), fminf(y, 1.f - y)), fminf(z, 1.f - z));
    const float f[8] = {2 * x - 1, 2 * y - 1, 2 * z - 1, (2 * x - 1) * (2 * x - 1), (2 * y - 1) * (2 * y - 1),
                        (2 * z - 1) * (2 * z - 1), d, 1.f};
    for (int c = 0; c < 8; ++c) out[static_cast<uint64_t>(v) * 8 + c] = to_bf16(f[c]);
}

// scale[b][c] = 1 + Gw[c] . cond[b] + Gb[c]; shift[b][c] = Bw[c] . cond[b] + Bb[c]
__global__ void k_film_params(const float *__restrict__ gw, const float *__restrict__ gb,
                              const float *__restrict__ bw, const float *__restrict__ bb, int C,
                              const float *__restrict__ cond, int B, float *__restrict__ scale,
                              float *__restrict__ shift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * C) return;
    const int b = i / C, c = i - b * C;
    const float c0 = cond[2 * b], c1 = cond[2 * b + 1];
    scale[i] = 1.f + gw[2 * c] * c0 + gw[2 * c + 1] * c1 + gb[c];
    shift[i] = bw[2 * c] * c0 + bw[2 * c + 1] * c1 + bb[c];
}

__device__ __forceinline__ float sigm(float y) { return 1.f / (1.f + __expf(-y)); }

// I: the index type, 32-bit whenever every index of the launch fits (the
// divisions below are then 32-bit ones, several times cheaper than 64-bit)
template <class I>
__global__ void k_film_act(const float *__restrict__ z, int C, Grid g, const float *__restrict__ scale,
                           const float *__restrict__ shift, uint16_t *__restrict__ out, int ostride, int ooff) {
    const I e = static_cast<I>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<I>(g.total) * C) return;
    const I u = e / C;
    const int c = static_cast<int>(e - u * C);
    const int b = static_cast<int>(u / g.V);
    const float y = z[e] * scale[b * C + c] + shift[b * C + c];
    out[u * ostride + ooff + c] = to_bf16(y * sigm(y));
}

// dY = dA silu'(y); dZ = dY scale (bfloat16); per-block sums of dY z and dY
// per channel into part[(b nbx + block)][2][C].  Needs C | kThreads.
__global__ __launch_bounds__(kThreads) void k_film_bwd(const float *__restrict__ da, int dstride, int doff,
                                                       const float *__restrict__ z, int C, Grid g,
                                                       const float *__restrict__ scale,
                                                       const float *__restrict__ shift,
                                                       uint16_t *__restrict__ dzb, double *__restrict__ part) {
    __shared__ double s1[kThreads], s2[kThreads];
    const int b = blockIdx.y;
    const uint64_t n = static_cast<uint64_t>(g.V) * C;
    const int c = threadIdx.x % C;
    const float sc = scale[b * C + c], sh = shift[b * C + c];
    double a1 = 0.0, a2 = 0.0;
    // the stride is a multiple of C, so the voxel advances by stride / C
    const uint64_t step = static_cast<uint64_t>(kThreads) * gridDim.x;
    uint64_t e = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
    uint64_t u = static_cast<uint64_t>(b) * g.V + e / C;
    for (; e < n; e += step, u += step / C) {
        const float zz = z[u * C + c];
        const float y = zz * sc + sh;
        const float s = sigm(y);
        const float dy = da[u * dstride + doff + c] * (s * (1.f + y * (1.f - s)));
        dzb[u * C + c] = to_bf16(dy * sc);
        a1 += static_cast<double>(dy) * zz;
        a2 += dy;
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    if (threadIdx.x < C) {
        double t1 = 0.0, t2 = 0.0;
        for (int k = threadIdx.x; k < kThreads; k += C) {
            t1 += s1[k];
            t2 += s2[k];
        }
        double *p = part + (static_cast<uint64_t>(b) * gridDim.x + blockIdx.x) * 2 * C;
        p[threadIdx.x] = t1;
        p[C + threadIdx.x] = t2;
    }
}

// Per-sample totals of the per-block sums: sums[b][2C] (fixed order).
__global__ void k_film_sums(const double *__restrict__ part, int nbx, int C, double *__restrict__ sums) {
    const int b = blockIdx.x, t = threadIdx.x;
    if (t >= 2 * C) return;
    double acc = 0.0;
    for (int k = 0; k < nbx; ++k) acc += part[(static_cast<uint64_t>(b) * nbx + k) * 2 * C + t];
    sums[static_cast<uint64_t>(b) * 2 * C + t] = acc;
}

// FiLM parameter gradients from the per-sample totals (fixed order).
__global__ void k_film_grads(const double *__restrict__ sums, int B, int C, const float *__restrict__ cond,
                             float *__restrict__ ggw, float *__restrict__ ggb, float *__restrict__ gbw,
                             float *__restrict__ gbb) {
    const int c = threadIdx.x;
    if (c >= C) return;
    double gw0 = 0, gw1 = 0, gb = 0, bw0 = 0, bw1 = 0, bbs = 0;
    for (int b = 0; b < B; ++b) {
        const double dsc = sums[static_cast<uint64_t>(b) * 2 * C + c];
        const double dsh = sums[static_cast<uint64_t>(b) * 2 * C + C + c];
        gw0 += dsc * cond[2 * b];
        gw1 += dsc * cond[2 * b + 1];
        gb += dsc;
        bw0 += dsh * cond[2 * b];
        bw1 += dsh * cond[2 * b + 1];
        bbs += dsh;
    }
    ggw[2 * c] = static_cast<float>(gw0);
    ggw[2 * c + 1] = static_cast<float>(gw1);
    ggb[c] = static_cast<float>(gb);
    gbw[2 * c] = static_cast<float>(bw0);
    gbw[2 * c + 1] = static_cast<float>(bw1);
    gbb[c] = static_cast<float>(bbs);
}

// coarse (i, j, k) = fine (2i, 2j, 2k); fine grid n^3 per sample, coarse (n+1)/2
__global__ void k_restrict(const uint16_t *__restrict__ in, int istride, int ioff, int C, int nf, int B,
                           uint16_t *__restrict__ out) {
    const int nc = (nf + 1) / 2;
    const uint64_t Vc = static_cast<uint64_t>(nc) * nc * nc, Vf = static_cast<uint64_t>(nf) * nf * nf;
    const uint64_t e = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= B * Vc * C) return;
    const uint64_t uc = e / C;
    const int c = static_cast<int>(e - uc * C);
    const uint64_t b = uc / Vc;
    const uint64_t v = uc - b * Vc;
    const uint64_t i = v % nc, j = (v / nc) % nc, k = v / (static_cast<uint64_t>(nc) * nc);
    const uint64_t f = b * Vf + ((2 * k) * nf + 2 * j) * nf + 2 * i;
    out[e] = in[f * istride + ioff + c];
}

__global__ void k_restrict_adj_add(const float *__restrict__ gc, int C, int nf, int B, float *__restrict__ out,
                                   int ostride, int ooff) {
    const int nc = (nf + 1) / 2;
    const uint64_t Vc = static_cast<uint64_t>(nc) * nc * nc, Vf = static_cast<uint64_t>(nf) * nf * nf;
    const uint64_t e = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= B * Vc * C) return;
    const uint64_t uc = e / C;
    const int c = static_cast<int>(e - uc * C);
    const uint64_t b = uc / Vc;
    const uint64_t v = uc - b * Vc;
    const uint64_t i = v % nc, j = (v / nc) % nc, k = v / (static_cast<uint64_t>(nc) * nc);
    const uint64_t f = b * Vf + ((2 * k) * nf + 2 * j) * nf + 2 * i;
    out[f * ostride + ooff + c] += gc[e];
}

// fine node x of 2n - 1: coarse x/2 (even) or the mean of x/2 and x/2 + 1 (odd)
template <class I>
__global__ void k_prolong(const uint16_t *__restrict__ in, int C, int nc, int B, uint16_t *__restrict__ out,
                          int ostride, int ooff) {
    const int nf = 2 * nc - 1;
    const I Vc = static_cast<I>(nc) * nc * nc, Vf = static_cast<I>(nf) * nf * nf;
    const I e = static_cast<I>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= B * Vf * C) return;
    const I uf = e / C;
    const int c = static_cast<int>(e - uf * C);
    const I b = uf / Vf;
    const I v = uf - b * Vf;
    const int x = static_cast<int>(v % nf), y = static_cast<int>((v / nf) % nf),
              z = static_cast<int>(v / (static_cast<I>(nf) * nf));
    const int xo = x & 1, yo = y & 1, zo = z & 1;
    const float w = (xo ? 0.5f : 1.f) * (yo ? 0.5f : 1.f) * (zo ? 0.5f : 1.f);
    float s = 0.f;
    for (int dz = 0; dz <= zo; ++dz)
        for (int dy = 0; dy <= yo; ++dy)
            for (int dx = 0; dx <= xo; ++dx) {
                const I cv = ((static_cast<I>(z / 2 + dz) * nc) + (y / 2 + dy)) * nc + (x / 2 + dx);
                s += from_bf16(in[(b * Vc + cv) * C + c]);
            }
    out[uf * ostride + ooff + c] = to_bf16(w * s);
}

// adjoint of k_prolong: coarse i collects fine 2i (1) and 2i -/+ 1 (1/2) per axis
template <class I>
__global__ void k_prolong_adj(const float *__restrict__ gf, int gstride, int goff, int C, int nc, int B,
                              float *__restrict__ out) {
    const int nf = 2 * nc - 1;
    const I Vc = static_cast<I>(nc) * nc * nc, Vf = static_cast<I>(nf) * nf * nf;
    const I e = static_cast<I>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= B * Vc * C) return;
    const I uc = e / C;
    const int c = static_cast<int>(e - uc * C);
    const I b = uc / Vc;
    const I v = uc - b * Vc;
    const int i = static_cast<int>(v % nc), j = static_cast<int>((v / nc) % nc),
              k = static_cast<int>(v / (static_cast<I>(nc) * nc));
    float s = 0.f;
    for (int dz = -1; dz <= 1; ++dz) {
        const int fz = 2 * k + dz;
        if (fz < 0 || fz >= nf) continue;
        const float wz = dz ? 0.5f : 1.f;
        for (int dy = -1; dy <= 1; ++dy) {
            const int fy = 2 * j + dy;
            if (fy < 0 || fy >= nf) continue;
            const float wy = dy ? 0.5f : 1.f;
            for (int dx = -1; dx <= 1; ++dx) {
                const int fx = 2 * i + dx;
                if (fx < 0 || fx >= nf) continue;
                const float wx = dx ? 0.5f : 1.f;
                const I f = b * Vf + (static_cast<I>(fz) * nf + fy) * nf + fx;
                s += wz * wy * wx * gf[f * gstride + goff + c];
            }
        }
    }
    out[e] = s;
}

__global__ void k_add_bias(float *__restrict__ z, int C, uint64_t total, const float *__restrict__ bias) {
    const uint64_t e = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total * C) return;
    z[e] += bias[e % C];
}

// Loss over the 4 field channels of out [B V][8] against target [B][4][V]
// (times scale[b][ch]); dout = 2 (out - target) / n in FP32 and bfloat16,
// zero for channels 4..7; per-block sums of squares.
__global__ __launch_bounds__(kThreads) void k_mse(const float *__restrict__ out, const float *__restrict__ target,
                                                  const float *__restrict__ scale, Grid g,
                                                  float *__restrict__ dout, uint16_t *__restrict__ doutb,
                                                  double *__restrict__ part) {
    __shared__ double red[kThreads];
    const uint64_t u = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
    double ss = 0.0;
    if (u < g.total) {
        const uint64_t b = u / g.V, v = u - b * g.V;
        const float inv_n = 2.f / static_cast<float>(g.total * 4);
        for (int c = 0; c < 8; ++c) {
            float d = 0.f;
            if (c < 4) {
                const float diff = out[u * 8 + c] - scale[b * 4 + c] * target[(b * 4 + c) * g.V + v];
                ss += static_cast<double>(diff) * diff;
                d = inv_n * diff;
            }
            dout[u * 8 + c] = d;
            doutb[u * 8 + c] = to_bf16(d);
        }
    }
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One block: each thread sums a fixed strided subset, then a fixed tree.
__global__ __launch_bounds__(kThreads) void k_sum_doubles(const double *__restrict__ part, int n, double scale,
                                                          double *__restrict__ out) {
    __shared__ double red[kThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = kThreads / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Per-channel sums of a [rows][C] FP32 array: per-block partials, then a fixed-order total.
__global__ __launch_bounds__(kThreads) void k_chan_partial(const float *__restrict__ a, int C, uint64_t rows,
                                                           double *__restrict__ part) {
    __shared__ double red[kThreads];
    const int c = threadIdx.x % C;
    double s = 0.0;
    for (uint64_t e = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x; e < rows * C;
         e += static_cast<uint64_t>(kThreads) * gridDim.x)
        s += a[e];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < C) {
        double t = 0.0;
        for (int k = threadIdx.x; k < kThreads; k += C) t += red[k];
        part[static_cast<uint64_t>(blockIdx.x) * C + threadIdx.x] = t;
    }
    (void)c;
}

__global__ void k_chan_final(const double *__restrict__ part, int nb, int C, float *__restrict__ out) {
    const int c = threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[static_cast<uint64_t>(k) * C + c];
    out[c] = static_cast<float>(s);
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, uint64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Per-axis sample of a node-centred grid of M nodes at position p in (0, 1):
// indices i0, i1 in {-1 (low wall), 0..M-1, M (high wall)} and the weight of i1.
__device__ __forceinline__ void axis_samples(double p, int M, int *i0, int *i1, double *w) {
    const double s = p * M - 0.5;
    if (s < 0.0) {
        *i0 = -1;
        *i1 = 0;
        *w = 2.0 * s + 1.0;
    } else if (s >= M - 1) {
        *i0 = M - 1;
        *i1 = M;
        *w = 2.0 * (s - (M - 1));
    } else {
        const int j = static_cast<int>(s);
        *i0 = j;
        *i1 = j + 1;
        *w = s - j;
    }
}

// Anchored trilinear interpolation of the prediction (u/U, v/U, w/U, T*) at
// lattice node (ix, iy, iz) of N^3.
__device__ void interp_at(const float *__restrict__ pred, int M, int ld, int N, int iso_axis, int ix, int iy,
                          int iz, double acc[4]) {
    int a0[3], a1[3];
    double w[3];
    axis_samples((ix + 0.5) / N, M, &a0[0], &a1[0], &w[0]);
    axis_samples((iy + 0.5) / N, M, &a0[1], &a1[1], &w[1]);
    axis_samples((iz + 0.5) / N, M, &a0[2], &a1[2], &w[2]);
    for (int c = 0; c < 4; ++c) acc[c] = 0.0;
    for (int corner = 0; corner < 8; ++corner) {
        int idx[3];
        double wt = 1.0;
        bool wall = false;
        for (int a = 0; a < 3; ++a) {
            const int hi = (corner >> a) & 1;
            idx[a] = hi ? a1[a] : a0[a];
            wt *= hi ? w[a] : 1.0 - w[a];
            wall |= idx[a] < 0 || idx[a] >= M;
        }
        if (wt == 0.0) continue;
        // velocity: 0 on any wall
        if (!wall) {
            const uint64_t v = (static_cast<uint64_t>(idx[2]) * M + idx[1]) * M + idx[0];
            for (int c = 0; c < 3; ++c) acc[c] += wt * pred[v * ld + c];
        }
        // temperature: the isothermal wall value, else the nearest node
        double T;
        if (idx[iso_axis] < 0) {
            T = 0.5;
        } else if (idx[iso_axis] >= M) {
            T = -0.5;
        } else {
            int cl[3];
            for (int a = 0; a < 3; ++a) cl[a] = idx[a] < 0 ? 0 : (idx[a] >= M ? M - 1 : idx[a]);
            T = pred[((static_cast<uint64_t>(cl[2]) * M + cl[1]) * M + cl[0]) * ld + 3];
        }
        acc[3] += wt * T;
    }
}

// With sym (side-heated cell only), the average over the cell's symmetry
// group: the half-turn about the y axis through the centre with T* -> -T*
// ((x, z) -> (1 - x, 1 - z), (u, w) -> (-u, -w)) and the mirror y -> 1 - y
// (v -> -v).  Lattice nodes map onto lattice nodes.
__global__ void k_upsample(const float *__restrict__ pred, int M, int ld, int N, int iso_axis, int sym, double U,
                           double T_hot, double T_cold, double *__restrict__ out) {
    const uint64_t V = static_cast<uint64_t>(N) * N * N;
    const uint64_t n = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= V) return;
    const int ix = static_cast<int>(n % N), iy = static_cast<int>((n / N) % N),
              iz = static_cast<int>(n / (static_cast<uint64_t>(N) * N));
    double acc[4];
    interp_at(pred, M, ld, N, iso_axis, ix, iy, iz, acc);
    if (sym) {
        double t[4];
        // half-turn about y: (u, v, w, T) -> (-u, v, -w, -T) at (N-1-ix, iy, N-1-iz)
        interp_at(pred, M, ld, N, iso_axis, N - 1 - ix, iy, N - 1 - iz, t);
        acc[0] -= t[0];
        acc[1] += t[1];
        acc[2] -= t[2];
        acc[3] -= t[3];
        // mirror in y: (u, v, w, T) -> (u, -v, w, T) at (ix, N-1-iy, iz)
        interp_at(pred, M, ld, N, iso_axis, ix, N - 1 - iy, iz, t);
        acc[0] += t[0];
        acc[1] -= t[1];
        acc[2] += t[2];
        acc[3] += t[3];
        // both
        interp_at(pred, M, ld, N, iso_axis, N - 1 - ix, N - 1 - iy, N - 1 - iz, t);
        acc[0] -= t[0];
        acc[1] -= t[1];
        acc[2] -= t[2];
        acc[3] -= t[3];
        for (int c = 0; c < 4; ++c) acc[c] *= 0.25;
    }
    const double Tm = 0.5 * (T_hot + T_cold), dT = T_hot - T_cold;
    out[n] = U * acc[0];
    out[V + n] = U * acc[1];
    out[2 * V + n] = U * acc[2];
    out[3 * V + n] = Tm + dT * acc[3];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int MT>
hipError_t conv_fwd_mt(const uint16_t *x, int x_shared, int cin, const uint16_t *wp, int kpad, int cout, float *z,
                       const Grid &g, hipStream_t s) {
    const unsigned nb = static_cast<unsigned>((g.total + 64 * MT - 1) / (64 * MT));
    const int nt = (cout + 15) / 16;
    switch (nt) {
#define LWS_CASE(K) \
    case K: k_conv_fwd<K, MT><<<nb, kThreads, 0, s>>>(x, x_shared, cin, wp, kpad, cout, z, g); break;
        LWS_CASE(1) LWS_CASE(2) LWS_CASE(3) LWS_CASE(4) LWS_CASE(5) LWS_CASE(6) LWS_CASE(7) LWS_CASE(8)
#undef LWS_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Four 16-voxel tiles per wave keep four gathers in flight per k-step: 1.1-1.4x
// over two at the training shapes with up to 64 input channels; with more, the
// longer reduction already hides the latency and two tiles are as fast.
hipError_t conv_fwd(const uint16_t *x, int x_shared, int cin, const uint16_t *wp, int kpad, int cout, float *z,
                    const Grid &g, hipStream_t s) {
    if (cin % 8 == 0 && cin <= kBrickCin && g.B <= 65535) {
        const int nbx = (g.W + kBrickX - 1) / kBrickX, nby = (g.H + kBrickY - 1) / kBrickY,
                  nbz = (g.D + kBrickZ - 1) / kBrickZ;
        const dim3 grid(static_cast<unsigned>(nbx * nby * nbz), static_cast<unsigned>(g.B));
        const size_t lds = static_cast<size_t>(kHaloVox) * cin * sizeof(uint16_t);
        switch ((cout + 15) / 16) {
#define LWS_CASE(K) \
    case K: k_conv_fwd_brick<K><<<grid, kThreads, lds, s>>>(x, x_shared, cin, wp, kpad, cout, z, g, nbx, nby); break;
            LWS_CASE(1) LWS_CASE(2) LWS_CASE(3) LWS_CASE(4) LWS_CASE(5) LWS_CASE(6) LWS_CASE(7) LWS_CASE(8)
#undef LWS_CASE
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    return cin <= 64 ? conv_fwd_mt<4>(x, x_shared, cin, wp, kpad, cout, z, g, s)
                     : conv_fwd_mt<2>(x, x_shared, cin, wp, kpad, cout, z, g, s);
}

hipError_t conv_wgrad(const uint16_t *x, int x_shared, int cin, const uint16_t *dz, int cout, float *dw,
                      const Grid &g, float *work, uint64_t chunk, hipStream_t s) {
    const unsigned nchunks = static_cast<unsigned>((g.total + chunk - 1) / chunk);
    const int mrows = 27 * cin;
    if (cin % 8 == 0 && cout % 8 == 0 && g.total + chunk < (uint64_t{1} << 32)) {   // 32-bit voxel indices
        const dim3 grid(static_cast<unsigned>((mrows + kWgRows - 1) / kWgRows), nchunks);
        const int nt = (cout + 15) / 16;
        const size_t lds = (static_cast<size_t>(16 * nt) * kWgVox +
                            static_cast<size_t>(wg_taps(cin)) * cin * kWgVox) * sizeof(uint16_t);
        switch (nt) {
#define LWS_CASE(K) \
    case K: k_conv_wgrad_lds<K, kWgVox><<<grid, kThreads, lds, s>>>(x, x_shared, cin, dz, cout, work, g, chunk); break;
            LWS_CASE(1) LWS_CASE(2) LWS_CASE(3) LWS_CASE(4)
#undef LWS_CASE
        default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const uint64_t n = static_cast<uint64_t>(mrows) * cout;
        k_sum_chunks<<<static_cast<unsigned>((n + kSumOut - 1) / kSumOut), kThreads, 0, s>>>(
            work, static_cast<int>(nchunks), n, dw);
        return hipGetLastError();
    }
    constexpr int MT = 2;
    const dim3 grid(static_cast<unsigned>((mrows + 64 * MT - 1) / (64 * MT)), nchunks);
    switch ((cout + 15) / 16) {
#define LWS_CASE(K) \
    case K: k_conv_wgrad<K, MT><<<grid, kThreads, 0, s>>>(x, x_shared, cin, dz, cout, work, g, chunk); break;
        LWS_CASE(1) LWS_CASE(2) LWS_CASE(3) LWS_CASE(4)
#undef LWS_CASE
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t n = static_cast<uint64_t>(mrows) * cout;
    k_sum_chunks<<<static_cast<unsigned>((n + kSumOut - 1) / kSumOut), kThreads, 0, s>>>(
        work, static_cast<int>(nchunks), n, dw);
    return hipGetLastError();
}

size_t wgrad_work_for(int cin, int cout, const Grid &g, uint64_t chunk) {
    const uint64_t nchunks = (g.total + chunk - 1) / chunk;
    return static_cast<size_t>(nchunks) * 27 * cin * cout * sizeof(float);
}

size_t wgrad_work(int cin, int cout, const Grid &g) {
    return wgrad_work_for(cin, cout, g, wgrad_chunk(g.total, cin));
}

// ---------------------------------------------------------------------------
// Allocation-free weight gradient: its per-chunk partial tiles go to this
// file-scope device array instead of a caller's workspace.  Each GPU the
// library runs on holds its own copy (until the process ends); host code
// uses the address hipGetSymbolAddress gives on that device, never the
// array's name.  Every call overwrites the partials it reads, so nothing is
// cleared; calls that overlap on one GPU race for it.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t{64} << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.
hipError_t scratch_on_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// Voxels per chunk when the partials must fit in the scratch array: the
// usual chunking, coarsened until the chunk tiles fit.
uint64_t wgrad_chunk_capped(uint64_t total, int cin, int cout) {
    const uint64_t tile = static_cast<uint64_t>(27) * cin * cout * sizeof(float);
    const uint64_t maxchunks = std::max<uint64_t>(1, kScratchBytes / tile);
    uint64_t c = std::max(wgrad_chunk(total, cin), (total + maxchunks - 1) / maxchunks);
    return (c + kWgVox - 1) / kWgVox * kWgVox;
}

hipError_t pack(const float *w, int cin, int cout, int dgrad, uint16_t *out, hipStream_t s) {
    int rows, kpad;
    pack_dims(cin, cout, dgrad, &rows, &kpad);
    const uint64_t n = static_cast<uint64_t>(rows) * kpad;
    k_pack<<<blocks_for(n), kThreads, 0, s>>>(w, cin, cout, dgrad, rows, kpad, out);
    return hipGetLastError();
}

}  // namespace
}  // namespace lwsk

// ---------------------------------------------------------------------------
// The network
// ---------------------------------------------------------------------------
namespace {

using namespace lwsk;

enum { E1a, E1b, E2a, E2b, E3a, E3b, D2, D1, OUT, NLAYER };

struct Layer {
    int cin, cout, level;
    bool film;
    size_t oW, oGw, oGb, oBw, oBb, ob;   // offsets in the flat parameter vector
    size_t pf, pd;                       // offsets of the packed operands (elements)
    int kpf, kpd;                        // their row lengths
};

}  // namespace

struct lws_net {
    int M = 0, maxB = 0, ch[3] = {16, 32, 64};
    int n[3] = {0, 0, 0};
    uint64_t V[3] = {0, 0, 0};
    Layer L[NLAYER];
    int64_t nparam = 0;
    int64_t step = 0;
    bool packed_ok = false;
    std::vector<void *> allocs;
    float *param = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *packed = nullptr;
    uint16_t *feat = nullptr;
    float *Z[NLAYER] = {};
    float *scale = nullptr, *shift = nullptr;   // [NLAYER][maxB][64]
    float *cond = nullptr, *tscale = nullptr;
    // activations (bfloat16)
    uint16_t *aE1a = nullptr, *cat1 = nullptr, *inE2a = nullptr, *aE2a = nullptr, *cat2 = nullptr,
             *inE3a = nullptr, *aE3a = nullptr, *s3 = nullptr, *aD2 = nullptr, *aD1 = nullptr;
    // gradients
    float *dout = nullptr, *dA = nullptr, *dcat1 = nullptr, *dcat2 = nullptr, *dA2 = nullptr, *dIn = nullptr;
    uint16_t *doutb = nullptr, *dzb = nullptr;
    float *work = nullptr;
    size_t work_bytes = 0;
    double *part = nullptr, *loss = nullptr, *fsum = nullptr;
    int nbx = 64;
    std::string err;
};

namespace {

int net_fail(lws_net_t *n, int code, const std::string &msg) {
    if (n) n->err = msg;
    return code;
}

int hip_check(lws_net_t *n, hipError_t e, const char *where) {
    if (e == hipSuccess) return LBM_OK;
    return net_fail(n, LBM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

template <class T>
bool alloc(lws_net_t *n, T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
    n->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return true;
}

lws_grid level_grid(const lws_net_t *n, int B, int level) {
    return lws_grid{B, n->n[level], n->n[level], n->n[level]};
}

float *pp(lws_net_t *n, size_t off) { return n->param + off; }
float *gp(lws_net_t *n, size_t off) { return n->grad + off; }

hipError_t pack_all(lws_net_t *n, hipStream_t s) {
    for (int l = 0; l < NLAYER; ++l) {
        const Layer &y = n->L[l];
        hipError_t e = pack(pp(n, y.oW), y.cin, y.cout, 0, n->packed + y.pf, s);
        if (e == hipSuccess) e = pack(pp(n, y.oW), y.cin, y.cout, 1, n->packed + y.pd, s);
        if (e != hipSuccess) return e;
    }
    n->packed_ok = true;
    return hipSuccess;
}

float *sc_of(lws_net_t *n, int l) { return n->scale + static_cast<size_t>(l) * n->maxB * 64; }
float *sh_of(lws_net_t *n, int l) { return n->shift + static_cast<size_t>(l) * n->maxB * 64; }

bool fits32(uint64_t n) { return n < (uint64_t{1} << 32); }

// Interpolation from level nc^3 to (2 nc - 1)^3 and its adjoint, with 32-bit
// indices when every index of the launch fits.
void prolong(const uint16_t *in, int C, int nc, int B, uint16_t *out, int ostride, int ooff, hipStream_t s) {
    const uint64_t nf = 2 * static_cast<uint64_t>(nc) - 1, nfine = B * nf * nf * nf;
    const unsigned blocks = blocks_for(nfine * C);
    if (fits32(nfine * std::max(C, ostride)))
        k_prolong<uint32_t><<<blocks, kThreads, 0, s>>>(in, C, nc, B, out, ostride, ooff);
    else
        k_prolong<uint64_t><<<blocks, kThreads, 0, s>>>(in, C, nc, B, out, ostride, ooff);
}
void prolong_adj(const float *gf, int gstride, int goff, int C, int nc, int B, float *out, hipStream_t s) {
    const uint64_t nf = 2 * static_cast<uint64_t>(nc) - 1, nfine = B * nf * nf * nf,
                   ncoarse = B * static_cast<uint64_t>(nc) * nc * nc;
    const unsigned blocks = blocks_for(ncoarse * C);
    if (fits32(nfine * gstride) && fits32(ncoarse * C))
        k_prolong_adj<uint32_t><<<blocks, kThreads, 0, s>>>(gf, gstride, goff, C, nc, B, out);
    else
        k_prolong_adj<uint64_t><<<blocks, kThreads, 0, s>>>(gf, gstride, goff, C, nc, B, out);
}

// conv + FiLM + SiLU of layer l into out (stride, offset)
hipError_t layer_fwd(lws_net_t *n, int l, const uint16_t *x, int x_shared, int B, uint16_t *out, int ostride,
                     int ooff, hipStream_t s) {
    const Layer &y = n->L[l];
    const Grid g = make_grid(level_grid(n, B, y.level));
    hipError_t e = conv_fwd(x, x_shared, y.cin, n->packed + y.pf, y.kpf, y.cout, n->Z[l], g, s);
    if (e != hipSuccess) return e;
    if (fits32(g.total * std::max(y.cout, ostride)))
        k_film_act<uint32_t><<<blocks_for(g.total * y.cout), kThreads, 0, s>>>(n->Z[l], y.cout, g, sc_of(n, l),
                                                                            sh_of(n, l), out, ostride, ooff);
    else
        k_film_act<uint64_t><<<blocks_for(g.total * y.cout), kThreads, 0, s>>>(n->Z[l], y.cout, g, sc_of(n, l),
                                                                            sh_of(n, l), out, ostride, ooff);
    return hipGetLastError();
}

// FiLM backward + weight gradient (+ data gradient into dx when dx != NULL)
hipError_t layer_bwd(lws_net_t *n, int l, const float *da, int dstride, int doff, const uint16_t *x,
                     int x_shared, int B, float *dx, hipStream_t s) {
    const Layer &y = n->L[l];
    const Grid g = make_grid(level_grid(n, B, y.level));
    const dim3 grid(static_cast<unsigned>(n->nbx), static_cast<unsigned>(B));
    k_film_bwd<<<grid, kThreads, 0, s>>>(da, dstride, doff, n->Z[l], y.cout, g, sc_of(n, l), sh_of(n, l), n->dzb,
                                         n->part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_film_sums<<<static_cast<unsigned>(B), 128, 0, s>>>(n->part, n->nbx, y.cout, n->fsum);
    k_film_grads<<<1, 64, 0, s>>>(n->fsum, B, y.cout, n->cond, gp(n, y.oGw), gp(n, y.oGb), gp(n, y.oBw),
                                  gp(n, y.oBb));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = conv_wgrad(x, x_shared, y.cin, n->dzb, y.cout, gp(n, y.oW), g, n->work,
                        wgrad_chunk(g.total, y.cin), s)) != hipSuccess)
        return e;
    if (dx) e = conv_fwd(n->dzb, 0, y.cout, n->packed + y.pd, y.kpd, y.cin, dx, g, s);
    return e;
}

hipError_t set_cond(lws_net_t *n, int B, const double *ra_pr, hipStream_t s) {
    std::vector<float> c(2 * static_cast<size_t>(B));
    for (int b = 0; b < B; ++b) {
        c[2 * b] = static_cast<float>((std::log10(ra_pr[2 * b]) - 5.5) / 1.5);
        c[2 * b + 1] = static_cast<float>((ra_pr[2 * b + 1] - 3.855) / 3.145);
    }
    hipError_t e = hipMemcpyAsync(n->cond, c.data(), c.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // c is a local host buffer
    if (e != hipSuccess) return e;
    for (int l = 0; l < NLAYER; ++l) {
        const Layer &y = n->L[l];
        if (!y.film) continue;
        k_film_params<<<blocks_for(static_cast<uint64_t>(B) * y.cout), kThreads, 0, s>>>(
            pp(n, y.oGw), pp(n, y.oGb), pp(n, y.oBw), pp(n, y.oBb), y.cout, n->cond, B, sc_of(n, l), sh_of(n, l));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

int check_ra_pr(lws_net_t *n, int B, const double *ra_pr) {
    if (B < 1 || B > n->maxB) return net_fail(n, LBM_EINVAL, "batch size outside [1, max_batch]");
    if (!ra_pr) return net_fail(n, LBM_EINVAL, "ra_pr is NULL");
    for (int i = 0; i < B; ++i)
        if (!(ra_pr[2 * i] > 0.0) || !(ra_pr[2 * i + 1] > 0.0) || !std::isfinite(ra_pr[2 * i]) ||
            !std::isfinite(ra_pr[2 * i + 1]))
            return net_fail(n, LBM_EINVAL, "Ra and Pr must be positive and finite");
    return LBM_OK;
}

hipError_t forward(lws_net_t *n, int B, hipStream_t s) {
    hipError_t e;
    if (!n->packed_ok && (e = pack_all(n, s)) != hipSuccess) return e;
    const int c1 = n->ch[0], c2 = n->ch[1], c3 = n->ch[2];
    if ((e = layer_fwd(n, E1a, n->feat, 1, B, n->aE1a, c1, 0, s)) != hipSuccess) return e;
    if ((e = layer_fwd(n, E1b, n->aE1a, 0, B, n->cat1, c2 + c1, c2, s)) != hipSuccess) return e;
    k_restrict<<<blocks_for(static_cast<uint64_t>(B) * n->V[1] * c1), kThreads, 0, s>>>(n->cat1, c2 + c1, c2, c1,
                                                                                     n->n[0], B, n->inE2a);
    if ((e = layer_fwd(n, E2a, n->inE2a, 0, B, n->aE2a, c2, 0, s)) != hipSuccess) return e;
    if ((e = layer_fwd(n, E2b, n->aE2a, 0, B, n->cat2, c3 + c2, c3, s)) != hipSuccess) return e;
    k_restrict<<<blocks_for(static_cast<uint64_t>(B) * n->V[2] * c2), kThreads, 0, s>>>(n->cat2, c3 + c2, c3, c2,
                                                                                     n->n[1], B, n->inE3a);
    if ((e = layer_fwd(n, E3a, n->inE3a, 0, B, n->aE3a, c3, 0, s)) != hipSuccess) return e;
    if ((e = layer_fwd(n, E3b, n->aE3a, 0, B, n->s3, c3, 0, s)) != hipSuccess) return e;
    prolong(n->s3, c3, n->n[2], B, n->cat2, c3 + c2, 0, s);
    if ((e = layer_fwd(n, D2, n->cat2, 0, B, n->aD2, c2, 0, s)) != hipSuccess) return e;
    prolong(n->aD2, c2, n->n[1], B, n->cat1, c2 + c1, 0, s);
    if ((e = layer_fwd(n, D1, n->cat1, 0, B, n->aD1, c1, 0, s)) != hipSuccess) return e;
    const Layer &o = n->L[OUT];
    const Grid g0 = make_grid(level_grid(n, B, 0));
    if ((e = conv_fwd(n->aD1, 0, o.cin, n->packed + o.pf, o.kpf, o.cout, n->Z[OUT], g0, s)) != hipSuccess)
        return e;
    k_add_bias<<<blocks_for(g0.total * o.cout), kThreads, 0, s>>>(n->Z[OUT], o.cout, g0.total, pp(n, o.ob));
    return hipGetLastError();
}

hipError_t backward(lws_net_t *n, int B, hipStream_t s) {
    hipError_t e;
    const int c1 = n->ch[0], c2 = n->ch[1], c3 = n->ch[2];
    const Layer &o = n->L[OUT];
    const Grid g0 = make_grid(level_grid(n, B, 0));
    // output layer: weights, bias, input gradient
    if ((e = conv_wgrad(n->aD1, 0, o.cin, n->doutb, o.cout, gp(n, o.oW), g0, n->work,
                        wgrad_chunk(g0.total, o.cin), s)) != hipSuccess)
        return e;
    // bias gradient: enough blocks to stream dout at full rate (64 blocks ran
    // at ~0.2 TB/s), within the partial buffer
    const size_t part_cap = static_cast<size_t>(n->maxB) * n->nbx * 2 * 64 + 4096;
    const int nbc = static_cast<int>(std::min<size_t>(1024, part_cap / o.cout));
    k_chan_partial<<<nbc, kThreads, 0, s>>>(n->dout, o.cout, g0.total, n->part);
    k_chan_final<<<1, 64, 0, s>>>(n->part, nbc, o.cout, gp(n, o.ob));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = conv_fwd(n->doutb, 0, o.cout, n->packed + o.pd, o.kpd, o.cin, n->dA, g0, s)) != hipSuccess) return e;
    // decoder
    if ((e = layer_bwd(n, D1, n->dA, c1, 0, n->cat1, 0, B, n->dcat1, s)) != hipSuccess) return e;
    prolong_adj(n->dcat1, c2 + c1, 0, c2, n->n[1], B, n->dA2, s);
    if ((e = layer_bwd(n, D2, n->dA2, c2, 0, n->cat2, 0, B, n->dcat2, s)) != hipSuccess) return e;
    prolong_adj(n->dcat2, c3 + c2, 0, c3, n->n[2], B, n->dA, s);
    // level 2
    if ((e = layer_bwd(n, E3b, n->dA, c3, 0, n->aE3a, 0, B, n->dA2, s)) != hipSuccess) return e;
    if ((e = layer_bwd(n, E3a, n->dA2, c3, 0, n->inE3a, 0, B, n->dIn, s)) != hipSuccess) return e;
    k_restrict_adj_add<<<blocks_for(static_cast<uint64_t>(B) * n->V[2] * c2), kThreads, 0, s>>>(
        n->dIn, c2, n->n[1], B, n->dcat2, c3 + c2, c3);
    // level 1
    if ((e = layer_bwd(n, E2b, n->dcat2, c3 + c2, c3, n->aE2a, 0, B, n->dA2, s)) != hipSuccess) return e;
    if ((e = layer_bwd(n, E2a, n->dA2, c2, 0, n->inE2a, 0, B, n->dIn, s)) != hipSuccess) return e;
    k_restrict_adj_add<<<blocks_for(static_cast<uint64_t>(B) * n->V[1] * c1), kThreads, 0, s>>>(
        n->dIn, c1, n->n[0], B, n->dcat1, c2 + c1, c2);
    // level 0
    if ((e = layer_bwd(n, E1b, n->dcat1, c2 + c1, c2, n->aE1a, 0, B, n->dA, s)) != hipSuccess) return e;
    return layer_bwd(n, E1a, n->dA, c1, 0, n->feat, 1, B, nullptr, s);
}

}  // namespace

extern "C" {

size_t lws_packed_elems(int cin, int cout, int for_data_grad) {
    if (cin < 1 || cout < 1) return 0;
    int rows, kpad;
    pack_dims(cin, cout, for_data_grad, &rows, &kpad);
    return static_cast<size_t>(rows) * kpad;
}

int lws_pack_weights(const float *w, int cin, int cout, int for_data_grad, uint16_t *packed, void *stream) {
    if (!w || !packed || cin < 1 || cout < 1 || cin > kMaxCin || cout > kMaxCin) return LBM_EINVAL;
    return pack(w, cin, cout, for_data_grad ? 1 : 0, packed, static_cast<hipStream_t>(stream)) == hipSuccess
               ? LBM_OK
               : LBM_EDEVICE;
}

int lws_conv3d_forward(const uint16_t *x, int x_shared, int cin, const uint16_t *packed, int cout, float *z,
                       lws_grid g, void *stream) {
    if (!x || !packed || !z || !grid_ok(g) || cin < 8 || cin % 8 || cin > kMaxCin || cout < 1 || cout > kMaxCout)
        return LBM_EINVAL;
    int rows, kpad;
    pack_dims(cin, cout, 0, &rows, &kpad);
    return conv_fwd(x, x_shared, cin, packed, kpad, cout, z, make_grid(g), static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? LBM_OK
               : LBM_EDEVICE;
}

int lws_conv3d_backward_data(const uint16_t *dz, int cout, const uint16_t *packed, int cin, float *dx, lws_grid g,
                             void *stream) {
    if (!dz || !packed || !dx || !grid_ok(g) || cout < 8 || cout % 8 || cout > kMaxCin || cin < 1 ||
        cin > kMaxCin)
        return LBM_EINVAL;
    int rows, kpad;
    pack_dims(cin, cout, 1, &rows, &kpad);
    return conv_fwd(dz, 0, cout, packed, kpad, cin, dx, make_grid(g), static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? LBM_OK
               : LBM_EDEVICE;
}

size_t lws_wgrad_work_bytes(int cin, int cout, lws_grid g) {
    if (!grid_ok(g) || cin < 1 || cout < 1) return 0;
    return wgrad_work(cin, cout, make_grid(g));
}

int lws_conv3d_backward_weight(const uint16_t *x, int x_shared, int cin, const uint16_t *dz, int cout, float *dw,
                               lws_grid g, void *work, size_t work_bytes, void *stream) {
    if (!x || !dz || !dw || !work || !grid_ok(g) || cin < 1 || cin > kMaxCin || cout < 1 || cout > kMaxCout)
        return LBM_EINVAL;
    const Grid gg = make_grid(g);
    if (work_bytes < wgrad_work(cin, cout, gg)) return LBM_ENOMEM;
    return conv_wgrad(x, x_shared, cin, dz, cout, dw, gg, static_cast<float *>(work), wgrad_chunk(gg.total, cin),
                      static_cast<hipStream_t>(stream)) == hipSuccess
               ? LBM_OK
               : LBM_EDEVICE;
}

int lws_conv3d_backward_weight_noalloc(const uint16_t *x, int x_shared, int cin, const uint16_t *dz, int cout,
                                       float *dw, lws_grid g, void *stream) {
    if (!x || !dz || !dw || !grid_ok(g) || cin < 1 || cin > kMaxCin || cout < 1 || cout > kMaxCout)
        return LBM_EINVAL;
    const Grid gg = make_grid(g);
    const uint64_t chunk = wgrad_chunk_capped(gg.total, cin, cout);
    if (wgrad_work_for(cin, cout, gg, chunk) > kScratchBytes) return LBM_EINVAL;   // cannot fit
    void *ptr = nullptr;
    if (scratch_on_current_device(&ptr) != hipSuccess) return LBM_EDEVICE;
    return conv_wgrad(x, x_shared, cin, dz, cout, dw, gg, static_cast<float *>(ptr), chunk,
                      static_cast<hipStream_t>(stream)) == hipSuccess
               ? LBM_OK
               : LBM_EDEVICE;
}

int lws_upsample_fields(const float *pred, int M, int ld, int N, int cell, double U, double T_hot, double T_cold,
                        int symmetrize, double *uvwT, void *stream) {
    if (!pred || !uvwT || M < 2 || ld < 4 || N < 1 || (cell != LBM_SIDE_HEATED && cell != LBM_RAYLEIGH_BENARD) ||
        !std::isfinite(U) || !std::isfinite(T_hot) || !std::isfinite(T_cold))
        return LBM_EINVAL;
    const uint64_t V = static_cast<uint64_t>(N) * N * N;
    k_upsample<<<blocks_for(V), kThreads, 0, static_cast<hipStream_t>(stream)>>>(
        pred, M, ld, N, cell == LBM_SIDE_HEATED ? 0 : 2, (symmetrize && cell == LBM_SIDE_HEATED) ? 1 : 0, U, T_hot,
        T_cold, uvwT);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

int lws_net_create(int M, int max_batch, const int ch[3], lws_net_t **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (M < 5 || M % 4 != 1 || M > 257 || max_batch < 1 || max_batch > 256) return LBM_EINVAL;
    int c[3] = {16, 32, 64};
    if (ch)
        for (int i = 0; i < 3; ++i) c[i] = ch[i];
    for (int i = 0; i < 3; ++i)
        if (c[i] < 16 || c[i] > 64 || c[i] % 16) return LBM_EINVAL;
    lws_net_t *n = new (std::nothrow) lws_net;
    if (!n) return LBM_ENOMEM;
    n->M = M;
    n->maxB = max_batch;
    for (int i = 0; i < 3; ++i) n->ch[i] = c[i];
    n->n[0] = M;
    n->n[1] = (M + 1) / 2;
    n->n[2] = (n->n[1] + 1) / 2;
    for (int i = 0; i < 3; ++i) n->V[i] = static_cast<uint64_t>(n->n[i]) * n->n[i] * n->n[i];
    const int c1 = c[0], c2 = c[1], c3 = c[2];
    const int spec[NLAYER][4] = {{8, c1, 0, 1},       {c1, c1, 0, 1}, {c1, c2, 1, 1},
                                 {c2, c2, 1, 1},      {c2, c3, 2, 1}, {c3, c3, 2, 1},
                                 {c3 + c2, c2, 1, 1}, {c2 + c1, c1, 0, 1}, {c1, 8, 0, 0}};
    size_t off = 0, poff = 0;
    for (int l = 0; l < NLAYER; ++l) {
        Layer &y = n->L[l];
        y.cin = spec[l][0];
        y.cout = spec[l][1];
        y.level = spec[l][2];
        y.film = spec[l][3] != 0;
        y.oW = off;
        off += static_cast<size_t>(27) * y.cin * y.cout;
        if (y.film) {
            y.oGw = off;
            y.oGb = off + 2 * y.cout;
            y.oBw = off + 3 * y.cout;
            y.oBb = off + 5 * y.cout;
            off += 6 * y.cout;
            y.ob = 0;
        } else {
            y.ob = off;
            off += y.cout;
        }
        int rows;
        pack_dims(y.cin, y.cout, 0, &rows, &y.kpf);
        y.pf = poff;
        poff += static_cast<size_t>(rows) * y.kpf;
        pack_dims(y.cin, y.cout, 1, &rows, &y.kpd);
        y.pd = poff;
        poff += static_cast<size_t>(rows) * y.kpd;
    }
    n->nparam = static_cast<int64_t>(off);
    const size_t B = max_batch;
    const size_t V0 = n->V[0], V1 = n->V[1], V2 = n->V[2];
    bool ok = alloc(n, &n->param, off) && alloc(n, &n->grad, off) && alloc(n, &n->m, off) &&
              alloc(n, &n->v, off) && alloc(n, &n->packed, poff) && alloc(n, &n->feat, V0 * 8) &&
              alloc(n, &n->scale, NLAYER * B * 64) && alloc(n, &n->shift, NLAYER * B * 64) &&
              alloc(n, &n->cond, 2 * B) && alloc(n, &n->tscale, 4 * B) && alloc(n, &n->aE1a, B * V0 * c1) &&
              alloc(n, &n->cat1, B * V0 * (c2 + c1)) && alloc(n, &n->inE2a, B * V1 * c1) &&
              alloc(n, &n->aE2a, B * V1 * c2) && alloc(n, &n->cat2, B * V1 * (c3 + c2)) &&
              alloc(n, &n->inE3a, B * V2 * c2) && alloc(n, &n->aE3a, B * V2 * c3) && alloc(n, &n->s3, B * V2 * c3) &&
              alloc(n, &n->aD2, B * V1 * c2) && alloc(n, &n->aD1, B * V0 * c1) && alloc(n, &n->dout, B * V0 * 8) &&
              alloc(n, &n->doutb, B * V0 * 8) &&
              alloc(n, &n->dA, B * std::max({V0 * c1, V2 * c3})) &&
              alloc(n, &n->dcat1, B * V0 * (c2 + c1)) && alloc(n, &n->dcat2, B * V1 * (c3 + c2)) &&
              alloc(n, &n->dA2, B * std::max({V1 * c2, V2 * c3})) &&
              alloc(n, &n->dIn, B * std::max({V1 * c1, V2 * c2})) &&
              alloc(n, &n->dzb, B * std::max({V0 * c1, V1 * c2, V2 * c3, V0 * 8})) &&
              alloc(n, &n->part, static_cast<size_t>(B) * n->nbx * 2 * 64 + 4096) && alloc(n, &n->loss, 1) &&
              alloc(n, &n->fsum, static_cast<size_t>(B) * 2 * 64);
    for (int l = 0; ok && l < NLAYER; ++l) {
        const Layer &y = n->L[l];
        ok = alloc(n, &n->Z[l], B * n->V[y.level] * y.cout);
        const Grid g = make_grid(lws_grid{max_batch, n->n[y.level], n->n[y.level], n->n[y.level]});
        n->work_bytes = std::max(n->work_bytes, wgrad_work(y.cin, y.cout, g));
    }
    ok = ok && alloc(n, &n->work, n->work_bytes / sizeof(float));
    if (!ok) {
        lws_net_destroy(n);
        return LBM_ENOMEM;
    }
    k_features<<<blocks_for(V0), kThreads>>>(M, n->feat);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        lws_net_destroy(n);
        return LBM_EDEVICE;
    }
    *out = n;
    return LBM_OK;
}

int lws_net_destroy(lws_net_t *net) {
    if (!net) return LBM_EINVAL;
    for (void *p : net->allocs) (void)hipFree(p);
    delete net;
    return LBM_OK;
}

int64_t lws_net_param_count(const lws_net_t *net) { return net ? net->nparam : -1; }

int lws_net_set_params(lws_net_t *net, const float *host) {
    if (!net) return LBM_EINVAL;
    if (!host) return net_fail(net, LBM_EINVAL, "host is NULL");
    const size_t bytes = net->nparam * sizeof(float);
    hipError_t e = hipMemcpy(net->param, host, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(net->m, 0, bytes);
    if (e == hipSuccess) e = hipMemset(net->v, 0, bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    net->step = 0;
    net->packed_ok = false;
    return hip_check(net, e, "set params");
}

int lws_net_get_params(lws_net_t *net, float *host) {
    if (!net) return LBM_EINVAL;
    if (!host) return net_fail(net, LBM_EINVAL, "host is NULL");
    return hip_check(net, hipMemcpy(host, net->param, net->nparam * sizeof(float), hipMemcpyDeviceToHost),
                     "get params");
}

int lws_net_get_grad(lws_net_t *net, float *host) {
    if (!net) return LBM_EINVAL;
    if (!host) return net_fail(net, LBM_EINVAL, "host is NULL");
    return hip_check(net, hipMemcpy(host, net->grad, net->nparam * sizeof(float), hipMemcpyDeviceToHost),
                     "get grad");
}

int lws_net_forward(lws_net_t *net, int B, const double *ra_pr, float *out, void *stream) {
    if (!net) return LBM_EINVAL;
    int rc = check_ra_pr(net, B, ra_pr);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = set_cond(net, B, ra_pr, s);
    if (e == hipSuccess) e = forward(net, B, s);
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(out, net->Z[OUT], static_cast<size_t>(B) * net->V[0] * 8 * sizeof(float),
                           hipMemcpyDeviceToDevice, s);
    return hip_check(net, e, "forward");
}

int lws_net_loss_grad(lws_net_t *net, int B, const double *ra_pr, const float *target, const double *scale,
                      double *loss, void *stream) {
    if (!net) return LBM_EINVAL;
    int rc = check_ra_pr(net, B, ra_pr);
    if (rc) return rc;
    if (!target) return net_fail(net, LBM_EINVAL, "target is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<float> ts(4 * static_cast<size_t>(B), 1.f);
    if (scale)
        for (size_t i = 0; i < ts.size(); ++i) ts[i] = static_cast<float>(scale[i]);
    hipError_t e = hipMemcpyAsync(net->tscale, ts.data(), ts.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = set_cond(net, B, ra_pr, s);
    if (e == hipSuccess) e = forward(net, B, s);
    if (e != hipSuccess) return hip_check(net, e, "forward");
    const Grid g0 = make_grid(level_grid(net, B, 0));
    const unsigned nb = blocks_for(g0.total);
    double *lpart = net->part;   // the FiLM partials are not live yet
    if (static_cast<size_t>(nb) > static_cast<size_t>(net->maxB) * net->nbx * 2 * 64 + 4096)
        return net_fail(net, LBM_EINVAL, "loss partial buffer too small");
    k_mse<<<nb, kThreads, 0, s>>>(net->Z[OUT], target, net->tscale, g0, net->dout, net->doutb, lpart);
    k_sum_doubles<<<1, kThreads, 0, s>>>(lpart, static_cast<int>(nb), 1.0 / static_cast<double>(g0.total * 4), net->loss);
    e = hipGetLastError();
    double l = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&l, net->loss, sizeof l, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = backward(net, B, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_check(net, e, "loss/backward");
    if (loss) *loss = l;
    if (!std::isfinite(l)) return net_fail(net, LBM_EDIVERGED, "loss is not finite");
    return LBM_OK;
}

int lws_net_adam(lws_net_t *net, double lr, void *stream) {
    if (!net) return LBM_EINVAL;
    if (!(lr > 0.0) || !std::isfinite(lr)) return net_fail(net, LBM_EINVAL, "learning rate must be positive");
    net->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = static_cast<float>(1.0 - std::pow(b1, static_cast<double>(net->step)));
    const float bc2 = static_cast<float>(1.0 - std::pow(b2, static_cast<double>(net->step)));
    k_adam<<<blocks_for(net->nparam), kThreads, 0, static_cast<hipStream_t>(stream)>>>(
        net->param, net->grad, net->m, net->v, static_cast<uint64_t>(net->nparam), static_cast<float>(lr), 0.9f,
        0.999f, 1e-8f, bc1, bc2);
    net->packed_ok = false;
    return hip_check(net, hipGetLastError(), "adam");
}

const char *lws_last_error(const lws_net_t *net) { return net ? net->err.c_str() : "NULL net"; }

}  // extern "C"
