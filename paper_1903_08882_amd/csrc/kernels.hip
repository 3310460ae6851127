// kernels.hip -- gfx950 kernels of the coupled D3Q19-MRT / D3Q7-MRT thermal
// lattice Boltzmann step (Xu, Shi & Xi 2019, arXiv:1903.08882).
//
// Storage: z-slabs of node blocks.  Each z-plane of the lattice is one slab;
// its N^2 nodes, numbered r = x + N y, are cut into sub-blocks of B = 2^b
// consecutive nodes (B * element size = 32 KB), and the 26 populations of a
// sub-block (f_0..f_18, g_0..g_6) are stored one after the other:
//   slot q of node (x, y, z) at byte
//     z slab + (r >> b) sub + start(q) B + (r & (B-1)) size(q),
// where size(q) is the storage width of population q and start(q) the sum of
// the widths before it.  All nodes of one launch block share z, so z enters
// through a wave-uniform base and a lane only carries a 32-bit byte offset.
// (Keeping the 26 copies of a node within one sub-block, instead of one
// full-lattice plane apart, is what lets the 52 access streams of a step run
// near copy bandwidth on HBM.)
// f is stored as the deviation f_i - w_i from the rest equilibrium (rho = 1,
// u = 0), g as is (its rest equilibrium at the mean wall temperature 0 is
// zero).  FP16 storage keeps f as FP16 (scaled by a power of two) and g in
// FP32; slots of one sub-block may have different widths.
//
// Streaming uses the in-place AA pattern, so each step reads and writes the
// same 26 slots per node and the state needs one copy:
//   parity 0 (canonical): slot i of node x holds f_i(x, t).
//     The step collides and writes f_i+(x) into slot opp(i) of the same node.
//   parity 1 (swapped): slot opp(i) of node x holds f_i+(x, t-1).
//     The step gathers f_i(x, t) = f_i+(x - e_i, t-1) from slot opp(i) of the
//     upstream node, collides, and writes f_i+(x) into slot i of x + e_i.
// A link that crosses a wall never leaves its node: in parity 1 the value
// coming back from the wall sits in slot i of x itself, and the outgoing value
// goes to slot opp(i) of x.  The wall rules of Sec. 2.2 / 2.3 are applied on
// exactly those accesses:
//   f:             f_opp(x, t+1) =  f_i+(x, t)                  (no slip)
//   g, fixed T:    g_opp(x, t+1) = -g_i+(x, t) + (6 + a_T)/21 T_w
//   g, adiabatic:  g_opp(x, t+1) =  g_i+(x, t)
// Every wall sits half a link from the nodes next to it; D3Q19 diagonal links
// that cross two walls bounce back the same way, and D3Q7 links cross one.
#include <type_traits>

#include <algorithm>

#include "lbm_internal.h"

namespace lbmk {
namespace {

// ---------------------------------------------------------------------------
// Lattice constants: velocity order of the paper's printed arrays.
// ---------------------------------------------------------------------------
constexpr int EX[kQF] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EY[kQF] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZ[kQF] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int OPP[kQF] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
constexpr int GX[kQG] = {0, 1, -1, 0, 0, 0, 0};
constexpr int GY[kQG] = {0, 0, 0, 1, -1, 0, 0};
constexpr int GZ[kQG] = {0, 0, 0, 0, 0, 1, -1};
constexpr int GOPP[kQG] = {0, 2, 1, 4, 3, 6, 5};

// Rest weights of f^eq (Sec. 2.2).
__host__ __device__ constexpr double wrest(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---------------------------------------------------------------------------
// Storage codecs
// ---------------------------------------------------------------------------
// S: storage type of the narrow populations, W: of the wide ones (the first
// GW thermal populations g_0 .. g_{GW-1}), R: arithmetic type.  FP16 storage
// keeps all seven thermal populations in FP32: with only g_0 wide the
// temperature carries FP16 noise of ~1e-4 and the 129^3, Ra 1e6 steady Nu is
// 0.85% low; with all of g wide it is within 0.12% (f stays FP16).
struct CF64 { using S = double; using W = double; using R = double; static constexpr int GW = 1; };
struct CF32 { using S = float; using W = float; using R = float; static constexpr int GW = 1; };
struct CF16 { using S = _Float16; using W = float; using R = float; static constexpr int GW = kQG; };
struct CF16C { using S = int16_t; using W = float; using R = float; static constexpr int GW = kQG; };

// The customised 16-bit deviation format of CF16C: sign, 4-bit exponent with
// bias 18, 11-bit mantissa, subnormals below 2^-17 (spacing 2^-28), no
// infinities; |v| >= 2^-2 saturates to the largest code.  One more mantissa
// bit than IEEE half over the range the deviations f_i - w_i occupy.  The
// codec runs 38 times per node and step, so both directions are a handful
// of branch-free instructions built on FP32 scaling by 2^-+109, which maps
// the format's normal range onto FP32 normals with exponent field e and its
// subnormals onto FP32 denormals (kept: this library is built without
// denormal flushing).
__device__ __forceinline__ int16_t c16_enc(float v) {
    // |v| 2^-109 is exact for |v| >= 2^-17; below, the FP32 denormal result
    // rounds |v| to a multiple of 2^-40 (ties to even) first
    const uint32_t a = __float_as_uint(fabsf(v) * 0x1p-109f);
    // drop 12 mantissa bits, ties to even; a carry moves into the exponent and
    // anything past the largest code (|v| >= 2^-2, inf, NaN) is clamped to it
    const uint32_t code = min((a + 0x7ffu + ((a >> 12) & 1u)) >> 12, 0x7fffu);
    return static_cast<int16_t>(static_cast<uint16_t>(code | ((__float_as_uint(v) >> 16) & 0x8000u)));
}
// Loaded sign-extended: shifting the 32-bit word left by 12 puts exponent and
// mantissa in place and ones in bits 27-31 of a negative code; clearing bits
// 27-30 leaves the sign.
__device__ __forceinline__ float c16_dec(int16_t c) {
    const uint32_t w = static_cast<uint32_t>(static_cast<int32_t>(c));
    return __uint_as_float((w << 12) & 0x87ffffffu) * 0x1p109f;
}

// Storage width and byte start (per node of a sub-block) of population q.
template <class C>
__host__ __device__ constexpr bool wide(int q) {
    return q >= kQF && q < kQF + C::GW;
}
template <class C>
__host__ __device__ constexpr uint32_t qsize(int q) {
    return wide<C>(q) ? sizeof(typename C::W) : sizeof(typename C::S);
}
template <class C>
__host__ __device__ constexpr uint32_t qstart(int q) {
    return q <= kQF ? q * sizeof(typename C::S)
                    : (q <= kQF + C::GW
                           ? kQF * sizeof(typename C::S) + (q - kQF) * sizeof(typename C::W)
                           : kQF * sizeof(typename C::S) + C::GW * sizeof(typename C::W) +
                                 (q - kQF - C::GW) * sizeof(typename C::S));
}

template <class C>
__device__ __forceinline__ typename C::R dec(typename C::S v, typename C::R inv_scale) {
    if constexpr (std::is_same<C, CF16>::value)
        return static_cast<float>(v) * inv_scale;
    else if constexpr (std::is_same<C, CF16C>::value)
        return c16_dec(v);
    else
        return v;
}
template <class C>
__device__ __forceinline__ typename C::S enc(typename C::R v, typename C::R scale) {
    if constexpr (std::is_same<C, CF16>::value)
        return static_cast<_Float16>(v * scale);
    else if constexpr (std::is_same<C, CF16C>::value)
        return c16_enc(v);
    else
        return v;
}

// ---------------------------------------------------------------------------
// Node of a (ceil(N^2 / blockDim), N) launch
// ---------------------------------------------------------------------------
struct Node {
    int x, y, z;
    uint64_t n;
};

// Launches are one-dimensional, gx blocks per z-plane.  The hardware hands
// consecutive workgroups to the XCDs in turn; they are renumbered so that
// each XCD works through one contiguous range of node chunks: neighbouring
// chunks share the cache lines of the neighbour-shifted accesses, and each
// XCD has its own L2.
constexpr uint32_t kXCD = 8;

__device__ __forceinline__ uint32_t xcd_order() {
    const uint32_t b = blockIdx.x, nb = gridDim.x;
    const uint32_t xcd = b % kXCD, idx = b / kXCD;
    const uint32_t per = nb / kXCD, rem = nb % kXCD;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Node of thread threadIdx.x in logical block lb of a lattice.
__device__ __forceinline__ bool node_at(const Geo &g, uint32_t lb, Node &d) {
    const uint32_t z = lb / g.gx;
    const uint32_t r = (lb - z * g.gx) * blockDim.x + threadIdx.x;
    d.z = static_cast<int>(z);
    d.y = __umulhi(r, g.magic);
    d.x = static_cast<int>(r) - d.y * g.N;
    d.n = static_cast<uint64_t>(d.z) * g.N2 + r;
    return r < g.N2;
}

__device__ __forceinline__ bool node_of(const Geo &g, Node &d) {
    return node_at(g, xcd_order(), d);
}

// x - e outside the box?  (the upstream node of link e)
__device__ __forceinline__ bool up_out(int ex, int ey, int ez, const Node &d, int N) {
    return (ex > 0 && d.x == 0) || (ex < 0 && d.x == N - 1) || (ey > 0 && d.y == 0) ||
           (ey < 0 && d.y == N - 1) || (ez > 0 && d.z == 0) || (ez < 0 && d.z == N - 1);
}
// x + e outside the box?  (the downstream node of link e)
__device__ __forceinline__ bool down_out(int ex, int ey, int ez, const Node &d, int N) {
    return (ex > 0 && d.x == N - 1) || (ex < 0 && d.x == 0) || (ey > 0 && d.y == N - 1) ||
           (ey < 0 && d.y == 0) || (ez > 0 && d.z == N - 1) || (ez < 0 && d.z == 0);
}
// The populations of one node as seen from its launch block: a wave-uniform
// byte base at the start of slab z - 1 and the node's in-plane index r.  Every
// slot a node touches (its own slab and slabs z +- 1) lies within
// [0, 3 slab) bytes of the base.
struct View {
    const char *base;
    int r;
};

__device__ __forceinline__ View view_of(const void *pop, const Geo &g, const Node &d) {
    View v;
    v.base = static_cast<const char *>(pop) +
             (static_cast<int64_t>(d.z) - 1) * static_cast<int64_t>(g.slab);
    v.r = d.x + d.y * g.N;
    return v;
}

// Byte offset from the base of slot q of the node displaced by (dx, dy, dz).
// For a displacement out of the box the value is meaningless and unused.
template <class C>
__device__ __forceinline__ uint32_t slot(const View &v, const Geo &g, int q, int dx, int dy,
                                         int dz) {
    const int r = v.r + dx + dy * g.N;
    return static_cast<uint32_t>(dz + 1) * g.slab + static_cast<uint32_t>(r >> g.bbits) * g.sub +
           (qstart<C>(q) << g.bbits) + static_cast<uint32_t>(r & g.bmask) * qsize<C>(q);
}

// Plain or streaming (non-temporal) access of one stored value.
template <bool NT, class T>
__device__ __forceinline__ T ld_raw(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void st_raw(T *p, T x) {
    if constexpr (NT) __builtin_nontemporal_store(x, p);
    else *p = x;
}

// Loads and stores of f (moving), g_j for j >= 1 (moving) and g_0 (resting).
// NT = true marks them streaming: used where every line a wave touches is read
// once and written back whole by the same wave (the canonical-storage step).
template <class C, bool NT = false>
__device__ __forceinline__ typename C::R ld_f(const View &v, uint32_t off,
                                              const Coef<typename C::R> &c) {
    return dec<C>(ld_raw<NT>(reinterpret_cast<const typename C::S *>(v.base + off)), c.isf);
}
template <class C, bool NT = false>
__device__ __forceinline__ typename C::R ld_g(const View &v, uint32_t off, int j,
                                              const Coef<typename C::R> &c) {
    if (j < C::GW) return static_cast<typename C::R>(ld_raw<NT>(reinterpret_cast<const typename C::W *>(v.base + off)));
    return dec<C>(ld_raw<NT>(reinterpret_cast<const typename C::S *>(v.base + off)), c.isg);
}
template <class C, bool NT = false>
__device__ __forceinline__ void st_f(const View &v, uint32_t off, typename C::R x,
                                     const Coef<typename C::R> &c) {
    st_raw<NT>(reinterpret_cast<typename C::S *>(const_cast<char *>(v.base) + off), enc<C>(x, c.sf));
}
template <class C, bool NT = false>
__device__ __forceinline__ void st_g(const View &v, uint32_t off, int j, typename C::R x,
                                     const Coef<typename C::R> &c) {
    char *p = const_cast<char *>(v.base) + off;
    if (j < C::GW) st_raw<NT>(reinterpret_cast<typename C::W *>(p), static_cast<typename C::W>(x));
    else st_raw<NT>(reinterpret_cast<typename C::S *>(p), enc<C>(x, c.sg));
}

// Component of D3Q7 link j along the isothermal axis (x side-heated, z RB).
template <int CELL>
__device__ __forceinline__ constexpr int iso_comp(int j) {
    return CELL == LBM_SIDE_HEATED ? GX[j] : GZ[j];
}

// ---------------------------------------------------------------------------
// Gather the pre-collision populations f_i(x, t), g_i(x, t) of a node.
// SW = false: canonical storage; SW = true: swapped storage (see top).
// f is returned as deviations f_i - w_i.  In canonical storage a wave reads
// and then rewrites exactly the lines of its own nodes, so those accesses are
// streaming (non-temporal): at 257^3 this took the canonical-storage step from
// 603 to 535 us and, with less dirty data left behind in the caches, the
// swapped-storage step after it from 670 to 641 us (FP32).  Streaming hints on
// the swapped-storage accesses, whose lines are shared with neighbouring
// waves, made that step slower.
// ---------------------------------------------------------------------------
template <class C, int CELL, bool SW>
__device__ __forceinline__ void gather(const typename C::S *__restrict__ pop, const Geo &g,
                                       const Node &d, const Coef<typename C::R> &c,
                                       typename C::R f[kQF], typename C::R h[kQG]) {
    using R = typename C::R;
    const View v = view_of(pop, g, d);
#pragma unroll
    for (int i = 0; i < kQF; ++i) {
        if constexpr (!SW) {
            f[i] = ld_f<C, true>(v, slot<C>(v, g, i, 0, 0, 0), c);
        } else {
            const bool out = up_out(EX[i], EY[i], EZ[i], d, g.N);
            const uint32_t off = out ? slot<C>(v, g, i, 0, 0, 0)
                                     : slot<C>(v, g, OPP[i], -EX[i], -EY[i], -EZ[i]);
            f[i] = ld_f<C>(v, off, c);
        }
    }
#pragma unroll
    for (int j = 0; j < kQG; ++j) {
        if constexpr (!SW) {
            h[j] = ld_g<C, true>(v, slot<C>(v, g, kQF + j, 0, 0, 0), j, c);
        } else {
            const bool out = up_out(GX[j], GY[j], GZ[j], d, g.N);
            const uint32_t off = out ? slot<C>(v, g, kQF + j, 0, 0, 0)
                                     : slot<C>(v, g, kQF + GOPP[j], -GX[j], -GY[j], -GZ[j]);
            R x = ld_g<C>(v, off, j, c);
            const int comp = iso_comp<CELL>(j);
            // arrived through the wall at the upstream side: anti-bounce-back
            if (comp != 0 && out) x = (comp > 0 ? c.abb_hot : c.abb_cold) - x;
            h[j] = x;
        }
    }
}

// Scatter the post-collision populations (see top for the two storage states).
template <class C, int CELL, bool SW>
__device__ __forceinline__ void scatter(typename C::S *__restrict__ pop, const Geo &g,
                                        const Node &d, const Coef<typename C::R> &c,
                                        const typename C::R f[kQF], const typename C::R h[kQG]) {
    using R = typename C::R;
    const View v = view_of(pop, g, d);
#pragma unroll
    for (int i = 0; i < kQF; ++i) {
        if constexpr (!SW) {
            st_f<C, true>(v, slot<C>(v, g, OPP[i], 0, 0, 0), f[i], c);
        } else {
            const bool out = down_out(EX[i], EY[i], EZ[i], d, g.N);
            const uint32_t off = out ? slot<C>(v, g, OPP[i], 0, 0, 0)
                                     : slot<C>(v, g, i, EX[i], EY[i], EZ[i]);
            st_f<C>(v, off, f[i], c);
        }
    }
#pragma unroll
    for (int j = 0; j < kQG; ++j) {
        if constexpr (!SW) {
            st_g<C, true>(v, slot<C>(v, g, kQF + GOPP[j], 0, 0, 0), j, h[j], c);
        } else {
            const bool out = down_out(GX[j], GY[j], GZ[j], d, g.N);
            const uint32_t off = out ? slot<C>(v, g, kQF + GOPP[j], 0, 0, 0)
                                     : slot<C>(v, g, kQF + j, GX[j], GY[j], GZ[j]);
            R x = h[j];
            const int comp = iso_comp<CELL>(j);
            // leaves through the wall at the downstream side: anti-bounce-back
            if (comp != 0 && out) x = (comp > 0 ? c.abb_cold : c.abb_hot) - x;
            st_g<C>(v, off, j, x, c);
        }
    }
}

// ---------------------------------------------------------------------------
// Macroscopic variables (Sec. 2.2, 2.3) from the deviations:
//   rho = 1 + sum f', T = sum g, F_z = rho g beta (T - T0),
//   rho u = sum e f' + F/2 (the rest weights carry no momentum).
// ---------------------------------------------------------------------------
template <class R>
struct Macro {
    R drho, jx, jy, jz, T, Fz, rho, ux, uy, uz;
};

template <class R>
__device__ __forceinline__ Macro<R> macros(const R f[kQF], const R h[kQG], const Coef<R> &c) {
    Macro<R> m;
    const R sax = (f[1] + f[2]) + (f[3] + f[4]) + (f[5] + f[6]);
    const R sdg = ((f[7] + f[10]) + (f[8] + f[9])) + ((f[11] + f[14]) + (f[12] + f[13])) +
                  ((f[15] + f[18]) + (f[16] + f[17]));
    m.drho = f[0] + sax + sdg;
    m.jx = (f[1] - f[2]) + (f[7] - f[10]) - (f[8] - f[9]) + (f[11] - f[14]) - (f[12] - f[13]);
    m.jy = (f[3] - f[4]) + (f[7] - f[10]) + (f[8] - f[9]) + (f[15] - f[18]) - (f[16] - f[17]);
    m.jz = (f[5] - f[6]) + (f[11] - f[14]) + (f[12] - f[13]) + (f[15] - f[18]) + (f[16] - f[17]);
    m.T = h[0] + (h[1] + h[2]) + (h[3] + h[4]) + (h[5] + h[6]);
    // a density deviation beyond what the storage represents marks the node
    // as diverged (NaN), which the FP32 thermal populations then carry
    if (!(fabs(m.drho) <= c.drho_max)) m.drho = static_cast<R>(NAN);
    m.rho = R(1) + m.drho;
    m.Fz = m.rho * c.gbeta * (m.T - c.T0);
    m.jz += R(0.5) * m.Fz;
    const R ir = R(1) / m.rho;
    m.ux = m.jx * ir;
    m.uy = m.jy * ir;
    m.uz = m.jz * ir;
    return m;
}

// ---------------------------------------------------------------------------
// Collision of one node, in place (Eq. MRT with F' = M^-1 (I - S/2) M F~ and
// Eq. MRT_T).  M and N have integer, mutually orthogonal rows, so
// m = M f' is taken through the opposite-pair sums s and differences d, and
// f+ = f + M^T diag(1/|M_k|^2) dm is expanded back the same way.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ Macro<R> collide(R f[kQF], R h[kQG], const Coef<R> &c) {
    const Macro<R> mc = macros(f, h, c);
    const R s1 = f[1] + f[2], d1 = f[1] - f[2];
    const R s3 = f[3] + f[4], d3 = f[3] - f[4];
    const R s5 = f[5] + f[6], d5 = f[5] - f[6];
    const R s7 = f[7] + f[10], d7 = f[7] - f[10];
    const R s8 = f[8] + f[9], d8 = f[8] - f[9];
    const R s11 = f[11] + f[14], d11 = f[11] - f[14];
    const R s12 = f[12] + f[13], d12 = f[12] - f[13];
    const R s15 = f[15] + f[18], d15 = f[15] - f[18];
    const R s16 = f[16] + f[17], d16 = f[16] - f[17];
    const R sax = s1 + s3 + s5;
    const R pxy = s7 + s8, pxz = s11 + s12, pyz = s15 + s16;
    const R sdg = pxy + pxz + pyz;

    const R jx = mc.jx, jy = mc.jy, jz = mc.jz;   // rho u (force corrected)
    const R ux = mc.ux, uy = mc.uy, uz = mc.uz;
    const R rxx = jx * ux, ryy = jy * uy, rzz = jz * uz;
    const R ruu = rxx + ryy + rzz;
    const R txx = R(2) * rxx - ryy - rzz;
    const R tww = ryy - rzz;

    // m - m^eq; the rest weights contribute -11 to e and 3 to eps (m^eq at
    // rho = 1, u = 0), hence the drho terms.
    const R ne_e = (R(-30) * f[0] - R(11) * sax + R(8) * sdg) + R(11) * mc.drho - R(19) * ruu;
    const R ne_eps = (R(12) * f[0] - R(4) * sax + sdg) - R(3) * mc.drho + R(5.5) * ruu;
    const R ne_pxx = (R(2) * s1 - s3 - s5 + pxy + pxz - R(2) * pyz) - txx;
    const R ne_qxx = (R(-4) * s1 + R(2) * (s3 + s5) + pxy + pxz - R(2) * pyz) + R(0.5) * txx;
    const R ne_pww = (s3 - s5 + pxy - pxz) - tww;
    const R ne_qww = (R(-2) * s3 + R(2) * s5 + pxy - pxz) + R(0.5) * tww;
    const R ne_xy = (s7 - s8) - jx * uy;
    const R ne_yz = (s15 - s16) - jy * uz;
    const R ne_xz = (s11 - s12) - jx * uz;
    const R ne_qx = (R(-4) * d1 + d7 - d8 + d11 - d12) + R(2.0 / 3.0) * jx;
    const R ne_qy = (R(-4) * d3 + d7 + d8 + d15 - d16) + R(2.0 / 3.0) * jy;
    const R ne_qz = (R(-4) * d5 + d11 + d12 + d15 + d16) + R(2.0 / 3.0) * jz;
    const R ne_mx = d7 - d8 - d11 + d12;
    const R ne_my = -d7 - d8 + d15 - d16;
    const R ne_mz = d11 + d12 - d15 - d16;

    // dm_k = -s_k (m_k - m^eq_k) + (1 - s_k/2) (M F~)_k with F = (0, 0, F_z);
    // the conserved rows give dm = 0 (rho) and F (momentum).  Divided by |M_k|^2.
    const R sa = c.s_a, sb = c.s_b;
    const R ha = R(1) - R(0.5) * sa, hb = R(1) - R(0.5) * sb;
    const R Fz = mc.Fz, uF = uz * Fz;
    const R a_e = (ha * R(38) * uF - sa * ne_e) * R(1.0 / 2394.0);
    const R a_eps = (-ha * R(11) * uF - sa * ne_eps) * R(1.0 / 252.0);
    const R a_pxx = (-ha * R(2) * uF - sa * ne_pxx) * R(1.0 / 36.0);
    const R a_qxx = (ha * uF - sa * ne_qxx) * R(1.0 / 72.0);
    const R a_pww = (-ha * R(2) * uF - sa * ne_pww) * R(1.0 / 12.0);
    const R a_qww = (ha * uF - sa * ne_qww) * R(1.0 / 24.0);
    const R a_xy = -sa * ne_xy * R(0.25);
    const R a_yz = (ha * uy * Fz - sa * ne_yz) * R(0.25);
    const R a_xz = (ha * ux * Fz - sa * ne_xz) * R(0.25);
    const R a_jz = Fz * R(0.1);
    const R a_qx = -sb * ne_qx * R(1.0 / 40.0);
    const R a_qy = -sb * ne_qy * R(1.0 / 40.0);
    const R a_qz = (-hb * R(2.0 / 3.0) * Fz - sb * ne_qz) * R(1.0 / 40.0);
    const R a_mx = -sb * ne_mx * R(0.125);
    const R a_my = -sb * ne_my * R(0.125);
    const R a_mz = -sb * ne_mz * R(0.125);

    // even part (same for i and opp(i)) ...
    const R Eax = R(-11) * a_e - R(4) * a_eps;
    const R Ex = Eax + R(2) * a_pxx - R(4) * a_qxx;
    const R Eyz = Eax - a_pxx + R(2) * a_qxx;
    const R Ey = Eyz + a_pww - R(2) * a_qww;
    const R Ez = Eyz - a_pww + R(2) * a_qww;
    const R Dc = R(8) * a_e + a_eps;
    const R Pxy = Dc + a_pxx + a_qxx + a_pww + a_qww;
    const R Pxz = Dc + a_pxx + a_qxx - a_pww - a_qww;
    const R Pyz = Dc - R(2) * (a_pxx + a_qxx);
    // ... and odd part (sign flips for opp(i))
    const R Ox = R(-4) * a_qx;
    const R Oy = R(-4) * a_qy;
    const R Oz = a_jz - R(4) * a_qz;
    const R cx = a_qx, cy = a_qy, cz = a_jz + a_qz;
    const R O7 = cx + cy + a_mx - a_my;
    const R O8 = -cx + cy - a_mx - a_my;
    const R O11 = cx + cz - a_mx + a_mz;
    const R O12 = -cx + cz + a_mx + a_mz;
    const R O15 = cy + cz + a_my - a_mz;
    const R O16 = -cy + cz - a_my - a_mz;

    f[0] += R(-30) * a_e + R(12) * a_eps;
    f[1] += Ex + Ox;
    f[2] += Ex - Ox;
    f[3] += Ey + Oy;
    f[4] += Ey - Oy;
    f[5] += Ez + Oz;
    f[6] += Ez - Oz;
    f[7] += Pxy + a_xy + O7;
    f[10] += Pxy + a_xy - O7;
    f[8] += Pxy - a_xy + O8;
    f[9] += Pxy - a_xy - O8;
    f[11] += Pxz + a_xz + O11;
    f[14] += Pxz + a_xz - O11;
    f[12] += Pxz - a_xz + O12;
    f[13] += Pxz - a_xz - O12;
    f[15] += Pyz + a_yz + O15;
    f[18] += Pyz + a_yz - O15;
    f[16] += Pyz - a_yz + O16;
    f[17] += Pyz - a_yz - O16;

    // D3Q7: n = N g, n^eq = (T, uT, vT, wT, a_T T, 0, 0), Q = diag(0, q_k x3, q_e, q_nu x2)
    const R T = mc.T;
    const R n1 = h[1] - h[2], n2 = h[3] - h[4], n3 = h[5] - h[6];
    const R p1 = h[1] + h[2], p2 = h[3] + h[4], p3 = h[5] + h[6];
    const R n4 = T - R(7) * h[0];
    const R n5 = R(2) * p1 - p2 - p3;
    const R n6 = p2 - p3;
    const R b1 = -c.q_k * (n1 - ux * T) * R(0.5);
    const R b2 = -c.q_k * (n2 - uy * T) * R(0.5);
    const R b3 = -c.q_k * (n3 - uz * T) * R(0.5);
    const R b4 = -c.q_e * (n4 - c.a_T * T) * R(1.0 / 42.0);
    const R b5 = -c.q_nu * n5 * R(1.0 / 12.0);
    const R b6 = -c.q_nu * n6 * R(0.25);
    const R c1 = b4 + R(2) * b5, c2 = b4 - b5 + b6, c3 = b4 - b5 - b6;
    h[0] += R(-6) * b4;
    h[1] += c1 + b1;
    h[2] += c1 - b1;
    h[3] += c2 + b2;
    h[4] += c2 - b2;
    h[5] += c3 + b3;
    h[6] += c3 - b3;
    return mc;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Observation outputs of a sample step: the planes [rho - 1, u, v, w, T] of
// the pre-collision state in the arithmetic type (N^3 values each, x
// fastest) and the heat that entered through each isothermal wall link during
// the step that produced the state (2 N^2 FP64 values: hot wall, cold wall).
template <class R>
struct ObsOut {
    R *planes;
    double *wall;
    double abb_hot, abb_cold;
};

// Wall heat flux of the last step at an isothermal wall node: the population
// that came back from the wall is g_in = -g_out+ + abb, so abb - 2 g_out+
// equals 2 g_in - abb (Sec. 2.3 anti-bounce-back).  h: pre-collision g.
template <int CELL, class R>
__device__ __forceinline__ void write_wall_flux(const ObsOut<R> &o, const Geo &g, const Node &d,
                                                const R h[kQG]) {
    if constexpr (CELL == LBM_SIDE_HEATED) {
        const uint64_t w2 = d.y + static_cast<uint64_t>(g.N) * d.z;
        if (d.x == 0) o.wall[w2] = 2.0 * static_cast<double>(h[1]) - o.abb_hot;
        if (d.x == g.N - 1) o.wall[g.N2 + w2] = 2.0 * static_cast<double>(h[2]) - o.abb_cold;
    } else {
        const uint64_t w2 = d.x + static_cast<uint64_t>(g.N) * d.y;
        if (d.z == 0) o.wall[w2] = 2.0 * static_cast<double>(h[5]) - o.abb_hot;
        if (d.z == g.N - 1) o.wall[g.N2 + w2] = 2.0 * static_cast<double>(h[6]) - o.abb_cold;
    }
}

template <class R>
__device__ __forceinline__ void write_planes(const ObsOut<R> &o, const Geo &g, const Node &d,
                                             const Macro<R> &m) {
    const uint64_t V = static_cast<uint64_t>(g.N2) * g.N;
    // plain stores: streaming ones cost the 257^3 FP32 sample step 33 us more
    o.planes[d.n] = m.drho;
    o.planes[V + d.n] = m.ux;
    o.planes[2 * V + d.n] = m.uy;
    o.planes[3 * V + d.n] = m.uz;
    o.planes[4 * V + d.n] = m.T;
}

// One coupled time step of every node.  OBS (sample steps only): also write
// the observation planes of the pre-collision state from the registers, so
// that the observables need no second pass over the populations.
template <class C, int CELL, bool SW, bool OBS>
__global__ __launch_bounds__(256) void k_step(typename C::S *__restrict__ pop, Geo g,
                                              Coef<typename C::R> c, ObsOut<typename C::R> o) {
    using R = typename C::R;
    Node d;
    if (!node_of(g, d)) return;
    R f[kQF], h[kQG];
    gather<C, CELL, SW>(pop, g, d, c, f, h);
    if constexpr (OBS) write_wall_flux<CELL>(o, g, d, h);
    const Macro<R> m = collide(f, h, c);
    if constexpr (OBS) write_planes(o, g, d, m);
    scatter<C, CELL, SW>(pop, g, d, c, f, h);
}

// One step of many cavities in one launch.  Logical block lb belongs to the
// last cavity whose first block is <= lb (binary search over the descriptor
// table, wave-uniform); retired cavities' blocks return at once.  All
// cavities of a batch share the storage parity.
template <class C, bool SW>
__global__ __launch_bounds__(256) void k_step_batch(const CavityDesc<typename C::R> *__restrict__ tab,
                                                    int K) {
    using R = typename C::R;
    const uint32_t lb = xcd_order();
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].start <= lb) lo = mid;
        else hi = mid - 1;
    }
    const CavityDesc<R> &D = tab[lo];
    if (!D.active) return;
    Node d;
    if (!node_at(D.g, lb - D.start, d)) return;
    typename C::S *pop = static_cast<typename C::S *>(D.pop);
    R f[kQF], h[kQG];
    if (D.cell == LBM_SIDE_HEATED) {
        gather<C, LBM_SIDE_HEATED, SW>(pop, D.g, d, D.c, f, h);
        collide(f, h, D.c);
        scatter<C, LBM_SIDE_HEATED, SW>(pop, D.g, d, D.c, f, h);
    } else {
        gather<C, LBM_RAYLEIGH_BENARD, SW>(pop, D.g, d, D.c, f, h);
        collide(f, h, D.c);
        scatter<C, LBM_RAYLEIGH_BENARD, SW>(pop, D.g, d, D.c, f, h);
    }
}

// Trilinear resampling of the fields (u, v, w, T) of an N^3 lattice onto M^3
// node-centred points, FP32 output [4][M^3].  Per axis the samples are the
// node values at (i + 1/2)/N and, beyond the first and last node, the wall
// value at 0 or 1: u = v = w = 0 on every wall, T = T_w on the isothermal
// walls; along the adiabatic axes T is held at the nearest node.
__global__ __launch_bounds__(256) void k_resample(int N, int cell, double T_hot, double T_cold,
                                                  const double *__restrict__ macro, int M,
                                                  float *__restrict__ out) {
    const uint64_t M3 = static_cast<uint64_t>(M) * M * M;
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= M3) return;
    const int c3[3] = {static_cast<int>(t % M), static_cast<int>((t / M) % M),
                       static_cast<int>(t / (static_cast<uint64_t>(M) * M))};
    // per axis: the two samples (node index, or -1 / N for the low / high wall)
    int i0[3], i1[3];
    double w1[3];
    for (int a = 0; a < 3; ++a) {
        const double sidx = (c3[a] + 0.5) * N / M - 0.5;   // position in node units
        int k = static_cast<int>(floor(sidx));
        double fr = sidx - k;
        if (k < 0) {            // between the low wall (-1/2) and node 0
            i0[a] = -1; i1[a] = 0; w1[a] = (sidx + 0.5) / 0.5;
        } else if (k >= N - 1) {  // between node N-1 and the high wall (N - 1/2)
            i0[a] = N - 1; i1[a] = N; w1[a] = (sidx - (N - 1)) / 0.5;
        } else {
            i0[a] = k; i1[a] = k + 1; w1[a] = fr;
        }
    }
    const uint64_t V = static_cast<uint64_t>(N) * N * N;
    const int iso = cell == LBM_SIDE_HEATED ? 0 : 2;
    for (int q = 0; q < 4; ++q) {
        const double *phi = macro + (1 + q) * V;
        double acc = 0.0;
        for (int corner = 0; corner < 8; ++corner) {
            int idx[3];
            double wt = 1.0;
            bool wall = false;
            double wall_value = 0.0;
            for (int a = 0; a < 3; ++a) {
                const bool hi_side = (corner >> a) & 1;
                int k = hi_side ? i1[a] : i0[a];
                wt *= hi_side ? w1[a] : 1.0 - w1[a];
                if (k < 0 || k >= N) {
                    if (q < 3) {                 // velocity: no slip on every wall
                        wall = true;
                        wall_value = 0.0;
                    } else if (a == iso) {       // temperature: isothermal wall
                        wall = true;
                        wall_value = k < 0 ? T_hot : T_cold;
                    } else {                     // adiabatic axis: nearest node
                        k = k < 0 ? 0 : N - 1;
                    }
                }
                idx[a] = k;
            }
            if (wt == 0.0) continue;
            const double val = wall ? wall_value
                                    : phi[idx[0] + static_cast<uint64_t>(N) * (idx[1] + static_cast<uint64_t>(N) * idx[2])];
            acc += wt * val;
        }
        out[q * M3 + t] = static_cast<float>(acc);
    }
}

// f = f^eq(1, u) (Sec. 2.2), g = g^eq(T, u) (Sec. 2.3), canonical slots.
template <class C>
__global__ __launch_bounds__(256) void k_init(typename C::S *__restrict__ pop, Geo g,
                                              Coef<typename C::R> c, const double *__restrict__ uvwT,
                                              double wT0, double wT1, double aT) {
    Node d;
    if (!node_of(g, d)) return;
    const uint64_t V = static_cast<uint64_t>(g.N2) * g.N;
    const double u = uvwT[d.n], v = uvwT[V + d.n], w = uvwT[2 * V + d.n], T = uvwT[3 * V + d.n];
    const double uu = u * u + v * v + w * w;
    using R = typename C::R;
    const View vw = view_of(pop, g, d);
#pragma unroll
    for (int i = 0; i < kQF; ++i) {
        const double eu = EX[i] * u + EY[i] * v + EZ[i] * w;
        const double fdev = wrest(i) * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        st_f<C>(vw, slot<C>(vw, g, i, 0, 0, 0), static_cast<R>(fdev), c);
    }
    const double k = 21.0 / (6.0 + aT);
#pragma unroll
    for (int j = 0; j < kQG; ++j) {
        const double eu = GX[j] * u + GY[j] * v + GZ[j] * w;
        const double gv = (j == 0 ? wT0 : wT1) * T * (1.0 + k * eu);
        st_g<C>(vw, slot<C>(vw, g, kQF + j, 0, 0, 0), j, static_cast<R>(gv), c);
    }
}

template <class C>
__global__ __launch_bounds__(256) void k_set_pop(typename C::S *__restrict__ pop, Geo g,
                                                 Coef<typename C::R> c,
                                                 const double *__restrict__ in) {
    Node d;
    if (!node_of(g, d)) return;
    const uint64_t V = static_cast<uint64_t>(g.N2) * g.N;
    using R = typename C::R;
    const View vw = view_of(pop, g, d);
#pragma unroll
    for (int i = 0; i < kQF; ++i)
        st_f<C>(vw, slot<C>(vw, g, i, 0, 0, 0), static_cast<R>(in[i * V + d.n] - wrest(i)), c);
#pragma unroll
    for (int j = 0; j < kQG; ++j)
        st_g<C>(vw, slot<C>(vw, g, kQF + j, 0, 0, 0), j, static_cast<R>(in[(kQF + j) * V + d.n]), c);
}

template <class C, int CELL, bool SW>
__global__ __launch_bounds__(256) void k_get_pop(const typename C::S *__restrict__ pop, Geo g,
                                                 Coef<typename C::R> c, double *__restrict__ out) {
    using R = typename C::R;
    Node d;
    if (!node_of(g, d)) return;
    const uint64_t V = static_cast<uint64_t>(g.N2) * g.N;
    R f[kQF], h[kQG];
    gather<C, CELL, SW>(pop, g, d, c, f, h);
#pragma unroll
    for (int i = 0; i < kQF; ++i) out[i * V + d.n] = static_cast<double>(f[i]) + wrest(i);
#pragma unroll
    for (int j = 0; j < kQG; ++j) out[(kQF + j) * V + d.n] = static_cast<double>(h[j]);
}

// FP64 macro planes [rho, u, v, w, T] of the current state (field output,
// residual, diagnostics).
template <class C, int CELL, bool SW>
__global__ __launch_bounds__(256) void k_macro(const typename C::S *__restrict__ pop, Geo g,
                                               Coef<typename C::R> c, double *__restrict__ macro) {
    using R = typename C::R;
    Node d;
    if (!node_of(g, d)) return;
    const uint64_t V = static_cast<uint64_t>(g.N2) * g.N;
    R f[kQF], h[kQG];
    gather<C, CELL, SW>(pop, g, d, c, f, h);
    const Macro<R> m = macros(f, h, c);
    macro[d.n] = 1.0 + static_cast<double>(m.drho);
    macro[V + d.n] = m.ux;
    macro[2 * V + d.n] = m.uy;
    macro[3 * V + d.n] = m.uz;
    macro[4 * V + d.n] = m.T;
}

// Observation planes and wall flux of the current state outside a step (the
// same values the OBS step kernel writes for the state it starts from).
template <class C, int CELL, bool SW>
__global__ __launch_bounds__(256) void k_obs_planes(const typename C::S *__restrict__ pop, Geo g,
                                                    Coef<typename C::R> c, ObsOut<typename C::R> o) {
    using R = typename C::R;
    Node d;
    if (!node_of(g, d)) return;
    R f[kQF], h[kQG];
    gather<C, CELL, SW>(pop, g, d, c, f, h);
    if (o.wall) write_wall_flux<CELL>(o, g, d, h);
    write_planes(o, g, d, macros(f, h, c));
}

// ---------------------------------------------------------------------------
// Reductions (FP64, fixed order: deterministic)
// ---------------------------------------------------------------------------
template <int K, bool MAX0>
__device__ __forceinline__ void block_reduce_to(double (&v)[K], double *__restrict__ out) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double t = __shfl_down(v[k], o, 64);
            v[k] = (MAX0 && k == 0) ? fmax(v[k], t) : v[k] + t;
        }
    __shared__ double sm[kRedBlock / 64][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sm[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
        const int k = threadIdx.x;
        double s = sm[0][k];
        for (int w = 1; w < kRedBlock / 64; ++w) s = (MAX0 && k == 0) ? fmax(s, sm[w][k]) : s + sm[w][k];
        out[k] = s;
    }
}

// Derivative along one axis at a node with index k on that axis from the
// values at k-1, k and k+1 (lo and hi unused where they would lie outside):
// central inside; at the first node next to a wall the quadratic through the
// wall value (w_lo or w_hi) half a cell away and the two nearest nodes, or
// with a mirror node (dphi/dn = 0) at an adiabatic wall.
template <class A>
__device__ __forceinline__ A dfd(A lo, A c, A hi, int k, int N, A w_lo, A w_hi, bool mirror) {
    if (k > 0 && k < N - 1) return A(0.5) * (hi - lo);
    if (k == 0) return mirror ? A(0.5) * (hi - c) : A(-4.0 / 3.0) * w_lo + c + hi * A(1.0 / 3.0);
    return mirror ? A(0.5) * (c - lo) : A(4.0 / 3.0) * w_hi - c - lo * A(1.0 / 3.0);
}

struct ObsArgs {
    double nu, kappa, T_hot, T_cold;
};

// z-planes per block of the observable reduction, and the in-plane nodes a
// block adds up (62 of the 64 lanes of each of its 4 waves).
constexpr int kObsZ = 16;
constexpr int kObsTile = 4 * 62;

// The value held by lane - 1 (from_left) or lane + 1 (from_right) of the
// wave: a DPP move across the whole 64-lane wave, no LDS traffic.  Lanes 0
// and 63 receive 0 (they are halo lanes whose terms are not added).
__device__ __forceinline__ int dpp_from_left(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_from_right(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}
template <class P>
__device__ __forceinline__ P from_left(P v) {
    if constexpr (sizeof(P) == 4) {
        return __int_as_float(dpp_from_left(__float_as_int(v)));
    } else {
        const long long b = __double_as_longlong(v);
        const uint32_t lo = static_cast<uint32_t>(dpp_from_left(static_cast<int>(b)));
        const long long hi = dpp_from_left(static_cast<int>(b >> 32));
        return __longlong_as_double((hi << 32) | lo);
    }
}
template <class P>
__device__ __forceinline__ P from_right(P v) {
    if constexpr (sizeof(P) == 4) {
        return __int_as_float(dpp_from_right(__float_as_int(v)));
    } else {
        const long long b = __double_as_longlong(v);
        const uint32_t lo = static_cast<uint32_t>(dpp_from_right(static_cast<int>(b)));
        const long long hi = dpp_from_right(static_cast<int>(b >> 32));
        return __longlong_as_double((hi << 32) | lo);
    }
}

// What a lane of the observable reduction holds of one plane z: (u, v, w, T)
// at its node and at y -+ 1, rho - 1, and (side-heated cell) the two wall
// fluxes of its row (y, z).
template <int CELL, class P>
struct ObsPlane {
    P c[4], yl[4], yh[4], d;
    double wh, wc;
};

// Loads of plane zc for in-plane node rc = x + N y (rows ryl, ryh for y -+ 1), every one
// issued by every lane at an address clamped into the arrays: a load under a
// branch would make the compiler wait for all loads in flight before its value
// is used, which serialises the planes.  Values at clamped addresses are not
// used.  wsrc: the wall fluxes, or (before the first step) any array of at
// least 2 N^2 doubles, whose values are then discarded.
template <int CELL, class P>
__device__ __forceinline__ void obs_load(ObsPlane<CELL, P> &o, const P *const (&F)[4],
                                         const P *D, const double *wsrc, int zc, int N, int N2,
                                         int rc, int y, int ryl, int ryh) {
    const uint64_t zo = static_cast<uint64_t>(zc) * N2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        o.c[q] = F[q][zo + rc];
        o.yl[q] = F[q][zo + ryl];
        o.yh[q] = F[q][zo + ryh];
    }
    o.d = D[zo + rc];
    if constexpr (CELL == LBM_SIDE_HEATED) {
        const uint64_t w = y + static_cast<uint64_t>(N) * zc;
        o.wh = wsrc[w];
        o.wc = wsrc[static_cast<uint64_t>(N2) + w];
    }
}

// A node's terms of plane z, added to the FP64 sums v: lo = (u, v, w, T) at
// z - 1, cur = plane z, hi = (u, v, w, T) at z + 1.  The differences and
// products are formed in P.  Where a neighbour would lie outside the cell its
// value is not used (dfd takes the wall formula there).
template <int CELL, class P>
__device__ __forceinline__ void obs_terms(double (&v)[LBM_NRAW], const P (&lo)[4],
                                          const ObsPlane<CELL, P> &cur, const P (&hi)[4],
                                          int x, int y, int z, int N, int N2, bool live,
                                          const double *wall, const ObsArgs &a) {
    constexpr int iso = CELL == LBM_SIDE_HEATED ? 0 : 2;
    const P nu = static_cast<P>(a.nu), kappa = static_cast<P>(a.kappa);
    const P Th = static_cast<P>(a.T_hot), Tc = static_cast<P>(a.T_cold);
    // r - 1 and r + 1 are the neighbouring lanes' own values (every lane
    // takes part in the moves)
    P xl[4], xh[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        xl[q] = from_left(cur.c[q]);
        xh[q] = from_right(cur.c[q]);
    }
    if (!live) return;
    const P *c = cur.c, *yl = cur.yl, *yh = cur.yh;
    P du[3][3];   // du[i][j] = d_i u_j
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        du[0][j] = dfd<P>(xl[j], c[j], xh[j], x, N, P(0), P(0), false);
        du[1][j] = dfd<P>(yl[j], c[j], yh[j], y, N, P(0), P(0), false);
        du[2][j] = dfd<P>(lo[j], c[j], hi[j], z, N, P(0), P(0), false);
    }
    const P dT[3] = {dfd<P>(xl[3], c[3], xh[3], x, N, Th, Tc, iso != 0),
                     dfd<P>(yl[3], c[3], yh[3], y, N, Th, Tc, true),
                     dfd<P>(lo[3], c[3], hi[3], z, N, Th, Tc, iso != 2)};
    P eu = P(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const P sij = du[i][j] + du[j][i];
            eu += sij * sij;
        }
    const P u = c[0], vv = c[1], w = c[2], Tn = c[3];
    const P dr = cur.d;
    const P div = du[0][0] + du[1][1] + du[2][2];
    v[LBM_RAW_U2] += static_cast<double>(u * u + vv * vv + w * w);
    v[LBM_RAW_W2] += static_cast<double>(w * w);
    v[LBM_RAW_WT] += static_cast<double>(w * Tn);
    v[LBM_RAW_UT] += static_cast<double>(u * Tn);
    v[LBM_RAW_EPS_U] += static_cast<double>(P(0.5) * nu * eu);
    v[LBM_RAW_EPS_T] += static_cast<double>(kappa * (dT[0] * dT[0] + dT[1] * dT[1] + dT[2] * dT[2]));
    v[LBM_RAW_DRHO2] += static_cast<double>(dr * dr);
    v[LBM_RAW_T] += static_cast<double>(Tn);
    v[LBM_RAW_DRHO] += static_cast<double>(dr);
    v[LBM_RAW_DIV2] += static_cast<double>(div * div);
    const int k = iso == 0 ? x : z;
    if (k == 0 || k == N - 1) {
        const bool hot = k == 0;
        const P T_in = iso == 0 ? (hot ? xh[3] : xl[3]) : (hot ? hi[3] : lo[3]);
        double fh = 0.0, fc = 0.0;
        if (wall) {
            if constexpr (CELL == LBM_SIDE_HEATED) {
                fh = cur.wh;
                fc = cur.wc;
            } else {
                fh = wall[x + static_cast<uint64_t>(N) * y];
                fc = wall[N2 + x + static_cast<uint64_t>(N) * y];
            }
        }
        // both walls' sums take a select: a sum chosen by a run-time index
        // would move the sums to scratch memory
        const P gh = -(P(-8) * Th + P(9) * Tn - T_in) * P(1.0 / 3.0);
        const P gc = (P(8) * Tc - P(9) * Tn + T_in) * P(1.0 / 3.0);
        v[LBM_RAW_FLUX_HOT] += hot ? fh : 0.0;
        v[LBM_RAW_GRAD_HOT] += hot ? static_cast<double>(gh) : 0.0;
        v[LBM_RAW_FLUX_COLD] += hot ? 0.0 : fc;
        v[LBM_RAW_GRAD_COLD] += hot ? 0.0 : static_cast<double>(gc);
    }
}

// Waves per SIMD the observable reduction is compiled for: 4 (128 VGPRs) for
// the Rayleigh-Benard cell with FP32 planes, 3-8% faster than the 3 waves its
// registers would otherwise allow; otherwise whatever the registers allow
// (held to 128 VGPRs the side-heated cell spills 16 bytes a lane, which
// costs more than the extra wave gains, and FP64 planes spill heavily).
template <int CELL, class P>
constexpr int kObsWaves = (sizeof(P) == 4 && CELL == LBM_RAYLEIGH_BENARD) ? 4 : 1;

// Observable partial sums from the observation planes [rho - 1, u, v, w, T]
// (type P; the differences and products are formed in P, each node's terms
// added to FP64 sums) and the wall flux (NULL before the first step).  A
// block takes kObsTile consecutive in-plane nodes r and marches them through
// ZC planes: the values at z - 1, z and z + 1 stay in registers, the
// neighbours r +- 1 come from the neighbouring lanes (each wave's outer lanes
// hold them), r +- N from the lines the block and its neighbours load at the
// same time, so each plane value comes from HBM about once.  Three plane
// buffers rotate through the march, the loads of plane z + 2 issued before
// plane z is worked on, and no buffer with loads in flight is ever copied.
// Logical block lb = chunk * ntile + tile; every block writes one row of
// partials.  At 257^3 in FP32: 108-121 us (195 us with one plane in flight
// and its loads under branches; 618 us with a lane per node, edge loads and
// FP64 differences; 665 us for the earlier pass over FP64 planes).
template <int CELL, class P, int ZC = kObsZ>
__global__ __launch_bounds__(kRedBlock) __attribute__((amdgpu_waves_per_eu(kObsWaves<CELL, P>)))
void k_observe(int N, uint32_t ntile, ObsArgs a,
                                                       const P *__restrict__ pl,
                                                       const double *__restrict__ wall,
                                                       double *__restrict__ part) {
    const uint32_t lb = xcd_order();
    const uint32_t tile = lb % ntile, chunk = lb / ntile;
    const int N2 = N * N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the first and last lane of each wave only carry the values of the
    // neighbours r - 1 and r + 1 of the 62 lanes between them
    const int ri = static_cast<int>(tile) * kObsTile + wave * 62 + lane - 1;
    const bool live = ri >= 0 && ri < N2 && lane >= 1 && lane <= 62;   // adds its node's terms
    const int rc = min(max(ri, 0), N2 - 1);                            // in-bounds node to load
    const int y = rc / N, x = rc - y * N;
    const int ryl = y > 0 ? rc - N : rc, ryh = y < N - 1 ? rc + N : rc;
    double v[LBM_NRAW];
#pragma unroll
    for (int k = 0; k < LBM_NRAW; ++k) v[k] = 0.0;
    const uint64_t V = static_cast<uint64_t>(N2) * N;
    const P *const F[4] = {pl + V, pl + 2 * V, pl + 3 * V, pl + 4 * V};   // u, v, w, T
    // the observation planes hold 5 N^3 values of at least 4 bytes, more than
    // the 2 N^2 doubles the wall fluxes take
    const double *wsrc = wall ? wall : reinterpret_cast<const double *>(pl);
    const int z0 = static_cast<int>(chunk) * ZC, z1 = min(N, z0 + ZC);
    const int mid_lo = (N - 1) / 2, mid_hi = N / 2;
    const double wm = (y == mid_lo || y == mid_hi) ? (mid_lo == mid_hi ? 1.0 : 0.5) : 0.0;
    ObsPlane<CELL, P> A, B, C;
    P lo[4];
    {
        const uint64_t zl = static_cast<uint64_t>(max(z0 - 1, 0)) * N2;
#pragma unroll
        for (int q = 0; q < 4; ++q) lo[q] = F[q][zl + rc];
    }
    obs_load(A, F, pl, wsrc, z0, N, N2, rc, y, ryl, ryh);
    obs_load(B, F, pl, wsrc, min(z0 + 1, N - 1), N, N2, rc, y, ryl, ryh);
    // planes z, z + 1 and z + 2 rotate through A, B and C
    int z = z0;
#pragma unroll 1
    while (true) {
        obs_load(C, F, pl, wsrc, min(z + 2, N - 1), N, N2, rc, y, ryl, ryh);
        obs_terms(v, lo, A, B.c, x, y, z, N, N2, live, wall, a);
#pragma unroll
        for (int q = 0; q < 4; ++q) lo[q] = A.c[q];
        if (++z >= z1) break;
        obs_load(A, F, pl, wsrc, min(z + 2, N - 1), N, N2, rc, y, ryl, ryh);
        obs_terms(v, lo, B, C.c, x, y, z, N, N2, live, wall, a);
#pragma unroll
        for (int q = 0; q < 4; ++q) lo[q] = B.c[q];
        if (++z >= z1) break;
        obs_load(B, F, pl, wsrc, min(z + 2, N - 1), N, N2, rc, y, ryl, ryh);
        obs_terms(v, lo, C, A.c, x, y, z, N, N2, live, wall, a);
#pragma unroll
        for (int q = 0; q < 4; ++q) lo[q] = C.c[q];
        if (++z >= z1) break;
    }
    // the mid-line weight depends on y only, which a thread keeps (0, 1/2 or
    // 1: the scaling is exact)
    v[LBM_RAW_FLUX_HOT_MID] = wm * v[LBM_RAW_FLUX_HOT];
    v[LBM_RAW_GRAD_HOT_MID] = wm * v[LBM_RAW_GRAD_HOT];
    v[LBM_RAW_FLUX_COLD_MID] = wm * v[LBM_RAW_FLUX_COLD];
    v[LBM_RAW_GRAD_COLD_MID] = wm * v[LBM_RAW_GRAD_COLD];
    block_reduce_to<LBM_NRAW, false>(v, part + static_cast<uint64_t>(lb) * kNPart);
}

// First level of the partial reduction: block b folds rows [b*per, (b+1)*per)
// of `in` into row b of `out`, in a fixed order (sum, or max for column 0
// when MAX0).
template <int K, bool MAX0>
__global__ __launch_bounds__(kRedBlock) void k_fold_rows(const double *__restrict__ in,
                                                         uint32_t nrows, uint32_t per,
                                                         double *__restrict__ out) {
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    const uint32_t lo = blockIdx.x * per, hi = min(nrows, lo + per);
    for (uint32_t b = lo + threadIdx.x; b < hi; b += kRedBlock)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double x = in[static_cast<uint64_t>(b) * kNPart + k];
            v[k] = (MAX0 && k == 0) ? fmax(v[k], x) : v[k] + x;
        }
    block_reduce_to<K, MAX0>(v, out + static_cast<uint64_t>(blockIdx.x) * kNPart);
}

// Sum the folded rows in a fixed order and scale to means.
__global__ __launch_bounds__(kRedBlock) void k_finalize_obs(const double *__restrict__ part,
                                                            uint32_t nblk, double inv_V,
                                                            double inv_A, double inv_L,
                                                            double *__restrict__ res,
                                                            int accumulate) {
    double v[LBM_NRAW];
#pragma unroll
    for (int k = 0; k < LBM_NRAW; ++k) v[k] = 0.0;
    for (uint32_t b = threadIdx.x; b < nblk; b += kRedBlock)
#pragma unroll
        for (int k = 0; k < LBM_NRAW; ++k) v[k] += part[static_cast<uint64_t>(b) * kNPart + k];
    __shared__ double tot[LBM_NRAW];
    block_reduce_to<LBM_NRAW, false>(v, tot);
    __syncthreads();
    if (threadIdx.x < LBM_NRAW) {
        const int k = threadIdx.x;
        const double s = (k <= LBM_RAW_FLUX_COLD || k == LBM_RAW_GRAD_HOT || k == LBM_RAW_GRAD_COLD)
                             ? inv_A
                             : (k < LBM_RAW_U2 ? inv_L : inv_V);
        const double m = tot[k] * s;
        res[kResCur + k] = m;
        if (accumulate) res[kResAcc + k] += m;
    }
    if (threadIdx.x == 0 && accumulate) res[kResAcc + LBM_NRAW] += 1.0;
}

// Maximum of u on the line x = y = 1/2 (over z) and of w on y = z = 1/2 (over
// x), one block per line; for even N the two central nodes are averaged.
// Ties go to the smaller index.  res[kResPeak + 0..3] = u_max, k_u, w_max, k_w.
__global__ __launch_bounds__(kRedBlock) void k_centerline(int N, const double *__restrict__ macro,
                                                          double *__restrict__ res) {
    const uint64_t V = static_cast<uint64_t>(N) * N * N, N2 = static_cast<uint64_t>(N) * N;
    const int lo = (N - 1) / 2, hi = N / 2;
    const bool horiz = blockIdx.x == 1;             // 0: u along z, 1: w along x
    const double *phi = macro + (horiz ? 3 : 1) * V;
    double best = -INFINITY;
    int arg = 0;
    for (int k = threadIdx.x; k < N; k += kRedBlock) {
        double v;
        if (!horiz)  // x = y = centre, varying z
            v = 0.25 * (phi[lo + N * lo + N2 * k] + phi[hi + N * lo + N2 * k] +
                        phi[lo + N * hi + N2 * k] + phi[hi + N * hi + N2 * k]);
        else         // y = z = centre, varying x
            v = 0.25 * (phi[k + N * lo + N2 * lo] + phi[k + N * hi + N2 * lo] +
                        phi[k + N * lo + N2 * hi] + phi[k + N * hi + N2 * hi]);
        if (v > best) {
            best = v;
            arg = k;
        }
    }
    __shared__ double sv[kRedBlock];
    __shared__ int si[kRedBlock];
    sv[threadIdx.x] = best;
    si[threadIdx.x] = arg;
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double a = sv[threadIdx.x], b = sv[threadIdx.x + w];
            const int ia = si[threadIdx.x], ib = si[threadIdx.x + w];
            if (b > a || (b == a && ib < ia)) {
                sv[threadIdx.x] = b;
                si[threadIdx.x] = ib;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res[kResPeak + 2 * blockIdx.x] = sv[0];
        res[kResPeak + 2 * blockIdx.x + 1] = si[0];
    }
}

// Plane sums for the Nusselt profile across the cell: for node plane k of
// the isothermal axis a (x side-heated, z Rayleigh-Benard), row group g adds
// u_a T and d_a T (the differences of the observables) over its share of the
// plane into part[g][2k] and part[g][2k + 1].  Side-heated: a thread owns one
// x and walks the rows (y, z) = g, g + kProfG, ...; Rayleigh-Benard: block
// (z, g) walks r = g 256 + t, stepping kProfG 256, and reduces.
constexpr int kProfG = kProfGroups;

template <int CELL>
__global__ __launch_bounds__(kRedBlock) void k_profile(int N, const double *__restrict__ macro,
                                                       double T_hot, double T_cold,
                                                       double *__restrict__ part) {
    const uint32_t N2 = static_cast<uint32_t>(N) * N;
    const uint64_t V = static_cast<uint64_t>(N2) * N;
    const double *T = macro + 4 * V;
    const uint32_t grp = blockIdx.y;
    double *out = part + static_cast<uint64_t>(grp) * 2 * N;
    if constexpr (CELL == LBM_SIDE_HEATED) {
        const int x = blockIdx.x * kRedBlock + threadIdx.x;
        if (x >= N) return;
        const double *ua = macro + V;
        double conv = 0.0, cond = 0.0;
        for (uint32_t row = grp; row < N2; row += kProfG) {
            const uint64_t n = x + static_cast<uint64_t>(N) * row;
            const double t = T[n];
            conv += ua[n] * t;
            cond += dfd(x > 0 ? T[n - 1] : 0.0, t, x < N - 1 ? T[n + 1] : 0.0, x, N, T_hot, T_cold, false);
        }
        out[2 * x] = conv;
        out[2 * x + 1] = cond;
    } else {
        const int z = blockIdx.x;
        const double *ua = macro + 3 * V;
        double v[2] = {0.0, 0.0};
        for (uint32_t r = grp * kRedBlock + threadIdx.x; r < N2; r += kProfG * kRedBlock) {
            const uint64_t n = r + static_cast<uint64_t>(N2) * z;
            const double t = T[n];
            v[0] += ua[n] * t;
            v[1] += dfd(z > 0 ? T[n - N2] : 0.0, t, z < N - 1 ? T[n + N2] : 0.0, z, N, T_hot, T_cold, false);
        }
        block_reduce_to<2, false>(v, out + 2 * z);
    }
}

// Nu(k) = H/(kappa dT) (<u_a T>_k - kappa <d_a T>_k) from the group sums,
// added in a fixed order.
__global__ __launch_bounds__(kRedBlock) void k_profile_final(int N, const double *__restrict__ part,
                                                             double scale, double kappa,
                                                             double *__restrict__ nu) {
    const double inv_A = 1.0 / (static_cast<double>(N) * N);
    for (int k = threadIdx.x; k < N; k += kRedBlock) {
        double conv = 0.0, cond = 0.0;
        for (int g = 0; g < kProfG; ++g) {
            conv += part[static_cast<uint64_t>(g) * 2 * N + 2 * k];
            cond += part[static_cast<uint64_t>(g) * 2 * N + 2 * k + 1];
        }
        nu[k] = scale * (conv * inv_A - kappa * cond * inv_A);
    }
}

// Reference copy: one 16-byte streaming load and store per thread over a
// grid that covers the copy (a grid-stride loop only beyond 2^30 blocks).
// Of the copy forms measured on MI355X (grid-stride loops with 1-4 words per
// thread and 2048-16384 blocks, plain or streaming, the runtime's copy) this
// one moved the most: 6.5 TB/s at 1 GiB against 5.1 for hipMemcpyAsync.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                              uint64_t n16) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void k_reset_acc(double *__restrict__ res) {
    if (threadIdx.x <= LBM_NRAW) res[kResAcc + threadIdx.x] = 0.0;
}

// Residual partials (max |dT|, sum |dT|, sum |T_old|, sum |du|, sum |u_old|),
// then the snapshot takes the current state.
__global__ __launch_bounds__(kRedBlock) void k_residual(Geo g, const double *__restrict__ macro,
                                                        double *__restrict__ snap,
                                                        double *__restrict__ part) {
    Node d;
    const bool live = node_of(g, d);
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (live) {
        const uint64_t V = static_cast<uint64_t>(g.N2) * g.N, n = d.n;
        const double T = macro[4 * V + n], Ts = snap[3 * V + n];
        double s = 0.0, so = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double u = macro[(1 + a) * V + n], us = snap[a * V + n];
            s += (u - us) * (u - us);
            so += us * us;
            snap[a * V + n] = u;
        }
        snap[3 * V + n] = T;
        v[0] = fabs(T - Ts);
        v[1] = v[0];
        v[2] = fabs(Ts);
        v[3] = sqrt(s);
        v[4] = sqrt(so);
    }
    const uint32_t b = blockIdx.x;
    block_reduce_to<5, true>(v, part + static_cast<uint64_t>(b) * kNPart);
}

__global__ __launch_bounds__(kRedBlock) void k_finalize_residual(const double *__restrict__ part,
                                                                 uint32_t nblk,
                                                                 double *__restrict__ res) {
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = threadIdx.x; b < nblk; b += kRedBlock)
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const double x = part[static_cast<uint64_t>(b) * kNPart + k];
            v[k] = k == 0 ? fmax(v[k], x) : v[k] + x;
        }
    __shared__ double tot[5];
    block_reduce_to<5, true>(v, tot);
    __syncthreads();
    if (threadIdx.x < 5) res[kResResid + threadIdx.x] = tot[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------
template <class R>
Coef<R> make_coef(const lbm_t *h) {
    const lbm_params &p = h->p;
    Coef<R> c;
    c.s_a = static_cast<R>(p.s_e);
    c.s_b = static_cast<R>(p.s_q);
    c.q_k = static_cast<R>(p.q_k);
    c.q_e = static_cast<R>(p.q_e);
    c.q_nu = static_cast<R>(p.q_nu);
    c.a_T = static_cast<R>(p.a_T);
    c.gbeta = static_cast<R>(p.gbeta);
    c.T0 = static_cast<R>(p.T0);
    c.abb_hot = static_cast<R>((6.0 + p.a_T) / 21.0 * p.T_hot);
    c.abb_cold = static_cast<R>((6.0 + p.a_T) / 21.0 * p.T_cold);
    const bool half = h->storage == LBM_FP16S;
    c.sf = static_cast<R>(half ? 1024.0 : 1.0);
    c.isf = static_cast<R>(half ? 1.0 / 1024.0 : 1.0);
    c.sg = static_cast<R>(1.0);
    c.isg = static_cast<R>(1.0);
    // FP16C cannot hold inf or NaN (it clamps at |f_i - w_i| = 1/4), so a
    // blow-up would go on with clamped values; a density deviation of 0.1,
    // several times what any flow at Mach <= 0.1 reaches, marks it instead
    c.drho_max = static_cast<R>(h->storage == LBM_FP16C ? 0.1 : INFINITY);
    return c;
}

Geo geo_for(const lbm_t *h, int block) {
    Geo g = h->geo;
    g.gx = (g.N2 + block - 1) / block;
    return g;
}

dim3 grid_of(const lbm_t *h, int block) {
    return dim3(geo_for(h, block).gx * h->geo.N, 1, 1);
}

template <class C>
typename C::S *pop_ptr(const lbm_t *h) {
    return reinterpret_cast<typename C::S *>(static_cast<char *>(h->buf) + h->L.off_pop);
}
double *dptr(const lbm_t *h, size_t off) {
    return reinterpret_cast<double *>(static_cast<char *>(h->buf) + off);
}

// Dispatch a functor on the storage codec of the handle.
template <class F>
hipError_t with_codec(const lbm_t *h, F &&fn) {
    switch (h->storage) {
    case LBM_FP64: return fn(CF64{});
    case LBM_FP32: return fn(CF32{});
    case LBM_FP16C: return fn(CF16C{});
    default: return fn(CF16{});
    }
}

template <class R>
ObsOut<R> obs_out(const lbm_t *h) {
    ObsOut<R> o;
    o.planes = reinterpret_cast<R *>(static_cast<char *>(h->buf) + h->L.off_macro);
    o.wall = dptr(h, h->L.off_wall);
    o.abb_hot = (6.0 + h->p.a_T) / 21.0 * h->p.T_hot;
    o.abb_cold = (6.0 + h->p.a_T) / 21.0 * h->p.T_cold;
    return o;
}

template <class C, int CELL, bool SW, bool OBS>
void step_one(const lbm_t *h, hipStream_t s) {
    k_step<C, CELL, SW, OBS><<<grid_of(h, h->block), h->block, lds_cap_bytes(h->waves[SW], h->block), s>>>(
        pop_ptr<C>(h), geo_for(h, h->block), make_coef<typename C::R>(h), obs_out<typename C::R>(h));
}

template <class C, int CELL, bool OBS>
void step_parity(const lbm_t *h, int parity, hipStream_t s) {
    if (parity) step_one<C, CELL, true, OBS>(h, s);
    else step_one<C, CELL, false, OBS>(h, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_step(const lbm_t *h, int parity, bool obs, hipStream_t s) {
    return with_codec(h, [&](auto cd) {
        using C = decltype(cd);
        if (h->p.cell == LBM_SIDE_HEATED) {
            if (obs) step_parity<C, LBM_SIDE_HEATED, true>(h, parity, s);
            else step_parity<C, LBM_SIDE_HEATED, false>(h, parity, s);
        } else {
            if (obs) step_parity<C, LBM_RAYLEIGH_BENARD, true>(h, parity, s);
            else step_parity<C, LBM_RAYLEIGH_BENARD, false>(h, parity, s);
        }
        return hipGetLastError();
    });
}

static_assert(sizeof(CavityDesc<double>) <= kMaxDescBytes, "descriptor table slot too small");
static_assert(sizeof(CavityDesc<float>) <= kMaxDescBytes, "descriptor table slot too small");

hipError_t build_batch_table(const lbm_batch *b, void *host_table, size_t *bytes) {
    return with_codec(b->cav[0], [&](auto cd) {
        using C = decltype(cd);
        using R = typename C::R;
        CavityDesc<R> *t = static_cast<CavityDesc<R> *>(host_table);
        uint32_t start = 0;
        for (int k = 0; k < b->K; ++k) {
            const lbm_t *h = b->cav[k];
            t[k].g = geo_for(h, b->block);
            t[k].c = make_coef<R>(h);
            t[k].pop = pop_ptr<C>(h);
            t[k].cell = h->p.cell;
            t[k].active = b->active[k];
            t[k].start = start;
            start += t[k].g.gx * t[k].g.N;
        }
        *bytes = sizeof(CavityDesc<R>) * b->K;
        return hipSuccess;
    });
}

uint32_t batch_blocks(const lbm_batch *b) {
    uint32_t n = 0;
    for (int k = 0; k < b->K; ++k) n += geo_for(b->cav[k], b->block).gx * b->cav[k]->geo.N;
    return n;
}

hipError_t launch_step_batch(const lbm_batch *b, int parity, hipStream_t s) {
    return with_codec(b->cav[0], [&](auto cd) {
        using C = decltype(cd);
        using R = typename C::R;
        const auto *tab = reinterpret_cast<const CavityDesc<R> *>(static_cast<char *>(b->buf) + b->off_table);
        const uint32_t nb = batch_blocks(b);
        const uint32_t lds = lds_cap_bytes(b->waves[parity ? 1 : 0], b->block);
        if (parity) k_step_batch<C, true><<<nb, b->block, lds, s>>>(tab, b->K);
        else k_step_batch<C, false><<<nb, b->block, lds, s>>>(tab, b->K);
        return hipGetLastError();
    });
}

uint32_t lds_cap_bytes(int waves, int block) {
    if (waves <= 0 || block <= 0) return 0;
    // LDS per CU and per block of the current device, queried once per device
    static int per_cu[64] = {0}, per_block[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (!per_cu[dev]) {
        int a = 0, b = 0;
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || a <= 0 ||
            b <= 0)
            return 0;
        per_block[dev] = b;
        per_cu[dev] = a;
    }
    // blocks per CU that give `waves` waves on each of the 4 SIMDs; reserve
    // just over 1/(blocks + 1) of the LDS so that one more block never fits
    // while `blocks` fit with room to spare
    const int blocks = std::max(1, waves * 4 * 64 / block);
    uint32_t bytes = (static_cast<uint32_t>(per_cu[dev] / (blocks + 1)) + 1024u) / 512u * 512u;
    if (bytes > static_cast<uint32_t>(per_block[dev])) return 0;
    return bytes;
}

void default_waves(int storage, int out[2]) {
    // measured on the 257^3 step with streaming canonical-storage accesses:
    // FP32 587 us capped against 604 uncapped, FP16 380 against 383, FP64
    // 1207 against 1215; FP16C, whose codec costs more ALU, 394 us uncapped
    // and within 1% of that under any cap
    out[0] = out[1] = 0;
    if (storage == LBM_FP32) {
        out[0] = 2;
        out[1] = 3;
    } else if (storage == LBM_FP16S) {
        out[0] = 3;
    } else if (storage == LBM_FP64) {
        out[0] = 2;
        out[1] = 2;
    }
}

hipError_t launch_resample(const lbm_t *h, int M, float *out, hipStream_t s) {
    double *macro = dptr(h, h->L.off_macro);
    hipError_t e = launch_macro(h, macro, s);
    if (e != hipSuccess) return e;
    const uint64_t M3 = static_cast<uint64_t>(M) * M * M;
    k_resample<<<static_cast<uint32_t>((M3 + 255) / 256), 256, 0, s>>>(
        h->geo.N, h->p.cell, h->p.T_hot, h->p.T_cold, macro, M, out);
    return hipGetLastError();
}

hipError_t launch_init(const lbm_t *h, const double *uvwT, hipStream_t s) {
    return with_codec(h, [&](auto cd) {
        using C = decltype(cd);
        k_init<C><<<grid_of(h, 256), 256, 0, s>>>(pop_ptr<C>(h), geo_for(h, 256),
                                                 make_coef<typename C::R>(h), uvwT, h->p.wT0,
                                                 h->p.wT1, h->p.a_T);
        return hipGetLastError();
    });
}

hipError_t launch_set_pop(const lbm_t *h, const double *in, hipStream_t s) {
    return with_codec(h, [&](auto cd) {
        using C = decltype(cd);
        k_set_pop<C><<<grid_of(h, 256), 256, 0, s>>>(pop_ptr<C>(h), geo_for(h, 256),
                                                    make_coef<typename C::R>(h), in);
        return hipGetLastError();
    });
}

hipError_t launch_get_pop(const lbm_t *h, double *out, hipStream_t s) {
    return with_codec(h, [&](auto cd) {
        using C = decltype(cd);
        auto c = make_coef<typename C::R>(h);
        const dim3 gr = grid_of(h, 256);
        const typename C::S *p = pop_ptr<C>(h);
        if (h->p.cell == LBM_SIDE_HEATED) {
            if (h->parity) k_get_pop<C, LBM_SIDE_HEATED, true><<<gr, 256, 0, s>>>(p, geo_for(h, 256), c, out);
            else k_get_pop<C, LBM_SIDE_HEATED, false><<<gr, 256, 0, s>>>(p, geo_for(h, 256), c, out);
        } else {
            if (h->parity) k_get_pop<C, LBM_RAYLEIGH_BENARD, true><<<gr, 256, 0, s>>>(p, geo_for(h, 256), c, out);
            else k_get_pop<C, LBM_RAYLEIGH_BENARD, false><<<gr, 256, 0, s>>>(p, geo_for(h, 256), c, out);
        }
        return hipGetLastError();
    });
}

hipError_t launch_macro(const lbm_t *h, double *macro_out, hipStream_t s) {
    return with_codec(h, [&](auto cd) {
        using C = decltype(cd);
        auto c = make_coef<typename C::R>(h);
        const dim3 gr = grid_of(h, 256);
        const Geo g = geo_for(h, 256);
        const typename C::S *p = pop_ptr<C>(h);
        if (h->p.cell == LBM_SIDE_HEATED) {
            if (h->parity) k_macro<C, LBM_SIDE_HEATED, true><<<gr, 256, 0, s>>>(p, g, c, macro_out);
            else k_macro<C, LBM_SIDE_HEATED, false><<<gr, 256, 0, s>>>(p, g, c, macro_out);
        } else {
            if (h->parity) k_macro<C, LBM_RAYLEIGH_BENARD, true><<<gr, 256, 0, s>>>(p, g, c, macro_out);
            else k_macro<C, LBM_RAYLEIGH_BENARD, false><<<gr, 256, 0, s>>>(p, g, c, macro_out);
        }
        return hipGetLastError();
    });
}

hipError_t launch_obs_planes(const lbm_t *h, hipStream_t s) {
    return with_codec(h, [&](auto cd) {
        using C = decltype(cd);
        auto c = make_coef<typename C::R>(h);
        auto o = obs_out<typename C::R>(h);
        const dim3 gr = grid_of(h, 256);
        const Geo g = geo_for(h, 256);
        const typename C::S *p = pop_ptr<C>(h);
        if (h->p.cell == LBM_SIDE_HEATED) {
            if (h->parity) k_obs_planes<C, LBM_SIDE_HEATED, true><<<gr, 256, 0, s>>>(p, g, c, o);
            else k_obs_planes<C, LBM_SIDE_HEATED, false><<<gr, 256, 0, s>>>(p, g, c, o);
        } else {
            if (h->parity) k_obs_planes<C, LBM_RAYLEIGH_BENARD, true><<<gr, 256, 0, s>>>(p, g, c, o);
            else k_obs_planes<C, LBM_RAYLEIGH_BENARD, false><<<gr, 256, 0, s>>>(p, g, c, o);
        }
        return hipGetLastError();
    });
}

uint32_t observe_tiles(int N) { return (static_cast<uint32_t>(N) * N + kObsTile - 1) / kObsTile; }
uint32_t observe_blocks(int N) { return observe_tiles(N) * ((N + kObsZ - 1) / kObsZ); }

hipError_t launch_observe_reduce(const lbm_t *h, bool accumulate, hipStream_t s) {
    const int N = h->geo.N;
    const double *wall = h->has_flux ? dptr(h, h->L.off_wall) : nullptr;
    const ObsArgs a{h->p.nu, h->p.kappa, h->p.T_hot, h->p.T_cold};
    double *part = dptr(h, h->L.off_part);
    const uint32_t ntile = observe_tiles(N), nblk = observe_blocks(N);
    hipError_t e = with_codec(h, [&](auto cd) {
        using R = typename decltype(cd)::R;
        const R *pl = reinterpret_cast<const R *>(static_cast<char *>(h->buf) + h->L.off_macro);
        if (h->p.cell == LBM_SIDE_HEATED)
            k_observe<LBM_SIDE_HEATED, R><<<nblk, kRedBlock, 0, s>>>(N, ntile, a, pl, wall, part);
        else
            k_observe<LBM_RAYLEIGH_BENARD, R><<<nblk, kRedBlock, 0, s>>>(N, ntile, a, pl, wall, part);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    const double Nd = N;
    double *fold = dptr(h, h->L.off_fold);
    const uint32_t per = (nblk + kFold - 1) / kFold;
    k_fold_rows<LBM_NRAW, false><<<kFold, kRedBlock, 0, s>>>(part, nblk, per, fold);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_finalize_obs<<<1, kRedBlock, 0, s>>>(fold, kFold, 1.0 / (Nd * Nd * Nd), 1.0 / (Nd * Nd), 1.0 / Nd,
                                           dptr(h, h->L.off_res), accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_observe(const lbm_t *h, bool accumulate, hipStream_t s) {
    hipError_t e = launch_obs_planes(h, s);
    if (e != hipSuccess) return e;
    return launch_observe_reduce(h, accumulate, s);
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const uint64_t n16 = bytes / 16;
    const uint64_t want = (n16 + 255) / 256;
    const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>(want, uint64_t{1} << 30));
    k_copy<<<blocks, 256, 0, s>>>(static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_reset_acc(const lbm_t *h, hipStream_t s) {
    k_reset_acc<<<1, 64, 0, s>>>(dptr(h, h->L.off_res));
    return hipGetLastError();
}

hipError_t launch_residual(const lbm_t *h, hipStream_t s) {
    double *macro = dptr(h, h->L.off_macro);
    hipError_t e = launch_macro(h, macro, s);
    if (e != hipSuccess) return e;
    double *part = dptr(h, h->L.off_part);
    k_residual<<<grid_of(h, kRedBlock), kRedBlock, 0, s>>>(geo_for(h, kRedBlock), macro, dptr(h, h->L.off_snap), part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double *fold = dptr(h, h->L.off_fold);
    const uint32_t per = (h->L.nblk_red + kFold - 1) / kFold;
    k_fold_rows<5, true><<<kFold, kRedBlock, 0, s>>>(part, h->L.nblk_red, per, fold);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_finalize_residual<<<1, kRedBlock, 0, s>>>(fold, kFold, dptr(h, h->L.off_res));
    return hipGetLastError();
}

hipError_t launch_centerline(const lbm_t *h, hipStream_t s) {
    double *macro = dptr(h, h->L.off_macro);
    hipError_t e = launch_macro(h, macro, s);
    if (e != hipSuccess) return e;
    k_centerline<<<2, kRedBlock, 0, s>>>(h->geo.N, macro, dptr(h, h->L.off_res));
    return hipGetLastError();
}

hipError_t launch_profile(const lbm_t *h, hipStream_t s) {
    double *macro = dptr(h, h->L.off_macro);
    hipError_t e = launch_macro(h, macro, s);
    if (e != hipSuccess) return e;
    const int N = h->geo.N;
    double *part = dptr(h, h->L.off_prof);
    if (h->p.cell == LBM_SIDE_HEATED)
        k_profile<LBM_SIDE_HEATED><<<dim3((N + kRedBlock - 1) / kRedBlock, kProfG), kRedBlock, 0, s>>>(
            N, macro, h->p.T_hot, h->p.T_cold, part);
    else
        k_profile<LBM_RAYLEIGH_BENARD><<<dim3(N, kProfG), kRedBlock, 0, s>>>(N, macro, h->p.T_hot,
                                                                           h->p.T_cold, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_profile_final<<<1, kRedBlock, 0, s>>>(N, part, h->p.H / (h->p.kappa * h->p.dT), h->p.kappa,
                                            part + static_cast<uint64_t>(kProfG) * 2 * N);
    return hipGetLastError();
}

hipError_t launch_snapshot(const lbm_t *h, hipStream_t s) {
    double *macro = dptr(h, h->L.off_macro);
    hipError_t e = launch_macro(h, macro, s);
    if (e != hipSuccess) return e;
    const uint64_t V = static_cast<uint64_t>(h->geo.N2) * h->geo.N;
    return hipMemcpyAsync(dptr(h, h->L.off_snap), macro + V, 4 * V * sizeof(double),
                          hipMemcpyDeviceToDevice, s);
}

Layout make_layout(int N, int storage) {
    Layout L;
    L.esize = storage == LBM_FP64 ? 8 : (storage == LBM_FP32 ? 4 : 2);
    const uint64_t V = static_cast<uint64_t>(N) * N * N;
    const uint64_t N2 = static_cast<uint64_t>(N) * N;
    // sub-blocks of 32 KB per (moving) population, or one power of two
    // covering the whole plane when that is smaller
    const uint64_t wide = storage == LBM_FP64 ? 8 : 4;   // width of the wide slots
    const uint64_t nwide = (storage == LBM_FP16S || storage == LBM_FP16C) ? CF16::GW : 1;
    L.bbits = 0;
    while ((uint64_t{1} << L.bbits) * L.esize < 32768 && (uint64_t{1} << L.bbits) < N2) ++L.bbits;
    const uint64_t B = uint64_t{1} << L.bbits;
    const uint64_t nsub = (N2 + B - 1) / B;
    L.node_bytes = (kNPop - nwide) * L.esize + nwide * wide;
    L.sub = L.node_bytes * B;
    L.slab = nsub * L.sub;
    L.pop_bytes = L.slab * N;
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t o = 0;
    L.off_pop = o;
    o = up(o + L.pop_bytes);
    L.off_macro = o;
    o = up(o + 5 * V * sizeof(double));
    L.off_snap = o;
    o = up(o + 4 * V * sizeof(double));
    L.off_wall = o;
    o = up(o + 2 * N2 * sizeof(double));
    L.nblk_red = static_cast<uint32_t>((N2 + kRedBlock - 1) / kRedBlock * N);
    L.off_part = o;
    o = up(o + static_cast<size_t>(L.nblk_red) * kNPart * sizeof(double));
    L.off_fold = o;
    o = up(o + static_cast<size_t>(kFold) * kNPart * sizeof(double));
    L.off_res = o;
    o = up(o + kResDoubles * sizeof(double));
    L.off_prof = o;   // Nusselt profile: kProfG row-group sums of 2 N, then N values
    o = up(o + (static_cast<size_t>(kProfG) * 2 + 1) * N * sizeof(double));
    L.total = o;
    return L;
}

}  // namespace lbmk
