// fpd_device.hpp -- device-side building blocks of the FPD / MRT-LBM fiber step on gfx950.
//
// Lattice: D2Q9, directions e_0 = (0,0), e_1..e_4 = (1,0),(0,1),(-1,0),(0,-1),
// e_5..e_8 = (1,1),(-1,1),(-1,-1),(1,-1); weights 4/9, 1/9, 1/36.  Node (x, y) sits at the
// square centre (x + 1/2, y + 1/2) (arXiv:2212.14153, Sec. II.C); walls at y = 0 (moving at
// -U) and y = ny (moving at +U) (Sec. IV.A); x periodic.
//
// Storage: deviations g_k = f_k - w_k from the rest equilibrium, one contiguous run of nx
// values (padded to 64) per direction and row, the nine directions of a row side by side
// (index y * stride + k * plane + x).  A buffer holds post-collision values; a step pulls them
// along -e_k (half-way bounce-back at the walls), collides, and writes the next buffer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fpd_internal.hpp"

namespace fpd {

// ----------------------------------------------------------------- storage codecs ----
// g = f - w in the storage type; `T` is the arithmetic type of the collision.

template <int ST> struct Codec;

template <> struct Codec<FPD_F64> {
    using store_t = double;
    using T = double;
    __device__ static inline T load(const store_t* p) { return *p; }
    __device__ static inline T load_nt(const store_t* p) { return __builtin_nontemporal_load(p); }
    __device__ static inline void store(store_t* p, T v) { __builtin_nontemporal_store(v, p); }
    __device__ static inline double to_f64(store_t v) { return v; }
    __device__ static inline store_t from_f64(double v) { return v; }
};

template <> struct Codec<FPD_F32> {
    using store_t = float;
    using T = float;
    __device__ static inline T load(const store_t* p) { return *p; }
    __device__ static inline T load_nt(const store_t* p) { return __builtin_nontemporal_load(p); }
    __device__ static inline void store(store_t* p, T v) { __builtin_nontemporal_store(v, p); }
    __device__ static inline double to_f64(store_t v) { return (double)v; }
    __device__ static inline store_t from_f64(double v) { return (float)v; }
};

// binary16 of g * 2^14: |g| < 1 keeps the scaled value far below the binary16 maximum,
// and the scale lifts the small deviations out of the subnormal range.
template <> struct Codec<FPD_F16DEV> {
    using store_t = _Float16;
    using T = float;
    static constexpr float kScale = 16384.0f;
    static constexpr float kInv = 1.0f / 16384.0f;
    __device__ static inline T load(const store_t* p) { return (float)(*p) * kInv; }
    __device__ static inline T load_nt(const store_t* p) {
        return (float)__builtin_nontemporal_load(p) * kInv;
    }
    __device__ static inline void store(store_t* p, T v) {
        __builtin_nontemporal_store((_Float16)(v * kScale), p);
    }
    __device__ static inline double to_f64(store_t v) { return (double)(float)v * (double)kInv; }
    __device__ static inline store_t from_f64(double v) { return (_Float16)(float)(v * 16384.0); }
    // the same conversions on the raw 16 bits (low half of b)
    __device__ static inline T from_bits(uint32_t b) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)b) * kInv;
    }
    __device__ static inline uint32_t to_bits(T v) {
        return __builtin_bit_cast(uint16_t, (_Float16)(v * kScale));
    }
    // The two-node lattice path collides the stored values as they are, g * 2^14
    // (mrt_collide_scaled): the scale leaves the nine decodes per node.
    static constexpr bool kScaledCollide = true;
    __device__ static inline T from_bits_scaled(uint32_t b) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
    }
    __device__ static inline uint32_t to_bits_scaled(T v) {
        return __builtin_bit_cast(uint16_t, (_Float16)v);
    }
    // two values in one word (lo in the low half): one packed round-to-nearest-even
    // conversion, the same bits as two to_bits_scaled
    __device__ static inline uint32_t pack2_scaled(T lo, T hi) {
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        const h2 v = {(_Float16)lo, (_Float16)hi};
        return __builtin_bit_cast(uint32_t, v);
    }
};

// bfloat16 of g, round to nearest even (deviations are finite here).
__device__ inline uint16_t f32_to_bf16(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

template <> struct Codec<FPD_BF16DEV> {
    using store_t = uint16_t;
    using T = float;
    __device__ static inline T load(const store_t* p) { return bf16_to_f32(*p); }
    __device__ static inline T load_nt(const store_t* p) {
        return bf16_to_f32(__builtin_nontemporal_load(p));
    }
    __device__ static inline void store(store_t* p, T v) {
        __builtin_nontemporal_store(f32_to_bf16(v), p);
    }
    __device__ static inline double to_f64(store_t v) { return (double)bf16_to_f32(v); }
    __device__ static inline store_t from_f64(double v) { return f32_to_bf16((float)v); }
    __device__ static inline T from_bits(uint32_t b) { return bf16_to_f32((uint16_t)b); }
    __device__ static inline uint32_t to_bits(T v) { return f32_to_bf16(v); }
    static constexpr bool kScaledCollide = false;   // no scale to take out
    __device__ static inline T from_bits_scaled(uint32_t b) { return from_bits(b); }
    __device__ static inline uint32_t to_bits_scaled(T v) { return to_bits(v); }
    // two values in one word (lo in the low half): the hardware's packed conversion, round
    // to nearest even like f32_to_bf16 (the same bits for every finite value)
    __device__ static inline uint32_t pack2_scaled(T lo, T hi) {
        typedef __bf16 b2 __attribute__((ext_vector_type(2)));
        const b2 v = {(__bf16)lo, (__bf16)hi};
        return __builtin_bit_cast(uint32_t, v);
    }
};

// ------------------------------------------------------------------- helpers --------

__device__ inline int imod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Blocks are handed to the 8 XCDs round-robin; give every XCD one contiguous run of tiles
// so neighbouring tiles (which share cache lines through the x-shifted pulls) meet in the
// same L2.  A bijection on [0, nblocks).
__device__ inline int xcd_tile(int bid, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7;
    const int xcd = bid & 7, local = bid >> 3;
    return xcd * q + (xcd < r ? xcd : r) + local;
}

// Columns and rows whose node centres can lie within rc of a bead at (Rx, Ry):
// columns i0 + [0, w) modulo nx (w <= nx), rows j0..j1 (clipped to the channel).
// A bead that is not finite or has left any sensible range (a simulation that blew up)
// gets an empty box, so no index is ever formed from it.
__device__ inline bool bead_sane(double Rx, double Ry) {
    return fabs(Rx) < 1.0e9 && fabs(Ry) < 1.0e9;  // false for NaN too
}

// With walls, rows j0..j1 are clipped to the channel; in a periodic box (per) they are
// j0 .. j1 with j0 in [0, ny) and j1 - j0 < ny, to be taken modulo ny.
__device__ inline void bead_box(double Rx, double Ry, double rc, int nx, int ny, bool per,
                                int& i0, int& w, int& j0, int& j1) {
    if (!bead_sane(Rx, Ry)) {
        i0 = 0;
        w = 0;
        j0 = 0;
        j1 = -1;
        return;
    }
    const int lo = (int)floor(Rx - 0.5 - rc);
    const int hi = (int)ceil(Rx - 0.5 + rc);
    w = hi - lo + 1;
    if (w >= nx) {
        w = nx;
        i0 = 0;
    } else {
        i0 = imod(lo, nx);
    }
    const int a = (int)floor(Ry - 0.5 - rc);
    const int b = (int)ceil(Ry - 0.5 + rc);
    if (per) {
        const int h = b - a + 1 < ny ? b - a + 1 : ny;
        j0 = h == ny ? 0 : imod(a, ny);
        j1 = j0 + h - 1;
        return;
    }
    j0 = a < 0 ? 0 : a;
    j1 = b > ny - 1 ? ny - 1 : b;
}

// Do the column sets c0 + [0, cw) and i0 + [0, w) (both modulo nx) intersect?
__device__ inline bool cols_overlap(int c0, int cw, int i0, int w, int nx) {
    return imod(c0 - i0, nx) < w || imod(i0 - c0, nx) < cw;
}

// Minimum-image x distance dx - nx * floor(dx / nx + 1/2).  For |dx| < 3 nx / 2 the shift is
// 0 or one period and dx -+ nx is exact (Sterbenz: the operands are within a factor of two),
// so the compare-and-subtract below returns the same bits as the formula without a
// division; farther images fall back to the formula.
__device__ inline double min_image(double dx, int nx) {
    const double n = (double)nx;
    if (dx >= 0.5 * n) {
        if (dx < 1.5 * n) return dx - n;
    } else if (dx < -0.5 * n) {
        if (dx >= -1.5 * n) return dx + n;
    } else {
        return dx;
    }
    return dx - n * floor(dx / n + 0.5);
}

// y distance: the minimum image in a periodic box, plain between walls.
__device__ inline double y_image(double dy, int ny, bool per) {
    return per ? min_image(dy, ny) : dy;
}

// phi of Eq. (2), 1/2 (tanh((a - r)/xi) + 1), in the equal logistic form
// 1 / (1 + exp(2 (r - a)/xi)): one exponential and one division instead of a tanh (whose
// FP64 library form is a chain of some 200 dependent double-double operations), and no
// cancellation against 1 in the tail far from the bead.
__device__ inline double phi_f64(double r, double a, double xi) {
    return 1.0 / (1.0 + exp(2.0 * (r - a) / xi));
}
// FP32 (the FP32 and two-byte storage paths): the hardware 2^x, reciprocal and square root
// (BeadGeom<float>), each within about one ulp, instead of the correctly rounded library forms (the
// fiber tiles evaluate phi for every nearby bead at every node).
__device__ inline float phi_f32(float r, float a, float inv_xi) {
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * (r - a) * inv_xi);  // 2 log2(e)
    return __builtin_amdgcn_rcpf(1.0f + e);
}

// dist2 is the one expression of the FP64 squared distance: the cutoff test and phi itself
// always see the same value.
__device__ inline double dist2(double dx, double dy) { return dx * dx + dy * dy; }

// Minimum image of an integer offset d in (-n, n): d mod n in [-(n/2), n - n/2).
__device__ inline int wrap_offset(int d, int n) {
    const int h = n >> 1;
    if (d >= n - h) return d - n;
    if (d < -h) return d + n;
    return d;
}

// A bead as the fiber arithmetic of precision T sees it: the squared distance of a node
// centre (x + 1/2, y + 1/2) from the bead (minimum image in x, and in y in a periodic box)
// and the cutoff test r2 < rc^2.  The fiber tiles (Eqs. 1, 2, 4) and the bead kernel
// (A_i, Eq. 5) evaluate phi only through this, on the same per-bead data, so whether a node
// sees a bead, and the phi it gets, never depends on the tiling.  Every integer support box
// (bead_box, the window, the occupancy bitmap) holds all nodes closer than rc + 1 to the
// bead, so this test, not a box, decides which nodes are in.
template <typename T> struct BeadGeom;

template <> struct BeadGeom<double> {
    double R[2];
    __device__ static inline BeadGeom make(double Rx, double Ry, int, int, bool) {
        return BeadGeom{{Rx, Ry}};
    }
    __device__ inline double r2(int x, int y, int nx, int ny, bool per) const {
        const double dx = min_image((double)x + 0.5 - R[0], nx);
        const double dy = y_image((double)y + 0.5 - R[1], ny, per);
        return dist2(dx, dy);
    }
    // the node that holds the bead: floor(R), wrapped (x, and y in a periodic box)
    __device__ inline void node(int nx, int ny, bool per, int& ox, int& oy) const {
        ox = imod((int)floor(R[0]), nx);
        oy = per ? imod((int)floor(R[1]), ny) : (int)floor(R[1]);
    }
    __device__ static inline double cut2(double rc2) { return rc2; }
    // phi at squared distance r2 < cut2
    __device__ static inline double phi(double r2, double a, double xi, double) {
        return phi_f64(sqrt(r2), a, xi);
    }
};

// FP32 (the FP32 and two-byte storage paths): the node (ox, oy) holding the bead, i.e.
// floor(R) wrapped into the lattice, and q = 1/2 - frac(R) rounded to FP32.  A node's
// offset x + 1/2 - Rx is the integer x - ox (minimum image) plus q: one rounding of q and
// one of the FP32 sum, at any lattice size, and no FP64 arithmetic per node and bead.
template <> struct BeadGeom<float> {
    int o[2];
    float q[2];
    __device__ static inline BeadGeom make(double Rx, double Ry, int nx, int ny, bool per) {
        BeadGeom g{{0, 0}, {0.0f, 0.0f}};
        if (!bead_sane(Rx, Ry)) return g;  // empty support box: never evaluated
        const double fx = floor(Rx), fy = floor(Ry);
        g.o[0] = imod((int)fx, nx);
        g.o[1] = per ? imod((int)fy, ny) : (int)fy;
        g.q[0] = (float)(0.5 - (Rx - fx));  // Rx - floor(Rx) is exact
        g.q[1] = (float)(0.5 - (Ry - fy));
        return g;
    }
    __device__ inline float r2(int x, int y, int nx, int ny, bool per) const {
        const int di = wrap_offset(x - o[0], nx);
        const int dj = per ? wrap_offset(y - o[1], ny) : y - o[1];
        const float dx = (float)di + q[0], dy = (float)dj + q[1];
        return __builtin_fmaf(dx, dx, dy * dy);  // one fixed contraction everywhere
    }
    __device__ inline void node(int, int, bool, int& ox, int& oy) const {
        ox = o[0];
        oy = o[1];
    }
    __device__ static inline float cut2(double rc2) { return (float)rc2; }
    __device__ static inline float phi(float r2, double a, double, double inv_xi) {
        return phi_f32(__builtin_amdgcn_sqrtf(r2), (float)a, (float)inv_xi);
    }
};

// -------------------------------------------------------------- pull streaming -----
// g[k] <- post-collision g*_k at x - e_k; x wraps (y too in a periodic box, per); a
// population that would come from behind a wall is the node's own reflected g*_{opp(k)}
// plus 6 w_k rho0 (e_k . u_wall), i.e. +-U/6 on the diagonals (u_wall = -U below, +U
// above).

template <class Cd>
__device__ inline void pull(const typename Cd::store_t* __restrict__ src, int nx, int ny,
                            int stride, long long plane, int x, int y, bool per,
                            typename Cd::T u6, typename Cd::T g[9]) {
    using S = typename Cd::store_t;
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const S* p0 = src;
    const S* p1 = src + plane;
    const S* p2 = src + 2 * plane;
    const S* p3 = src + 3 * plane;
    const S* p4 = src + 4 * plane;
    const S* p5 = src + 5 * plane;
    const S* p6 = src + 6 * plane;
    const S* p7 = src + 7 * plane;
    const S* p8 = src + 8 * plane;
    const long long r0 = (long long)y * stride;  // 64-bit: buffers may exceed 2^31 values
    g[0] = Cd::load_nt(p0 + r0 + x);
    g[1] = Cd::load(p1 + r0 + xm);
    g[3] = Cd::load(p3 + r0 + xp);
    if (y > 0 || per) {
        const long long rm = y > 0 ? r0 - stride : (long long)(ny - 1) * stride;
        g[2] = Cd::load_nt(p2 + rm + x);
        g[5] = Cd::load(p5 + rm + xm);
        g[6] = Cd::load(p6 + rm + xp);
    } else {
        g[2] = Cd::load(p4 + r0 + x);
        g[5] = Cd::load(p7 + r0 + x) - u6;
        g[6] = Cd::load(p8 + r0 + x) + u6;
    }
    if (y < ny - 1 || per) {
        const long long rp = y < ny - 1 ? r0 + stride : 0;
        g[4] = Cd::load_nt(p4 + rp + x);
        g[7] = Cd::load(p7 + rp + xp);
        g[8] = Cd::load(p8 + rp + xm);
    } else {
        g[4] = Cd::load(p2 + r0 + x);
        g[7] = Cd::load(p5 + r0 + x) - u6;
        g[8] = Cd::load(p6 + r0 + x) + u6;
    }
}

// Two-byte storage: a lane updates G = nodes_per_lane consecutive nodes x0 .. x0 + G - 1
// (x0 a multiple of G) of one row and moves populations as aligned G/2-dword vectors, so
// every memory request carries 2 G bytes per lane.  A value left of x0, or right of the
// group, is an end of the neighbouring lane's vector (a wave's 64 lanes hold 64 G
// consecutive nodes of one row); at a wave's edge and at the periodic wrap it is a 2-byte
// load.  All lanes of the wave must call these (the cross-lane moves need every lane);
// lanes with x0 >= nx load nothing.  Rows start at multiples of 64 elements in 16-byte
// aligned buffers, so the vector loads are aligned.

// The loads of one direction row for the group, pulled along an x shift SX = e_kx: node
// x0 + i takes the row's value at x0 + i - SX (x wraps).  w holds the vector at x0; e the
// value beyond the group edge that a wave-edge or wrapping lane loads itself; c the value
// at x = 0 for a node nx - 1 inside the group (SX = -1).  All loads of a group are issued
// before any cross-lane move, so a wave waits for memory once.
template <int G>
struct GroupRaw {
    uint32_t w[G / 2];
    uint32_t e, c;
    __device__ inline uint32_t elem(int i) const { return (w[i >> 1] >> (16 * (i & 1))) & 0xffffu; }
};

template <int G, int SX>
__device__ inline GroupRaw<G> group_load(const uint16_t* __restrict__ row, int x0, int nx,
                                         bool first, bool last) {
    const bool in = x0 < nx;
    GroupRaw<G> r;
#pragma unroll
    for (int i = 0; i < G / 2; ++i) r.w[i] = 0u;
    r.e = 0u;
    r.c = 0u;
    if (in) {
        // rows read without an x shift share no cache line with a neighbouring tile:
        // non-temporal
        if constexpr (G == 2) {
            const uint32_t* q = (const uint32_t*)(row + x0);
            r.w[0] = SX == 0 ? __builtin_nontemporal_load(q) : *q;
        } else {
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            const u32x2* q = (const u32x2*)(row + x0);
            const u32x2 v = SX == 0 ? __builtin_nontemporal_load(q) : *q;
            r.w[0] = v.x;
            r.w[1] = v.y;
        }
    }
    if (SX == 1) {
        if (in && (first || x0 == 0)) r.e = row[x0 == 0 ? nx - 1 : x0 - 1];
    } else if (SX == -1) {
        if (in && x0 + G - 1 < nx && (last || x0 + G >= nx)) r.e = row[imod(x0 + G, nx)];
        if (in && x0 + G - 1 >= nx) r.c = row[0];
    }
    return r;
}

// Whole-wave moves by one lane (DPP wave_shr:1 / wave_shl:1 of the gfx9 family: one VALU
// move each, no LDS permute): lane i receives lane i - 1's value (shr) or lane i + 1's
// (shl); the lane with no source (0, resp. 63) receives 0 and takes its value from memory.
__device__ inline uint32_t wave_shr1(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ inline uint32_t wave_shl1(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}

// Values in the collision's units: the stored values as they are for a codec that
// collides scaled (Codec::kScaledCollide), else the deviations g.
template <class Cd, int G, int SX>
__device__ inline void group_finish(const GroupRaw<G>& r, int x0, int nx, bool first,
                                    bool last, typename Cd::T v[G]) {
    const bool in = x0 < nx;
    if (SX == 0) {
#pragma unroll
        for (int i = 0; i < G; ++i) v[i] = Cd::from_bits_scaled(r.elem(i));
    } else if (SX == 1) {
        uint32_t l = wave_shr1(r.elem(G - 1));  // x0 - 1: left lane's last
        if (in && (first || x0 == 0)) l = r.e;
        v[0] = Cd::from_bits_scaled(l);
#pragma unroll
        for (int i = 1; i < G; ++i) v[i] = Cd::from_bits_scaled(r.elem(i - 1));
    } else {
        uint32_t rr = wave_shl1(r.elem(0));  // x0 + G: right lane's first
        if (in && x0 + G - 1 < nx && (last || x0 + G >= nx)) rr = r.e;
#pragma unroll
        for (int i = 0; i < G - 1; ++i)
            v[i] = Cd::from_bits_scaled(x0 + i + 1 < nx ? r.elem(i + 1) : r.c);
        v[G - 1] = Cd::from_bits_scaled(rr);
    }
}

// pull() for the group of nodes x0 .. x0 + G - 1 of row y; g[i] receives node x0 + i, in
// the collision's units (group_finish; the wall term u6 comes in the same units).
template <class Cd, int G>
__device__ inline void pull_group(const uint16_t* __restrict__ src, int nx, int ny, int stride,
                                  long long plane, int x0, int y, bool per, bool first,
                                  bool last, typename Cd::T u6, typename Cd::T g[G][9]) {
    using T = typename Cd::T;
    const long long r0 = (long long)y * stride;
    const uint16_t* row = src + r0;
    const bool bottom = y == 0 && !per, top = y == ny - 1 && !per;
    const uint16_t* rm = y > 0 ? row - stride : (per ? row + (long long)(ny - 1) * stride : row);
    const uint16_t* rp = y < ny - 1 ? row + stride : (per ? src : row);
    // g_2, g_5, g_6 come from the row below, or reflected at the bottom wall; g_4, g_7,
    // g_8 from the row above, or reflected at the top wall
    const GroupRaw<G> q0 = group_load<G, 0>(row, x0, nx, first, last);
    const GroupRaw<G> q1 = group_load<G, 1>(row + plane, x0, nx, first, last);
    const GroupRaw<G> q3 = group_load<G, -1>(row + 3 * plane, x0, nx, first, last);
    GroupRaw<G> q2, q5, q6, q4, q7, q8;
    if (!bottom) {
        q2 = group_load<G, 0>(rm + 2 * plane, x0, nx, first, last);
        q5 = group_load<G, 1>(rm + 5 * plane, x0, nx, first, last);
        q6 = group_load<G, -1>(rm + 6 * plane, x0, nx, first, last);
    } else {
        q2 = group_load<G, 0>(row + 4 * plane, x0, nx, first, last);
        q5 = group_load<G, 0>(row + 7 * plane, x0, nx, first, last);
        q6 = group_load<G, 0>(row + 8 * plane, x0, nx, first, last);
    }
    if (!top) {
        q4 = group_load<G, 0>(rp + 4 * plane, x0, nx, first, last);
        q7 = group_load<G, -1>(rp + 7 * plane, x0, nx, first, last);
        q8 = group_load<G, 1>(rp + 8 * plane, x0, nx, first, last);
    } else {
        q4 = group_load<G, 0>(row + 2 * plane, x0, nx, first, last);
        q7 = group_load<G, 0>(row + 5 * plane, x0, nx, first, last);
        q8 = group_load<G, 0>(row + 6 * plane, x0, nx, first, last);
    }
    T v[G];
#define FPD_PUT(K, Q, SX)                                               \
    group_finish<Cd, G, SX>(Q, x0, nx, first, last, v);                 \
    _Pragma("unroll") for (int i = 0; i < G; ++i) g[i][K] = v[i];
    FPD_PUT(0, q0, 0)
    FPD_PUT(1, q1, 1)
    FPD_PUT(3, q3, -1)
    if (!bottom) {
        FPD_PUT(2, q2, 0)
        FPD_PUT(5, q5, 1)
        FPD_PUT(6, q6, -1)
    } else {
        FPD_PUT(2, q2, 0)
        FPD_PUT(5, q5, 0)
        FPD_PUT(6, q6, 0)
#pragma unroll
        for (int i = 0; i < G; ++i) {
            g[i][5] -= u6;
            g[i][6] += u6;
        }
    }
    if (!top) {
        FPD_PUT(4, q4, 0)
        FPD_PUT(7, q7, -1)
        FPD_PUT(8, q8, 1)
    } else {
        FPD_PUT(4, q4, 0)
        FPD_PUT(7, q7, 0)
        FPD_PUT(8, q8, 0)
#pragma unroll
        for (int i = 0; i < G; ++i) {
            g[i][7] -= u6;
            g[i][8] += u6;
        }
    }
#undef FPD_PUT
}

// ---------------------------------------------------------- MRT collision ---------
// Multiple-relaxation-time collision on deviations g = f - w in the Lallemand-Luo moment
// basis (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy), with Guo's forcing: the velocity is
// (j + F/2)/rho and the source (I - S/2) applied to the force moments
//   (0, 6 u.F, -6 u.F, F_x, -F_x, F_y, -F_y, 2(u_x F_x - u_y F_y), u_x F_y + u_y F_x).
// 1/x in the arithmetic of T: FP64 divides; FP32 (the FP32 and two-byte paths) takes the
// hardware reciprocal, within about one ulp, instead of the correctly rounded division
// sequence (ten instructions per node in the collision).
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
// a / b in the same sense (FP64: the division itself)
__device__ inline double quot(double a, double b) { return a / b; }
__device__ inline float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// The moment matrix has entries in {0, +-1, +-2, +-4} and is applied as adds in registers;
// moments of w are (1, -2, 1, 0, ...), so e and eps are carried as deviations too and no
// O(1) cancellation enters |m - m_eq|.
// kForce = false: the collision without a force term (F = 0), as a separate instance
// rather than F = 0 at run time, whose products with zero the compiler must keep.  With
// F = +0 the forced instance gives the same bits (every force term is then +0 or -0
// added to a sum, so only the sign of an exact zero could differ).
template <typename T, bool kForce = true>
__device__ inline void mrt_collide(T g[9], T Fx, T Fy, T s_nu, T s_q, T s_e, T s_eps) {
    const T s14 = (g[1] + g[2]) + (g[3] + g[4]);
    const T s58 = (g[5] + g[6]) + (g[7] + g[8]);
    const T drho = g[0] + s14 + s58;
    const T rho = T(1) + drho;
    const T d13 = g[1] - g[3], d24 = g[2] - g[4];
    const T a58 = (g[5] - g[7]), b68 = (g[6] - g[8]);
    T jx = d13 + a58 - b68;           // g1 - g3 + g5 - g6 - g7 + g8
    T jy = d24 + a58 + b68;           // g2 - g4 + g5 + g6 - g7 - g8
    T me = T(2) * s58 - s14 - T(4) * g[0];
    T meps = s58 - T(2) * s14 + T(4) * g[0];
    T qx = (a58 - b68) - T(2) * d13;
    T qy = (a58 + b68) - T(2) * d24;
    T pxx = (g[1] + g[3]) - (g[2] + g[4]);
    T pxy = (g[5] + g[7]) - (g[6] + g[8]);

    const T inv_rho = recip(rho);
    // rho u = j + F/2 (Guo), u = rho u / rho
    const T rux = kForce ? jx + T(0.5) * Fx : jx, ruy = kForce ? jy + T(0.5) * Fy : jy;
    const T ux = rux * inv_rho, uy = ruy * inv_rho;
    const T ru2 = rux * ux + ruy * uy;

    // m* = m - s (m - m_eq) + (1 - s/2) F_m, moment by moment
    me = me - s_e * (me - (T(-2) * drho + T(3) * ru2));
    meps = meps - s_eps * (meps - (drho - T(3) * ru2));
    qx = qx - s_q * (qx + rux);
    qy = qy - s_q * (qy + ruy);
    pxx = pxx - s_nu * (pxx - (rux * ux - ruy * uy));
    pxy = pxy - s_nu * (pxy - rux * uy);
    if constexpr (kForce) {
        const T uF = ux * Fx + uy * Fy;
        me += (T(1) - T(0.5) * s_e) * (T(6) * uF);
        meps += (T(1) - T(0.5) * s_eps) * (T(-6) * uF);
        const T hq = T(1) - T(0.5) * s_q;
        qx -= hq * Fx;
        qy -= hq * Fy;
        const T hn = T(1) - T(0.5) * s_nu;
        pxx += hn * T(2) * (ux * Fx - uy * Fy);
        pxy += hn * (ux * Fy + uy * Fx);
        jx += Fx;
        jy += Fy;
    }

    // g = M^{-1} m*, M^{-1} = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const T a = drho * T(1.0 / 9.0);
    const T b = me * T(1.0 / 36.0);
    const T c = meps * T(1.0 / 36.0);
    const T d = jx * T(1.0 / 6.0);
    const T e = qx * T(1.0 / 12.0);
    const T f = jy * T(1.0 / 6.0);
    const T h = qy * T(1.0 / 12.0);
    const T p = pxx * T(0.25);
    const T q = pxy * T(0.25);
    const T axis = a - b - T(2) * c;
    const T diag = a + T(2) * b + c;
    const T de = d + e, fh = f + h;
    g[0] = a - T(4) * b + T(4) * c;
    g[1] = axis + (d - T(2) * e) + p;
    g[3] = axis - (d - T(2) * e) + p;
    g[2] = axis + (f - T(2) * h) - p;
    g[4] = axis - (f - T(2) * h) - p;
    g[5] = diag + de + fh + q;
    g[6] = diag - de + fh - q;
    g[7] = diag - de - fh + q;
    g[8] = diag + de - fh - q;
}

// mrt_collide on h = S g, the deviations scaled by S = 2^14 as the FP16 format stores them:
// the moments of h are S times those of g; rho and u come from the unscaled drho and j, the
// equilibria and force terms enter scaled by S, and the result is S g*.  The same operator
// as mrt_collide; the scale leaves the nine decodes and encodes of each node.
template <typename T, bool kForce = true>
__device__ inline void mrt_collide_scaled(T g[9], T Fx, T Fy, T s_nu, T s_q, T s_e, T s_eps) {
    constexpr T S = T(16384), iS = T(1.0 / 16384.0);
    const T s14 = (g[1] + g[2]) + (g[3] + g[4]);
    const T s58 = (g[5] + g[6]) + (g[7] + g[8]);
    const T drho = g[0] + s14 + s58;
    const T rho = T(1) + drho * iS;
    const T d13 = g[1] - g[3], d24 = g[2] - g[4];
    const T a58 = (g[5] - g[7]), b68 = (g[6] - g[8]);
    T jx = d13 + a58 - b68;
    T jy = d24 + a58 + b68;
    T me = T(2) * s58 - s14 - T(4) * g[0];
    T meps = s58 - T(2) * s14 + T(4) * g[0];
    T qx = (a58 - b68) - T(2) * d13;
    T qy = (a58 + b68) - T(2) * d24;
    T pxx = (g[1] + g[3]) - (g[2] + g[4]);
    T pxy = (g[5] + g[7]) - (g[6] + g[8]);

    const T Fxs = S * Fx, Fys = S * Fy;       // force density in the scaled units
    const T inv_rho_s = iS * recip(rho);
    // S rho u = S (j + F/2), u = S rho u / (S rho)
    const T rux = kForce ? jx + T(0.5) * Fxs : jx, ruy = kForce ? jy + T(0.5) * Fys : jy;
    const T ux = rux * inv_rho_s, uy = ruy * inv_rho_s;
    const T ru2 = rux * ux + ruy * uy;

    me = me - s_e * (me - (T(-2) * drho + T(3) * ru2));
    meps = meps - s_eps * (meps - (drho - T(3) * ru2));
    qx = qx - s_q * (qx + rux);
    qy = qy - s_q * (qy + ruy);
    pxx = pxx - s_nu * (pxx - (rux * ux - ruy * uy));
    pxy = pxy - s_nu * (pxy - rux * uy);
    if constexpr (kForce) {
        const T uF = ux * Fxs + uy * Fys;
        me += (T(1) - T(0.5) * s_e) * (T(6) * uF);
        meps += (T(1) - T(0.5) * s_eps) * (T(-6) * uF);
        const T hq = T(1) - T(0.5) * s_q;
        qx -= hq * Fxs;
        qy -= hq * Fys;
        const T hn = T(1) - T(0.5) * s_nu;
        pxx += hn * T(2) * (ux * Fxs - uy * Fys);
        pxy += hn * (ux * Fys + uy * Fxs);
        jx += Fxs;
        jy += Fys;
    }

    const T a = drho * T(1.0 / 9.0);
    const T b = me * T(1.0 / 36.0);
    const T c = meps * T(1.0 / 36.0);
    const T d = jx * T(1.0 / 6.0);
    const T e = qx * T(1.0 / 12.0);
    const T f = jy * T(1.0 / 6.0);
    const T h = qy * T(1.0 / 12.0);
    const T p = pxx * T(0.25);
    const T q = pxy * T(0.25);
    const T axis = a - b - T(2) * c;
    const T diag = a + T(2) * b + c;
    const T de = d + e, fh = f + h;
    g[0] = a - T(4) * b + T(4) * c;
    g[1] = axis + (d - T(2) * e) + p;
    g[3] = axis - (d - T(2) * e) + p;
    g[2] = axis + (f - T(2) * h) - p;
    g[4] = axis - (f - T(2) * h) - p;
    g[5] = diag + de + fh + q;
    g[6] = diag - de + fh - q;
    g[7] = diag - de - fh + q;
    g[8] = diag + de - fh - q;
}

// Rest weights, for decoding g back to f.
__device__ inline double lattice_w(int k) {
    return k == 0 ? 4.0 / 9.0 : (k < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

}  // namespace fpd
