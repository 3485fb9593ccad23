// fpd_kernels.hip -- gfx950 kernels of the FPD / MRT-LBM fiber time step
// (arXiv:2212.14153, Sec. II.C, integration steps (1)-(3)).
//
// One step is two launches:
//   step_kernel  every node: pull-stream, MRT collision with the local shear rate from
//                eta^n (Eq. 1) and Guo forcing with f^n (Eq. 4), store.  Tiles that meet
//                the fiber's support window stage the nearby beads in LDS with their forces
//                F_i^n (Eqs. 10-12, O(N) work), evaluate phi_i (Eq. 2) per node and record
//                f^n in the window for the bead kernel.
//   bead_kernel  one block per bead: V_i^{n+1} from Eq. (5) over the bead's support box
//                (FP64 accumulation), R_i^{n+1} = R_i^n + V_i^{n+1}, A_i^{n+1} at the new
//                position, and the bead's share of the next support window and health bits
//                (integer atomic min / max / or: order-independent).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>

#include "fpd_device.hpp"

namespace fpd {

// ------------------------------------------------------------------ reductions ------

// One DPP move of a double (two 32-bit halves): lanes outside ROW_MASK, and lanes whose
// source lies outside their row of 16, receive 0.  Controls of the gfx9 family:
// row_shr:n = 0x110 + n, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (all lanes active), in a fixed order, returned to every
// lane: running sums along each row of 16 lanes by shifts of 1, 2, 4, 8, then rows 0 + 1
// and 2 + 3 by broadcasting lane 15 of a row into the next, and the two halves by
// broadcasting lane 31; lane 63 then holds the total.  Register moves only, no LDS.
__device__ inline double wave_sum(double v) {
    v += dpp_move<0x111, 0xf>(v);
    v += dpp_move<0x112, 0xf>(v);
    v += dpp_move<0x114, 0xf>(v);
    v += dpp_move<0x118, 0xf>(v);
    v += dpp_move<0x142, 0xa>(v);
    v += dpp_move<0x143, 0xc>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Sum over the block in a fixed order (deterministic); result valid in every thread.
__device__ inline double block_sum(double v, double* scratch) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nthreads = blockDim.x * blockDim.y;
    const int lane = tid & 63, wave = tid >> 6, nwaves = (nthreads + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += scratch[w];
    __syncthreads();
    return s;
}

// Sums over kBeadLanes virtual lanes held R per thread (R = kBeadLanes / blockDim.x, 1-D
// blocks): v[r] is the partial sum of virtual lane tid + r * blockDim.x, which lies in
// virtual wave (tid >> 6) + r * blockDim.x / 64 at the same lane, so the wave sums and the
// order over virtual waves are those of a block of kBeadLanes threads.  Result in every
// thread; scratch holds kBeadLanes / 64 entries per sum.
template <int R>
__device__ inline double lanes_sum(const double (&v)[R], double* scratch) {
    const int tid = threadIdx.x, lane = tid & 63, wpr = (int)blockDim.x >> 6;
    __syncthreads();  // scratch may still be read by a previous sum
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double w = wave_sum(v[r]);
        if (lane == 0) scratch[r * wpr + (tid >> 6)] = w;
    }
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < kBeadLanes / 64; ++q) s += scratch[q];
    return s;
}

// Two lanes_sum at once (bitwise the same results), through one round of the scratch array.
template <int R>
__device__ inline void lanes_sum2(const double (&a)[R], const double (&b)[R], double& sa,
                                  double& sb, double* scratch) {
    constexpr int nw = kBeadLanes / 64;
    const int tid = threadIdx.x, lane = tid & 63, wpr = (int)blockDim.x >> 6;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double wa = wave_sum(a[r]), wb = wave_sum(b[r]);
        if (lane == 0) {
            scratch[r * wpr + (tid >> 6)] = wa;
            scratch[nw + r * wpr + (tid >> 6)] = wb;
        }
    }
    __syncthreads();
    sa = 0.0;
    sb = 0.0;
    for (int q = 0; q < nw; ++q) {
        sa += scratch[q];
        sb += scratch[nw + q];
    }
}

// ----------------------------------------------------------- bead forces ------------

// Forces of Eqs. (10)-(12) on bead t, gathered bond by bond: the stretching energy
// k_s/(2 l0^2) (L_m - l0)^2 of bond m = (m, m+1) and the bending energy
// -k_b t_m . t_{m+1} of the pair of bonds (m, m+1), whose forces on the three beads
// m, m+1, m+2 are k_b times -a_m, a_m - b_m, b_m with
// a_m = (I - t_m t_m) t_{m+1} / L_m and b_m = (I - t_{m+1} t_{m+1}) t_m / L_{m+1}.
// Tangents t_m and lengths L_m of all bonds, computed once per block into LDS (one thread
// per bond) so that the per-bead gathers below keep few values in registers.
struct Bonds {
    double t[kMaxBeads][2];
    double L[kMaxBeads];
};

__device__ inline void fill_bonds(const BeadState* bs, int N, Bonds& B) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nthreads = blockDim.x * blockDim.y;
    for (int m = tid; m < N - 1; m += nthreads) {
        const double dx = bs->R[m + 1][0] - bs->R[m][0];
        const double dy = bs->R[m + 1][1] - bs->R[m][1];
        const double L = sqrt(dx * dx + dy * dy);
        B.t[m][0] = dx / L;
        B.t[m][1] = dy / L;
        B.L[m] = L;
    }
    __syncthreads();
}

// k_b (I - t_u t_u) t_v / L_u added with sign `sg` to F.
__device__ inline void add_proj(const Bonds& B, int u, int v, double sg_kb, double F[2]) {
    const double t0 = B.t[u][0], t1 = B.t[u][1];
    const double v0 = B.t[v][0], v1 = B.t[v][1];
    const double vt = v0 * t0 + v1 * t1;
    const double inv = sg_kb / B.L[u];
    F[0] += (v0 - vt * t0) * inv;
    F[1] += (v1 - vt * t1) * inv;
}

// Bead t of a fiber of L beads (tc = t mod L is its index inside its fiber; the bonds of
// the whole bead list are indexed globally, and a bond between two fibers is never used).
__device__ inline void bead_force(const Bonds& B, int L, int t, double ks_l02, double l0,
                                  double kb, const double fext[2], double F[2]) {
    const int tc = t % L;
    F[0] = fext[0];  // external driving force (Sec. III.B), zero for the fiber runs
    F[1] = fext[1];
    if (tc >= 1) {  // bond (t-1, t): pulls t back towards t-1 when stretched
        const double s = ks_l02 * (B.L[t - 1] - l0);
        F[0] -= s * B.t[t - 1][0];
        F[1] -= s * B.t[t - 1][1];
    }
    if (tc <= L - 2) {  // bond (t, t+1)
        const double s = ks_l02 * (B.L[t] - l0);
        F[0] += s * B.t[t][0];
        F[1] += s * B.t[t][1];
    }
    if (kb == 0.0) return;
    if (tc <= L - 3) add_proj(B, t, t + 1, -kb, F);         // pair (t, t+1): -k_b a_t
    if (tc >= 1 && tc <= L - 2) {                           // pair (t-1, t): middle bead
        add_proj(B, t - 1, t, kb, F);                       //   + k_b a_{t-1}
        add_proj(B, t, t - 1, -kb, F);                      //   - k_b b_{t-1}
    }
    if (tc >= 2) add_proj(B, t - 1, t - 2, kb, F);          // pair (t-2, t-1): + k_b b_{t-2}
}

// Excluded volume between fibers (no force the paper names; off unless ev_k > 0): bead t
// is pushed away from every bead j of another fiber closer than ev_d with the force of the
// pair energy (k/2)(d - r)^2, summed over j in increasing order (minimum image along the
// periodic directions; the positions are those of the step's start).
__device__ inline void ev_force(const Fiber& fib, int nx, int ny, bool per, int t,
                                double F[2]) {
    const BeadState* bs = fib.bs;
    const double k = bs->ev_k, d = bs->ev_d;
    if (!(k > 0.0)) return;
    const int L = fib.chain_len, ct = t / L;
    const double Rx = bs->R[t][0], Ry = bs->R[t][1];
    for (int j = 0; j < fib.n; ++j) {
        if (j / L == ct) continue;
        double dx = Rx - bs->R[j][0], dy = Ry - bs->R[j][1];
        dx = min_image(dx, nx);
        dy = y_image(dy, ny, per);
        const double r = sqrt(dx * dx + dy * dy);
        if (!(r < d) || r == 0.0) continue;
        const double s = k * (d - r) / r;
        F[0] += s * dx;
        F[1] += s * dy;
    }
}

// Window slot (raw bounds) -> x0 (mod nx), width, y0, height; clamped to the reserved
// window (a clamp means the fiber outgrew it: FPD_HEALTH_SUPPORT is raised by block 0).
struct Window {
    int x0, w, y0, h;
    bool clamped;
};

__device__ inline Window decode_window(const int* raw, int nx, int ny, bool per, int wmax,
                                       int hmax) {
    Window r{0, 0, 0, 0, false};
    const int lo = raw[0], hi = raw[1], j0 = raw[2], j1 = raw[3];
    if (lo > hi || j0 > j1) return r;
    r.w = hi - lo + 1;
    if (r.w >= nx) {
        r.w = nx;
        r.x0 = 0;
    } else {
        r.x0 = imod(lo, nx);
    }
    if (per) {  // rows wrap like columns
        r.h = j1 - j0 + 1;
        if (r.h >= ny) {
            r.h = ny;
            r.y0 = 0;
        } else {
            r.y0 = imod(j0, ny);
        }
    } else {
        r.y0 = j0 < 0 ? 0 : j0;
        const int y1 = j1 > ny - 1 ? ny - 1 : j1;
        r.h = y1 >= r.y0 ? y1 - r.y0 + 1 : 0;
    }
    if (r.w > wmax || r.h > hmax) {
        r.clamped = true;
        r.w = min(r.w, wmax);
        r.h = min(r.h, hmax);
    }
    return r;
}

__device__ inline void atomic_max_nonneg(unsigned long long* p, double v) {
    if (v >= 0.0) atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// ------------------------------------------------------------ occupancy bitmap ----

__device__ inline int occ_words(const Fiber& fib) { return (fib.occ_nx * fib.occ_ny + 31) >> 5; }

// Does any cell under the tile's nodes (columns [x0, x0 + w), rows [y0, y0 + h), clipped
// to the lattice) hold a mark in `slot`?
// The cells of one cell row are consecutive bits, so a tile (at most 256 nodes wide and
// 16 rows high, i.e. at most 9 x 2 cells of 32) reads a few words, all issued together.
__device__ inline bool occ_hit(const Fiber& fib, int slot, int x0, int w, int y0, int h,
                               int nx, int ny) {
    const unsigned* m = fib.bs->occ[slot];
    const int s = fib.occ_shift;
    const int c0 = x0 >> s, c1 = (min(x0 + w, nx) - 1) >> s;
    const int r0 = y0 >> s, r1 = (min(y0 + h, ny) - 1) >> s;
    unsigned any = 0u;
    for (int r = r0; r <= r1; ++r) {
        const int b0 = r * fib.occ_nx + c0, b1 = r * fib.occ_nx + c1;  // bit range
        for (int wd = b0 >> 5; wd <= (b1 >> 5); ++wd) {
            const int lo = max(b0 - (wd << 5), 0), hi = min(b1 - (wd << 5), 31);
            const unsigned mask = (hi - lo == 31) ? 0xffffffffu
                                                  : (((1u << (hi - lo + 1)) - 1u) << lo);
            any |= m[wd] & mask;
        }
    }
    return any != 0u;
}

// Mark the cells of the unwrapped node range [lo, hi] x [jlo, jhi] (x wraps; y wraps in a
// periodic box, else it is clipped to the channel).
// (Positions pass bead_sane, so every index here fits an int.)
__device__ inline void occ_mark(const Fiber& fib, int slot, int lo, int hi, int jlo, int jhi,
                                int nx, int ny, bool per) {
    unsigned* m = fib.bs->occ[slot];
    const int s = fib.occ_shift;
    if (!per) {
        jlo = jlo < 0 ? 0 : jlo;
        jhi = jhi > ny - 1 ? ny - 1 : jhi;
    }
    if (hi - lo + 1 >= nx) {
        lo = 0;
        hi = nx - 1;
    }
    if (per && jhi - jlo + 1 >= ny) {
        jlo = 0;
        jhi = ny - 1;
    }
    for (int y = jlo; y <= jhi;) {
        const int yw = per ? imod(y, ny) : y;
        const int r = yw >> s;
        for (int x = lo; x <= hi;) {
            const int xw = imod(x, nx);
            const int c = xw >> s;
            const int cell = r * fib.occ_nx + c;
            atomicOr(&m[cell >> 5], 1u << (cell & 31));
            x += min((c + 1) << s, nx) - xw;  // to the next cell (or the wrap)
        }
        y += min((r + 1) << s, ny) - yw;
    }
}

// The tile that contains node (floor Rx mod nx, floor Ry) owns bead b: it publishes F_b,
// C_b and the strain of bond (b, b+1).
__device__ inline void own_bead(const Fiber& fib, const Bonds& B, int b, const double F[2],
                                double C0, double C1) {
    BeadState* bs = fib.bs;
    bs->F[b][0] = F[0];
    bs->F[b][1] = F[1];
    bs->C[b][0] = C0;
    bs->C[b][1] = C1;
    if (b % fib.chain_len <= fib.chain_len - 2) {  // bond (b, b+1) inside the fiber
        const double strain = fabs(B.L[b] - fib.l0) / fib.l0;
        if (!(strain <= 0.5)) atomicOr(&bs->health, FPD_HEALTH_STRAIN);
        atomic_max_nonneg(&bs->max_strain_bits, strain);
    }
}

// ------------------------------------------------- bead list for a tile (LDS) ------
// One bead of a tile's list: its position as the fiber arithmetic of T sees it and its
// Eq. (4) coefficients C_b = F_b / A_b rounded to T.
template <typename T> struct TileBead {
    BeadGeom<T> g;
    T C[2];
};
// Ordered compaction of the beads whose support box meets the tile's columns
// [cx0, cx0 + cw) and rows [ry0, ry0 + rh): bead order is kept, so per-node sums over
// beads run in the same order as in a full loop.  Bond tangents and forces are computed
// only when some bead is near (with several fibers most window tiles have none).
template <typename T>
__device__ inline int gather_beads(const Fiber& fib, int nx, int ny, bool per, int cx0, int cw,
                                   int ry0, int rh, TileBead<T>* sB, int* sIdx, int* s_wave,
                                   Bonds& B, bool forces_ready) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nthreads = blockDim.x * blockDim.y;
    const int lane = tid & 63, wave = tid >> 6, nwaves = (nthreads + 63) >> 6;
    const BeadState* bs = fib.bs;
    int total = 0;
    for (int base = 0; base < fib.n; base += nthreads) {
        const int b = base + tid;
        bool hit = false;
        double Rx = 0.0, Ry = 0.0;
        if (b < fib.n) {
            Rx = bs->R[b][0];
            Ry = bs->R[b][1];
            int i0, w, j0, j1;
            bead_box(Rx, Ry, fib.rc, nx, ny, per, i0, w, j0, j1);
            const bool rows_hit = per ? (j0 <= j1 && cols_overlap(ry0, rh, j0, j1 - j0 + 1, ny))
                                      : ((j0 <= j1) && (j0 <= ry0 + rh - 1) && (j1 >= ry0));
            hit = rows_hit && cols_overlap(cx0, cw, i0, w, nx);
        }
        const unsigned long long m = __ballot(hit);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) s_wave[wave] = __popcll(m);
        __syncthreads();
        int off = total, chunk = 0;
        for (int w = 0; w < nwaves; ++w) {
            if (w < wave) off += s_wave[w];
            chunk += s_wave[w];
        }
        if (hit) {
            sB[off + before].g = BeadGeom<T>::make(Rx, Ry, nx, ny, per);
            sIdx[off + before] = b;
        }
        total += chunk;
        __syncthreads();
    }
    if (total == 0) return 0;  // block-uniform
    if (forces_ready) {
        for (int i = tid; i < total; i += nthreads) {
            const int b = sIdx[i];
            sB[i].C[0] = (T)bs->C[b][0];
            sB[i].C[1] = (T)bs->C[b][1];
        }
    } else {
        fill_bonds(bs, fib.n, B);
        for (int i = tid; i < total; i += nthreads) {
            // F_b^n from the current positions, C_b = F_b / A_b (Eq. 4 coefficient)
            const int b = sIdx[i];
            double F[2];
            bead_force(B, fib.chain_len, b, fib.ks_l02, fib.l0, fib.kb, fib.fext, F);
            if (bs->ev_k > 0.0) {  // the excluded volume, summed by ev_kernel this step
                F[0] += bs->Fev[b][0];
                F[1] += bs->Fev[b][1];
            }
            const double A = bs->A[b];
            const double C0 = F[0] / A, C1 = F[1] / A;
            sB[i].C[0] = (T)C0;
            sB[i].C[1] = (T)C1;
            int ox, oy;
            sB[i].g.node(nx, ny, per, ox, oy);
            if (ox >= cx0 && ox < cx0 + cw && oy >= ry0 && oy < ry0 + rh)
                own_bead(fib, B, b, F, C0, C1);
        }
    }
    __syncthreads();
    return total;
}

// ------------------------------------------------------------- fused lattice step ---

// LDS of a lattice tile: the beads near it (TileBead records of the tile's precision) and
// their Eq. (4) coefficients.
struct TileLds {
    alignas(16) unsigned char beads[kMaxBeads * sizeof(TileBead<double>)];
    Bonds bonds;
    int idx[kMaxBeads];
    int wave[16];
};

// The fiber's support window for this step (empty without a fiber).
__device__ inline Window tile_window(const StepArgs& a) {
    if (a.fib.n <= 0) return Window{0, 0, 0, 0, false};
    return decode_window(a.fib.bs->win[a.parity], a.L.nx, a.L.ny, a.L.periodic != 0,
                         a.fib.rect_wmax,
                         a.fib.rect_hmax);
}

// One axis of a partition from a window axis (start x0, length w on n nodes) grown by m
// nodes: wrapping along a periodic axis, clipped at the walls otherwise.
__device__ inline void grow_axis(int x0, int w, int m, int n, bool wrap, int& p0, int& pw) {
    if (w <= 0) {
        p0 = 0;
        pw = 0;
    } else if (wrap) {
        pw = w + 2 * m >= n ? n : w + 2 * m;
        p0 = pw == n ? 0 : imod(x0 - m, n);
    } else {
        p0 = max(x0 - m, 0);
        pw = min(x0 + w - 1 + m, n - 1) - p0 + 1;
    }
}

// Whether a window axis grown by m nodes lies inside a partition axis (p0, pw).
__device__ inline bool axis_inside(int x0, int w, int m, int p0, int pw, int n, bool wrap) {
    if (w <= 0) return true;
    if (wrap) {
        if (pw >= n) return true;
        return w + 2 * m <= pw && imod(x0 - m - p0, n) + w + 2 * m <= pw;
    }
    const int lo = max(x0 - m, 0), hi = min(x0 + w - 1 + m, n - 1);
    return lo >= p0 && hi <= p0 + pw - 1;
}

// The bookkeeping of a step, by every thread of one block: the step's bead kernel fills
// the other window and occupancy slots from scratch, and the next step's partition is this
// step's window grown by kPartMargin.  check (a split step): the partition this step was
// split by held the window and the ring of one node around it, else FPD_HEALTH_SUPPORT
// (fiber tiles outside it then ran without their fiber terms).
__device__ inline void step_duties(const StepArgs& a, const Window& win, bool check) {
    BeadState* bs = a.fib.bs;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    if (tid == 0) {
        int* nxt = bs->win[1 - a.parity];
        nxt[0] = 0x7fffffff;
        nxt[1] = -0x7fffffff;
        nxt[2] = 0x7fffffff;
        nxt[3] = -0x7fffffff;
        unsigned h = win.clamped ? FPD_HEALTH_SUPPORT : 0u;
        const int nx = a.L.nx, ny = a.L.ny;
        const bool per = a.L.periodic != 0;
        const int ww = win.h > 0 ? win.w : 0;
        if (check) {
            const int* P = bs->part[a.parity];
            if (!axis_inside(win.x0, ww, 1, P[0], P[1], nx, true) ||
                !axis_inside(win.y0, win.h, 1, P[2], P[3], ny, per))
                h |= FPD_HEALTH_SUPPORT;
        }
        int* Q = bs->part[1 - a.parity];
        grow_axis(win.x0, ww, kPartMargin, nx, true, Q[0], Q[1]);
        grow_axis(win.y0, ww > 0 ? win.h : 0, kPartMargin, ny, per, Q[2], Q[3]);
        if (Q[1] == 0 || Q[3] == 0) Q[1] = Q[3] = 0;
        if (h) atomicOr(&bs->health, h);
    }
    for (int i = tid; i < occ_words(a.fib); i += blockDim.x * blockDim.y)
        bs->occ[1 - a.parity][i] = 0u;
}

// The tiles a partition axis (p0, pw) meets, for tiles of width t (the last of `tiles` is
// n - (tiles - 1) t wide): the first and how many, at most cap (the fiber kernel's grid).
__device__ inline void part_axis(int p0, int pw, int n, int t, int tiles, int cap, int& first,
                                 int& count) {
    first = 0;
    count = 0;
    if (pw <= 0) return;
    if (pw >= n) {
        count = min(tiles, cap);
        return;
    }
    const int last = p0 + pw - 1;  // past n: the wrapped part, from tile 0 on
    const int tl = last < n ? last / t : tiles + (last - n) / t;
    first = p0 / t;
    count = min(min(tl - first + 1, tiles), cap);
}

struct TileSpan {
    int tx0, ntx, ty0, nty, tiles_y;
};

// The tiles of this step's partition (a run modulo the tiling along each axis); the fluid
// and the fiber kernels of a step take exactly this set apart, so every tile runs once.
__device__ inline TileSpan part_span(const StepArgs& a, int tw) {
    const int* P = a.fib.bs->part[a.parity];
    TileSpan sp;
    sp.tiles_y = a.n_tiles / a.tiles_x;
    part_axis(P[0], P[1], a.L.nx, tw, a.tiles_x, a.part_gw, sp.tx0, sp.ntx);
    part_axis(P[2], P[3], a.L.ny, a.rows_per_block, sp.tiles_y, a.part_gh, sp.ty0, sp.nty);
    if (sp.ntx == 0 || sp.nty == 0) sp.ntx = sp.nty = 0;
    return sp;
}

__device__ inline bool in_span(const TileSpan& sp, int tx, int ty, int tiles_x) {
    return imod(tx - sp.tx0, tiles_x) < sp.ntx && imod(ty - sp.ty0, sp.tiles_y) < sp.nty;
}

// Step (1) at one node (x, y) of a fiber tile: phi_i^n (Eq. 2), eta^n (Eq. 1, with a
// fixed profile phi_s(y) if one is set) and the relaxation rates, f^n (Eq. 4, plus the
// uniform body force), recorded in the force window.  Fx, Fy are overwritten; s_nu and
// s_q keep the fluid values where sum phi = 0.
template <typename T>
__device__ inline void fiber_node(const StepArgs& a, bool per, const TileBead<T>* sB, int nb,
                                  int x, int y, int wx0, int wy0, int ww, int wh, T& Fx, T& Fy,
                                  T& s_nu, T& s_q) {
    using G = BeadGeom<T>;
    const int nx = a.L.nx, ny = a.L.ny;
    const T rc2 = G::cut2(a.fib.rc2);
    T sphi = T(0), fx = T(0), fy = T(0);
    for (int i = 0; i < nb; ++i) {
        const T r2 = sB[i].g.r2(x, y, nx, ny, per);
        if (!(r2 < rc2)) continue;
        const T ph = G::phi(r2, a.fib.a, a.fib.xi, a.fib.inv_xi);
        sphi += ph;
        fx += ph * sB[i].C[0];
        fy += ph * sB[i].C[1];
    }
    Fx = fx + (T)a.gx;
    Fy = fy + (T)a.gy;
    if (a.row_phi) sphi += (T)a.row_phi[y];  // fixed profile phi_s(y) (sandwich slabs)
    if (a.fib.clamp && sphi > T(1)) sphi = T(1);
    if (sphi > T(0)) {  // else the fluid rates, exactly as on the other tiles
        const T nu_f = (T)a.fib.nu_f;
        const T eta = nu_f + ((T)a.fib.nu_s - nu_f) * sphi;
        s_nu = recip(T(3) * eta + T(0.5));
        s_q = a.fib.s_q_fixed > 0.0 ? (T)a.fib.s_q_fixed
                                    : quot(T(8) * (T(2) - s_nu), T(8) - s_nu);
    }
    const int wi = imod(x - wx0, nx), wj = per ? imod(y - wy0, ny) : y - wy0;
    if (wi < ww && wj >= 0 && wj < wh) {
        T* rf = (T*)a.fib.rect_f + 2 * ((long long)wj * a.fib.rect_wmax + wi);
        rf[0] = Fx;
        rf[1] = Fy;
    }
}

// Boundary in y as a compile-time choice: kWalls and kPeriodic fix it (the code for the
// other one drops out), kAnyBoundary reads it from the arguments (batches that mix both).
constexpr int kWalls = 0, kPeriodic = 1, kAnyBoundary = 2;

__device__ inline bool periodic_of(int bc, const StepArgs& a) {
    return bc == kAnyBoundary ? a.L.periodic != 0 : bc == kPeriodic;
}

// One tile (block_x nodes on rows_per_block rows) of one simulation.
// Must be reached by every thread of the block (it synchronises when the tile meets the
// fiber).  In a one-kernel step (PART = kPartAll) the tile numbered 0 also does the step's
// bookkeeping (step_duties); a fluid-part tile (kPartFluid) reads no fiber state at all.
// FR: the forces F^n and F/A of this step come from a forces kernel (a batch); else the
// tiles near the fiber compute them from the positions.
template <int ST, int SPT, int BC, bool FR, int PART = kPartAll>
__device__ inline void lattice_tile(const StepArgs& a, const Window& win, int tile,
                                    TileLds& lds) {
    using Cd = Codec<ST>;
    const bool per = periodic_of(BC, a);
    using T = typename Cd::T;
    using S = typename Cd::store_t;
    TileBead<T>* sB = (TileBead<T>*)lds.beads;
    int* s_wave = lds.wave;
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int bx = blockDim.x;
    const int tw = bx;
    const int xtile = tx * tw;
    const int x = xtile + threadIdx.x;
    const int ytile = ty * a.rows_per_block;
    const int ybase = ytile + threadIdx.y * SPT;
    const int nx = a.L.nx, ny = a.L.ny, stride = a.L.stride;
    const long long plane = a.L.plane;
    const S* __restrict__ src = (const S*)a.src;
    S* __restrict__ dst = (S*)a.dst;
    const T u6 = (T)a.u6;
    const T s_e = (T)a.s_e, s_eps = (T)a.s_eps;

    // the first row's populations are requested before the fiber checks below, so their
    // latency overlaps the reads of the window, the occupancy bitmap and the bead list
    T g0[9];
    if (x < nx && ybase < ny) pull<Cd>(src, nx, ny, stride, plane, x, ybase, per, u6, g0);
    // a fluid-part tile checks the partition while those loads are in flight
    if constexpr (PART == kPartFluid)
        if (in_span(part_span(a, tw), tx, ty, a.tiles_x)) return;  // block-uniform

    // Block-uniform: does this tile meet the fiber's support window?
    int nb = 0, wx0 = 0, wy0 = 0, ww = 0, wh = 0;
    bool fiber_tile = false;
    if (PART != kPartFluid && a.fib.n > 0) {
        wx0 = win.x0;
        wy0 = win.y0;
        ww = win.w;
        wh = win.h;
        if (PART == kPartAll && tile == 0) step_duties(a, win, false);
        const bool rows_hit =
            per ? cols_overlap(ytile, a.rows_per_block, wy0, wh, ny)
                         : (ytile <= wy0 + wh - 1 && ytile + a.rows_per_block - 1 >= wy0);
        fiber_tile = ww > 0 && wh > 0 && rows_hit && cols_overlap(xtile, tw, wx0, ww, nx) &&
                     occ_hit(a.fib, a.parity, xtile, tw, ytile, a.rows_per_block, nx, ny);
        if (fiber_tile)
            nb = gather_beads<T>(a.fib, nx, ny, per, xtile, tw, ytile, a.rows_per_block, sB,
                                 lds.idx, s_wave, lds.bonds, FR);
    }

    // a tile inside the window that no bead's support reaches is fluid only: no node of
    // it lies in a support box, so its force-window entries are never read
    if (fiber_tile && nb == 0) fiber_tile = false;
    // a fixed profile phi_s(y) makes every tile take the fiber path (with no beads to
    // gather outside the window); plain: no force and no viscosity change on this tile
    if (PART != kPartFluid && a.row_phi) fiber_tile = true;
    const bool plain = !fiber_tile && a.gx == 0.0 && a.gy == 0.0;  // block-uniform
#pragma unroll
    for (int r = 0; r < SPT; ++r) {
        const int y = ybase + r;
        if (x >= nx || y >= ny) continue;
        // the fiber terms first: the populations of later rows are not live during the
        // bead loop
        T Fx = (T)a.gx, Fy = (T)a.gy, s_nu = (T)a.s_nu_f, s_q = (T)a.s_q_f;
        if (fiber_tile)
            fiber_node<T>(a, per, sB, nb, x, y, wx0, wy0, ww, wh, Fx, Fy, s_nu, s_q);
        T g[9];
        if (r == 0) {
#pragma unroll
            for (int k = 0; k < 9; ++k) g[k] = g0[k];
        } else {
            pull<Cd>(src, nx, ny, stride, plane, x, y, per, u6, g);
        }
        if (plain)  // no force anywhere on this tile: the unforced collision
            mrt_collide<T, false>(g, T(0), T(0), (T)a.s_nu_f, (T)a.s_q_f, s_e, s_eps);
        else
            mrt_collide<T>(g, Fx, Fy, s_nu, s_q, s_e, s_eps);
        S* o = dst + (long long)y * stride + x;
#pragma unroll
        for (int k = 0; k < 9; ++k) Cd::store(o + k * plane, g[k]);
    }
}

// lattice_tile for 2-byte storage: a tile is G * block_x nodes wide and each lane updates
// G neighbouring nodes with the same per-node arithmetic as the one-node path.
template <int ST, int SPT, int BC, bool FR, int PART = kPartAll>
__device__ inline void lattice_tile_group(const StepArgs& a, const Window& win, int tile,
                                          TileLds& lds) {
    using Cd = Codec<ST>;
    const bool per = periodic_of(BC, a);
    using T = typename Cd::T;
    constexpr int G = nodes_per_lane(ST);
    static_assert(sizeof(typename Cd::store_t) == 2 && (G == 2 || G == 4),
                  "group path is for 2-byte storage");
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int tw = G * (int)blockDim.x;
    const int xtile = tx * tw;
    const int x0 = xtile + G * (int)threadIdx.x;
    const int lane = (int)threadIdx.x & 63;
    const bool first = lane == 0, last = lane == 63;
    const int ytile = ty * a.rows_per_block;
    const int ybase = ytile + threadIdx.y * SPT;
    const int nx = a.L.nx, ny = a.L.ny, stride = a.L.stride;
    const long long plane = a.L.plane;
    const uint16_t* __restrict__ src = (const uint16_t*)a.src;
    uint16_t* __restrict__ dst = (uint16_t*)a.dst;
    // the pulled values and the collision in the codec's units (scaled for FP16)
    constexpr bool kScaled = Cd::kScaledCollide;
    const T u6 = kScaled ? (T)(a.u6 * 16384.0) : (T)a.u6;
    const T s_e = (T)a.s_e, s_eps = (T)a.s_eps;

    int nb = 0, wx0 = 0, wy0 = 0, ww = 0, wh = 0;
    bool fiber_tile = false;
    if (PART != kPartFluid && a.fib.n > 0) {
        wx0 = win.x0;
        wy0 = win.y0;
        ww = win.w;
        wh = win.h;
        if (PART == kPartAll && tile == 0) step_duties(a, win, false);
        const bool rows_hit =
            per ? cols_overlap(ytile, a.rows_per_block, wy0, wh, ny)
                         : (ytile <= wy0 + wh - 1 && ytile + a.rows_per_block - 1 >= wy0);
        fiber_tile = ww > 0 && wh > 0 && rows_hit && cols_overlap(xtile, tw, wx0, ww, nx) &&
                     occ_hit(a.fib, a.parity, xtile, tw, ytile, a.rows_per_block, nx, ny);
        if (fiber_tile)
            nb = gather_beads<T>(a.fib, nx, ny, per, xtile, tw, ytile, a.rows_per_block,
                                 (TileBead<T>*)lds.beads, lds.idx, lds.wave, lds.bonds, FR);
    }

    // a tile inside the window that no bead's support reaches is fluid only: no node of
    // it lies in a support box, so its force-window entries are never read
    if (fiber_tile && nb == 0) fiber_tile = false;
    // a fixed profile phi_s(y) makes every tile take the fiber path (with no beads to
    // gather outside the window); plain: no force and no viscosity change on this tile
    if (PART != kPartFluid && a.row_phi) fiber_tile = true;
    const bool plain = !fiber_tile && a.gx == 0.0 && a.gy == 0.0;  // block-uniform
#pragma unroll
    for (int r = 0; r < SPT; ++r) {
        const int y = ybase + r;
        if (y >= ny) continue;  // uniform over a wave (its lanes share one row)
        // the fiber terms first: the populations are not live during the bead loops
        T Fx[G], Fy[G], s_nu[G], s_q[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            Fx[i] = (T)a.gx;
            Fy[i] = (T)a.gy;
            s_nu[i] = (T)a.s_nu_f;
            s_q[i] = (T)a.s_q_f;
            if (fiber_tile && x0 + i < nx)
                fiber_node<T>(a, per, (const TileBead<T>*)lds.beads, nb, x0 + i, y, wx0, wy0,
                              ww, wh, Fx[i], Fy[i], s_nu[i], s_q[i]);
        }
        T g[G][9];
        pull_group<Cd, G>(src, nx, ny, stride, plane, x0, y, per, first, last, u6, g);
        if (x0 >= nx) continue;
        uint32_t bits[9][G / 2];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if constexpr (kScaled) {
                if (plain)
                    mrt_collide_scaled<T, false>(g[i], T(0), T(0), (T)a.s_nu_f, (T)a.s_q_f,
                                                 s_e, s_eps);
                else
                    mrt_collide_scaled<T>(g[i], Fx[i], Fy[i], s_nu[i], s_q[i], s_e, s_eps);
            } else {
                if (plain)  // no force anywhere on this tile: the unforced collision
                    mrt_collide<T, false>(g[i], T(0), T(0), (T)a.s_nu_f, (T)a.s_q_f, s_e,
                                          s_eps);
                else
                    mrt_collide<T>(g[i], Fx[i], Fy[i], s_nu[i], s_q[i], s_e, s_eps);
            }
        }
#pragma unroll
        for (int i = 0; i < G; i += 2)
#pragma unroll
            for (int k = 0; k < 9; ++k) bits[k][i >> 1] = Cd::pack2_scaled(g[i][k], g[i + 1][k]);
        uint16_t* o = dst + (long long)y * stride + x0;
        if (x0 + G - 1 < nx) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                if constexpr (G == 2) {
                    __builtin_nontemporal_store(bits[k][0], (uint32_t*)(o + k * plane));
                } else {
                    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                    u32x2 v;
                    v.x = bits[k][0];
                    v.y = bits[k][1];
                    __builtin_nontemporal_store(v, (u32x2*)(o + k * plane));
                }
            }
        } else {
            for (int i = 0; i < G && x0 + i < nx; ++i)
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    __builtin_nontemporal_store(
                        (uint16_t)(bits[k][i >> 1] >> (16 * (i & 1))), o + i + k * plane);
        }
    }
}

template <int ST, int SPT, int BC, bool FR, int PART = kPartAll>
__device__ inline void tile_any(const StepArgs& a, const Window& win, int tile, TileLds& lds) {
    if constexpr (nodes_per_lane(ST) > 1)
        lattice_tile_group<ST, SPT, BC, FR, PART>(a, win, tile, lds);
    else
        lattice_tile<ST, SPT, BC, FR, PART>(a, win, tile, lds);
}

// Called by every thread of one block ahead of the step's lattice kernel, and only while a
// recording runs, so the lattice kernels carry no trace of it.
__device__ inline void record_ends(const StepArgs& a) {
    RecordBuf* r = a.rec;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const unsigned long long n = r->count;
    if (n % (unsigned long long)r->every == 0ull) {
        const int width = 1 + 4 * r->fibers;
        double* rec = r->data + (size_t)((n / r->every) % (unsigned long long)r->cap) * width;
        if (tid == 0) rec[0] = (double)n;
        const int L = a.fib.chain_len;
        for (int c = tid; c < r->fibers; c += blockDim.x * blockDim.y) {
            const double(*R)[2] = a.fib.bs->R + c * L;
            double cx = 0.0, cy = 0.0;
            for (int i = 0; i < L; ++i) {
                cx += R[i][0];
                cy += R[i][1];
            }
            rec[1 + 4 * c] = R[L - 1][0] - R[0][0];
            rec[2 + 4 * c] = R[L - 1][1] - R[0][1];
            rec[3 + 4 * c] = cx / L;
            rec[4 + 4 * c] = cy / L;
        }
    }
    __syncthreads();  // every thread has read the count
    if (tid == 0) r->count = n + 1ull;
}

__global__ void __launch_bounds__(kBeadThreads) record_kernel(StepArgs a) {
    record_ends(a);
}

template <int ST, int SPT, int BC>
__global__ void __launch_bounds__(256) step_kernel(StepArgs a) {
    __shared__ TileLds lds;
    const int tile = a.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    tile_any<ST, SPT, BC, false>(a, tile_window(a), tile, lds);
}

// A split step: the lattice step as two kernels over complementary tile sets.  fluid_kernel
// (the full grid, in step_kernel's block order) updates the tiles outside the step's
// partition and reads no fiber state, so it runs while the bead kernel of the step before
// still finishes; fiber_kernel (a.part_gw * a.part_gh blocks over the partition, block 0
// also doing the step's bookkeeping) updates the tiles inside it after that bead kernel.
// A tile runs the same code in either as in step_kernel, so the results are the same bits.
template <int ST, int SPT, int BC>
__global__ void __launch_bounds__(256) fluid_kernel(StepArgs a) {
    __shared__ TileLds lds;
    const int tile = a.xcd_remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if constexpr (nodes_per_lane(ST) > 1) {  // (the one-node tiles check after their loads)
        const TileSpan sp = part_span(a, nodes_per_lane(ST) * (int)blockDim.x);
        if (in_span(sp, tile % a.tiles_x, tile / a.tiles_x, a.tiles_x)) return;
    }
    tile_any<ST, SPT, BC, false, kPartFluid>(a, Window{0, 0, 0, 0, false}, tile, lds);
}

template <int ST, int SPT, int BC>
__global__ void __launch_bounds__(256) fiber_kernel(StepArgs a) {
    __shared__ TileLds lds;
    const Window win = tile_window(a);
    if (blockIdx.x == 0) step_duties(a, win, true);
    const TileSpan sp = part_span(a, nodes_per_lane(ST) * (int)blockDim.x);
    const int ox = (int)blockIdx.x % a.part_gw, oy = (int)blockIdx.x / a.part_gw;
    if (ox >= sp.ntx || oy >= sp.nty) return;  // block-uniform
    const int tx = (sp.tx0 + ox) % a.tiles_x, ty = (sp.ty0 + oy) % sp.tiles_y;
    tile_any<ST, SPT, BC, false, kPartFiber>(a, win, ty * a.tiles_x + tx, lds);
}

// The argument table is read-only while a batch kernel runs: viewing it in the constant
// address space lets the per-simulation arguments come in through scalar loads.
typedef const StepArgs __attribute__((address_space(4))) ConstStepArgs;

__device__ inline StepArgs load_args(const StepArgs* table, int i) {
    const ConstStepArgs* c = (const ConstStepArgs*)table;
    StepArgs a;
    __builtin_memcpy(&a, c + i, sizeof(StepArgs));
    return a;
}

typedef const int __attribute__((address_space(4))) ConstInt;

// A work item's simulation and index from its table (uniform: one scalar load of both).
__device__ inline ItemRef item_ref(const ItemRef* table, int item) {
    const ConstInt* e = (const ConstInt*)(table + item);
    return ItemRef{e[0], e[1]};
}

// Lattice kernel over a batch of simulations of different sizes: one block per (simulation,
// tile) item of the work table, the grid sized to the table, so the blocks resident at any
// moment work on neighbouring tiles of one simulation as in a single-simulation launch.
template <int ST, int SPT, int BC>
__global__ void __launch_bounds__(256) batch_step_kernel(BatchArgs b) {
    __shared__ TileLds lds;
    const int item = blockIdx.x;
    // the entry is read together with the count (one wait for both; the test of e.sim,
    // never negative, keeps its load ahead of the branch): the grid is sized from the
    // count and never exceeds the table's capacity, so the read stays inside it
    const ItemRef e = item_ref(b.tile_items, item);
    if (item >= b.counts[1] || e.sim < 0) return;
    const StepArgs a = load_args(b.args, 2 * e.sim + b.gpar);
    tile_any<ST, SPT, BC, true>(a, tile_window(a), e.local, lds);
}

// ----------------------------------------------------------------- bead kernel -----

// Node t of a bead's support box (columns i0 .. i0 + w - 1, rows from j0, both wrapped),
// its squared distance from the bead in the fiber arithmetic T of the storage (FP64 for
// FPD_F64, FP32 otherwise) and whether it passes the cutoff test: BeadGeom<T>, the same
// evaluation as in the lattice tiles.  t >= total: out.
template <typename T>
__device__ inline void box_node(const Fiber& fib, const BeadGeom<T>& geo, int t, int total,
                                int i0, int w, int j0, int nx, int ny, bool per, int& x, int& y,
                                T& r2, bool& in) {
    x = i0;
    y = j0;
    r2 = T(0);
    in = false;
    if (t < total) {
        y = j0 + t / w;
        if (y >= ny) y -= ny;  // periodic box: rows wrap
        x = i0 + t % w;
        if (x >= nx) x -= nx;
        r2 = geo.r2(x, y, nx, ny, per);
        in = r2 < BeadGeom<T>::cut2(fib.rc2);
    }
}

// phi of one bead at a node that passed the cutoff test (squared distance r2)
template <typename T>
__device__ inline double bead_phi(const Fiber& fib, T r2) {
    return (double)BeadGeom<T>::phi(r2, fib.a, fib.xi, fib.inv_xi);
}

// This bead's share of the next support window and of the occupancy bitmap (slot
// win_out), from its position: integer atomics, so the result does not depend on the
// order in which beads finish.
__device__ inline void publish_support(const Fiber& fib, int win_out, double Rx, double Ry,
                                       int nx, int ny, bool per) {
    if (!bead_sane(Rx, Ry)) return;
    int* nw = fib.bs->win[win_out];
    const int lo = (int)floor(Rx - 0.5 - fib.rc), hi = (int)ceil(Rx - 0.5 + fib.rc);
    const int jlo = (int)floor(Ry - 0.5 - fib.rc), jhi = (int)ceil(Ry - 0.5 + fib.rc);
    atomicMin(&nw[0], lo);
    atomicMax(&nw[1], hi);
    atomicMin(&nw[2], jlo);
    atomicMax(&nw[3], jhi);
    occ_mark(fib, win_out, lo, hi, jlo, jhi, nx, ny, per);
}

// One block per bead.  With do_velocity: V_i^{n+1} = sum_x phi_i^n (j^{n+1} + f^n / 2) /
// rho^{n+1} / A_i^n over the bead's support box (Eq. 5, FP64 sums), then the Euler update
// R_i^{n+1} = R_i^n + V_i^{n+1}.  Always: A_i = sum_x phi_i at the (new) position.
// VB nodes per thread and pass in the velocity phase: their loads are issued together, so
// a pass waits for memory once (short latency chains for a few beads), at the cost of
// registers (fewer resident blocks when a batch has thousands of beads).  The loads depend
// only on the cutoff test, so phi is evaluated while they are in flight.  The sums run
// over kBeadLanes virtual lanes (NT threads of R = kBeadLanes / NT lanes each): lane v
// takes nodes t = v, v + kBeadLanes, ... in increasing t, whatever VB and NT.
template <int ST, int VB, int NT>
__device__ inline void bead_block(const StepArgs& a, int b, int do_velocity, int win_out,
                                  double* scratch, double* s_R) {
    constexpr int R = kBeadLanes / NT;
    using Cd = Codec<ST>;
    using T = typename Cd::T;
    using S = typename Cd::store_t;
    const Fiber& fib = a.fib;
    BeadState* bs = fib.bs;
    const int tid = threadIdx.x;
    const int nx = a.L.nx, ny = a.L.ny;
    const bool per = a.L.periodic != 0;
    double Rx = bs->R[b][0], Ry = bs->R[b][1];
    // A_i^n and the support window with the position, so the three loads overlap
    const double A_old = do_velocity ? bs->A[b] : 0.0;
    int wraw[4] = {1, 0, 1, 0};
    if (do_velocity)
#pragma unroll
        for (int q = 0; q < 4; ++q) wraw[q] = bs->win[a.parity][q];

    double Vx = 0.0, Vy = 0.0;  // valid in thread 0
    if (do_velocity) {
        int i0, w, j0, j1;
        bead_box(Rx, Ry, fib.rc, nx, ny, per, i0, w, j0, j1);
        const BeadGeom<T> geo = BeadGeom<T>::make(Rx, Ry, nx, ny, per);
        const int rows = j1 - j0 + 1;
        const int total = (rows > 0 && w > 0) ? rows * w : 0;
        const Window win = decode_window(wraw, nx, ny, per, fib.rect_wmax, fib.rect_hmax);
        const int wx0 = win.x0, wy0 = win.y0, ww = win.w, wh = win.h;
        const T* rf = (const T*)fib.rect_f;
        const S* cur = (const S*)a.dst;
        double sx[R], sy[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            sx[r] = 0.0;
            sy[r] = 0.0;
            for (int t0 = tid + r * NT; t0 < total; t0 += VB * kBeadLanes) {
                double ph[VB];
                T r2[VB];
                bool in[VB];
                int ii[VB], jj[VB];
                T g[VB][9];
                T fw[VB][2];
#pragma unroll
                for (int u = 0; u < VB; ++u)
                    box_node<T>(fib, geo, t0 + u * kBeadLanes, total, i0, w, j0, nx, ny, per,
                                ii[u], jj[u], r2[u], in[u]);
#pragma unroll
                for (int u = 0; u < VB; ++u) {
                    fw[u][0] = (T)a.gx;  // outside the window f^n is the body force alone
                    fw[u][1] = (T)a.gy;
                    if (in[u]) {
                        pull<Cd>(cur, nx, ny, a.L.stride, a.L.plane, ii[u], jj[u], per,
                                 (T)a.u6, g[u]);
                        // f^n at this node from the window the lattice kernel filled (the
                        // window covers every support box unless it was clamped, which
                        // raises FPD_HEALTH_SUPPORT)
                        const int wi = imod(ii[u] - wx0, nx);
                        const int wj = per ? imod(jj[u] - wy0, ny) : jj[u] - wy0;
                        if (wi < ww && wj >= 0 && wj < wh) {
                            const T* fp = rf + 2 * ((long long)wj * fib.rect_wmax + wi);
                            fw[u][0] = fp[0];
                            fw[u][1] = fp[1];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < VB; ++u)
                    ph[u] = in[u] ? bead_phi<T>(fib, r2[u]) : 0.0;
#pragma unroll
                for (int u = 0; u < VB; ++u) {
                    if (ph[u] == 0.0) continue;
                    double drho = 0.0;
#pragma unroll
                    for (int k = 0; k < 9; ++k) drho += (double)g[u][k];
                    const double jx = ((double)g[u][1] - (double)g[u][3]) +
                                      ((double)g[u][5] - (double)g[u][6]) -
                                      ((double)g[u][7] - (double)g[u][8]);
                    const double jy = ((double)g[u][2] - (double)g[u][4]) +
                                      ((double)g[u][5] + (double)g[u][6]) -
                                      ((double)g[u][7] + (double)g[u][8]);
                    const double rho = 1.0 + drho;
                    sx[r] += ph[u] * ((jx + 0.5 * (double)fw[u][0]) / rho);
                    sy[r] += ph[u] * ((jy + 0.5 * (double)fw[u][1]) / rho);
                }
            }
        }
        double Sx, Sy;
        lanes_sum2<R>(sx, sy, Sx, Sy, scratch);
        if (tid == 0) {
            Vx = Sx / A_old;
            Vy = Sy / A_old;
            bs->V[b][0] = Vx;
            bs->V[b][1] = Vy;
            s_R[0] = Rx + Vx;  // forward Euler, dt = 1
            s_R[1] = Ry + Vy;
            bs->R[b][0] = s_R[0];
            bs->R[b][1] = s_R[1];
        }
        __syncthreads();
        Rx = s_R[0];
        Ry = s_R[1];
        // the next support window and occupancy cells from the new position, by the
        // block's last thread (its wave has the fewest nodes in the A_i sum below); the
        // atomics complete while the block sums A_i
        if (tid == NT - 1) publish_support(fib, win_out, Rx, Ry, nx, ny, per);
    }

    int i0, w, j0, j1;
    bead_box(Rx, Ry, fib.rc, nx, ny, per, i0, w, j0, j1);
    const BeadGeom<T> geo = BeadGeom<T>::make(Rx, Ry, nx, ny, per);
    const int rows = j1 - j0 + 1;
    const int total = (rows > 0 && w > 0) ? rows * w : 0;
    double sa[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        sa[r] = 0.0;
        for (int t = tid + r * NT; t < total; t += kBeadLanes) {
            int x, y;
            T r2;
            bool in;
            box_node<T>(fib, geo, t, total, i0, w, j0, nx, ny, per, x, y, r2, in);
            if (in) sa[r] += bead_phi<T>(fib, r2);
        }
    }
    const double A_new = lanes_sum<R>(sa, scratch);
    if (tid == 0) {
        bs->A[b] = A_new;
        // the support window (after the Euler update, else here) and the health bits
        if (!do_velocity) {
            publish_support(fib, win_out, Rx, Ry, nx, ny, per);
            Vx = bs->V[b][0];
            Vy = bs->V[b][1];
        }
        unsigned h = 0u;
        if (!isfinite(Rx) || !isfinite(Ry) || !isfinite(Vx) || !isfinite(Vy) ||
            !isfinite(A_new))
            h |= FPD_HEALTH_NAN;
        if (Vx * Vx + Vy * Vy > 0.09 / 3.0) h |= FPD_HEALTH_MACH;
        if (!per && (Ry - fib.a - fib.xi < 0.0 || Ry + fib.a + fib.xi > (double)ny))
            h |= FPD_HEALTH_WALL;
        if (h) atomicOr(&bs->health, h);
    }
}

template <int ST>
__global__ void __launch_bounds__(kBeadBlock) bead_kernel(StepArgs a, int do_velocity,
                                                          int win_out) {
    __shared__ double scratch[2 * (kBeadLanes / 64)];
    __shared__ double s_R[2];
    bead_block<ST, kBeadVelBatch, kBeadBlock>(a, blockIdx.x, do_velocity, win_out, scratch,
                                              s_R);
}

// Bead kernel over a batch: one block per (simulation, bead) item.
template <int ST>
__global__ void __launch_bounds__(kBatchBeadBlock) batch_bead_kernel(BatchArgs b) {
    __shared__ double scratch[2 * (kBeadLanes / 64)];
    __shared__ double s_R[2];
    const int item = blockIdx.x;
    const ItemRef e = item_ref(b.bead_items, item);  // with the count, as in the lattice kernel
    if (item >= b.counts[2] || e.sim < 0) return;
    const StepArgs a = load_args(b.args, 2 * e.sim + b.gpar);
    bead_block<ST, kBatchBeadVelBatch, kBatchBeadBlock>(a, e.local, 1, 1 - a.parity,
                                                        scratch, s_R);
}

// Excluded-volume forces of every bead at the step's start (one block).
__global__ void __launch_bounds__(kBeadThreads) ev_kernel(StepArgs a) {
    const Fiber& fib = a.fib;
    for (int t = threadIdx.x; t < fib.n; t += blockDim.x) {
        double F[2] = {0.0, 0.0};
        ev_force(fib, a.L.nx, a.L.ny, a.L.periodic != 0, t, F);
        fib.bs->Fev[t][0] = F[0];
        fib.bs->Fev[t][1] = F[1];
    }
}

// Forces F^n and C = F / A for every bead (read-back; the lattice kernel computes the same
// values for the beads near its tiles).
__global__ void __launch_bounds__(kBeadThreads) forces_kernel(StepArgs a) {
    __shared__ Bonds B;
    const Fiber& fib = a.fib;
    BeadState* bs = fib.bs;
    fill_bonds(bs, fib.n, B);
    for (int t = threadIdx.x; t < fib.n; t += blockDim.x) {
        double F[2];
        bead_force(B, fib.chain_len, t, fib.ks_l02, fib.l0, fib.kb, fib.fext, F);
        ev_force(fib, a.L.nx, a.L.ny, a.L.periodic != 0, t, F);
        bs->F[t][0] = F[0];
        bs->F[t][1] = F[1];
        bs->C[t][0] = F[0] / bs->A[t];
        bs->C[t][1] = F[1] / bs->A[t];
    }
}

// ---------------------------------------------------- conversions and read-back ----

__device__ inline int ex_of(int k) {
    return (k == 1 || k == 5 || k == 8) ? 1 : ((k == 3 || k == 6 || k == 7) ? -1 : 0);
}
__device__ inline int ey_of(int k) {
    return (k == 2 || k == 5 || k == 6) ? 1 : ((k == 4 || k == 7 || k == 8) ? -1 : 0);
}
__device__ inline int opp_of(int k) {
    return k == 0 ? 0 : (k < 5 ? ((k + 1) & 3) + 1 : ((k - 3) & 3) + 5);
}

// Post-collision storage whose pull gives the pre-collision f64[9][ny][nx].
template <int ST>
__global__ void unstream_kernel(Lattice L, double u_wall, const double* __restrict__ f64,
                                typename Codec<ST>::store_t* __restrict__ dst) {
    using Cd = Codec<ST>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= L.nx || y >= L.ny) return;
    const long long S = (long long)L.nx * L.ny;
    for (int k = 0; k < 9; ++k) {
        int yd = y + ey_of(k);
        if (L.periodic) yd = imod(yd, L.ny);
        double v;
        if (yd >= 0 && yd < L.ny) {
            const int xd = imod(x + ex_of(k), L.nx);
            v = f64[k * S + (long long)yd * L.nx + xd] - lattice_w(k);
        } else {
            const int kb = opp_of(k);
            const double uw = ey_of(kb) > 0 ? -u_wall : u_wall;
            v = f64[kb * S + (long long)y * L.nx + x] - lattice_w(kb) -
                6.0 * lattice_w(kb) * ex_of(kb) * uw;
        }
        dst[k * L.plane + (long long)y * L.stride + x] = Cd::from_f64(v);
    }
}

template <int ST>
__global__ void stream_out_kernel(Lattice L, double u_wall, const typename Codec<ST>::store_t* src,
                                  double* __restrict__ f64) {
    using Cd = Codec<ST>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= L.nx || y >= L.ny) return;
    // decode in FP64 so the wall term is added exactly once, in double
    const int xm = (x == 0) ? L.nx - 1 : x - 1, xp = (x == L.nx - 1) ? 0 : x + 1;
    const long long P = L.plane;
    const long long S_ = (long long)L.nx * L.ny;
    auto at = [&](int k, int xx, int yy) -> double {
        return Cd::to_f64(src[k * P + (long long)yy * L.stride + xx]);
    };
    const double u6 = u_wall / 6.0;
    const int ym = y > 0 ? y - 1 : L.ny - 1, yp = y < L.ny - 1 ? y + 1 : 0;
    double g[9];
    g[0] = at(0, x, y);
    g[1] = at(1, xm, y);
    g[3] = at(3, xp, y);
    if (y > 0 || L.periodic) {
        g[2] = at(2, x, ym);
        g[5] = at(5, xm, ym);
        g[6] = at(6, xp, ym);
    } else {
        g[2] = at(4, x, y);
        g[5] = at(7, x, y) - u6;
        g[6] = at(8, x, y) + u6;
    }
    if (y < L.ny - 1 || L.periodic) {
        g[4] = at(4, x, yp);
        g[7] = at(7, xp, yp);
        g[8] = at(8, xm, yp);
    } else {
        g[4] = at(2, x, y);
        g[7] = at(5, x, y) - u6;
        g[8] = at(6, x, y) + u6;
    }
    for (int k = 0; k < 9; ++k) f64[k * S_ + (long long)y * L.nx + x] = lattice_w(k) + g[k];
}

// Initial flow of row y: u = 0 or u_x = U (2 y / H - 1) (node centres).
__device__ inline double init_ux(const Lattice& L, double u_wall, int init_flow, int y) {
    return init_flow == FPD_INIT_LINEAR_COUETTE
               ? u_wall * (2.0 * ((double)y + 0.5) / (double)L.ny - 1.0)
               : 0.0;
}

// Equilibrium f_k at rho = 1 and velocity (ux, 0).  The one expression every kernel that
// writes an initial state uses, so they all round alike.
__device__ inline double init_feq(int k, double ux) {
    const double eu = ex_of(k) * ux;
    return lattice_w(k) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * ux * ux);
}

// Equilibrium f at rho = 1 and u = 0 or u_x = U (2 y / H - 1).
__global__ void init_eq_kernel(Lattice L, double u_wall, int init_flow, double* f64) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= L.nx || y >= L.ny) return;
    const double ux = init_ux(L, u_wall, init_flow, y);
    const long long S = (long long)L.nx * L.ny;
    for (int k = 0; k < 9; ++k) f64[k * S + (long long)y * L.nx + x] = init_feq(k, ux);
}

// The initial state straight into a population buffer, with no FP64 staging array: the
// post-collision values whose pull gives the equilibrium of init_eq_kernel (what
// unstream_kernel makes of that kernel's output, value for value).  The equilibrium does
// not depend on x, so a pulled value needs only the row it comes from.
template <int ST>
__global__ void init_state_kernel(Lattice L, double u_wall, int init_flow,
                                  typename Codec<ST>::store_t* __restrict__ dst) {
    using Cd = Codec<ST>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= L.nx || y >= L.ny) return;
    for (int k = 0; k < 9; ++k) {
        int yd = y + ey_of(k);
        if (L.periodic) yd = imod(yd, L.ny);
        double v;
        if (yd >= 0 && yd < L.ny) {
            v = init_feq(k, init_ux(L, u_wall, init_flow, yd)) - lattice_w(k);
        } else {
            const int kb = opp_of(k);
            const double uw = ey_of(kb) > 0 ? -u_wall : u_wall;
            v = init_feq(kb, init_ux(L, u_wall, init_flow, y)) - lattice_w(kb) -
                6.0 * lattice_w(kb) * ex_of(kb) * uw;
        }
        dst[k * L.plane + (long long)y * L.stride + x] = Cd::from_f64(v);
    }
}

// 8-byte zero fill (a kernel rather than a memset, so the fill can sit in a captured graph).
__global__ void zero_kernel(unsigned long long* __restrict__ p, size_t n) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// A fresh fiber in a zeroed bead state: positions from R (device [n][2]), empty support
// windows (the bead kernel then fills one), the excluded-volume constants.
__global__ void fiber_setup_kernel(BeadState* bs, const double* __restrict__ R, int n,
                                   double ev_k, double ev_d) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        bs->R[i][0] = R[2 * i];
        bs->R[i][1] = R[2 * i + 1];
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 2; ++k) {
            bs->win[k][0] = 0x7fffffff;
            bs->win[k][1] = -0x7fffffff;
            bs->win[k][2] = 0x7fffffff;
            bs->win[k][3] = -0x7fffffff;
        }
        bs->ev_k = ev_k;
        bs->ev_d = ev_d;
    }
}

// Bead positions (device [n][2]) and, if asked, the health bits out of a bead state (no
// bead state, n = 0: health 0).
__global__ void beads_out_kernel(const BeadState* bs, int n, double* __restrict__ R,
                                 unsigned* health) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        R[2 * i] = bs->R[i][0];
        R[2 * i + 1] = bs->R[i][1];
    }
    if (threadIdx.x == 0 && health) *health = bs ? bs->health : 0u;
}

// rho, u = (j + f^n/2)/rho and eta^n at node (x, y) from the current state (F/A of every
// bead in bs->C, computed by forces_kernel beforehand).
template <int ST>
__device__ inline void node_fields(const StepArgs& a, int x, int y, double& rho, double& ux,
                                   double& uy, double& eta) {
    using Cd = Codec<ST>;
    using T = typename Cd::T;
    const int nx = a.L.nx, ny = a.L.ny;
    const bool per = a.L.periodic != 0;
    T g[9];
    pull<Cd>((const typename Cd::store_t*)a.src, nx, ny, a.L.stride, a.L.plane, x, y, per,
             (T)a.u6, g);
    double drho = 0.0;
    for (int k = 0; k < 9; ++k) drho += (double)g[k];
    const double jx = ((double)g[1] - (double)g[3]) + ((double)g[5] - (double)g[6]) -
                      ((double)g[7] - (double)g[8]);
    const double jy = ((double)g[2] - (double)g[4]) + ((double)g[5] + (double)g[6]) -
                      ((double)g[7] + (double)g[8]);
    double fx = 0.0, fy = 0.0, sphi = 0.0;
    const Fiber& fib = a.fib;
    for (int b = 0; b < fib.n; ++b) {
        const double dx = min_image((double)x + 0.5 - fib.bs->R[b][0], nx);
        const double dy = y_image((double)y + 0.5 - fib.bs->R[b][1], ny, per);
        const double r2 = dist2(dx, dy);
        if (r2 >= fib.rc2) continue;
        const double ph = phi_f64(sqrt(r2), fib.a, fib.xi);
        sphi += ph;
        fx += ph * fib.bs->C[b][0];
        fy += ph * fib.bs->C[b][1];
    }
    fx += a.gx;
    fy += a.gy;
    if (a.row_phi) sphi += a.row_phi[y];
    if (fib.clamp && sphi > 1.0) sphi = 1.0;
    rho = 1.0 + drho;
    ux = (jx + 0.5 * fx) / rho;
    uy = (jy + 0.5 * fy) / rho;
    eta = fib.nu_f + (fib.nu_s - fib.nu_f) * sphi;
}

template <int ST>
__global__ void fields_kernel(StepArgs a, double* rho_o, double* ux_o, double* uy_o,
                              double* eta_o) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int nx = a.L.nx, ny = a.L.ny;
    if (x >= nx || y >= ny) return;
    double rho, ux, uy, eta;
    node_fields<ST>(a, x, y, rho, ux, uy, eta);
    const long long s = (long long)y * nx + x;
    if (rho_o) rho_o[s] = rho;
    if (ux_o) ux_o[s] = ux;
    if (uy_o) uy_o[s] = uy;
    if (eta_o) eta_o[s] = eta;
}

// ------------------------------------------ single-particle diagnostics (Sec. III.B) --
__device__ inline int box_x(const NodeBox& B, int nx, int bx) { return imod(B.cx0 + bx, nx); }
__device__ inline int box_y(const NodeBox& B, int ny, bool per, int by) {
    return per ? imod(B.cy0 + by, ny) : B.cy0 + by;
}

// rho - 1, v, eta of every node of the box into fields[4][ch][cw].
template <int ST>
__global__ void box_fields_kernel(StepArgs a, NodeBox B, double* __restrict__ fields) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = B.cw * B.ch;
    if (idx >= n) return;
    const int bx = idx % B.cw, by = idx / B.cw;
    const int x = box_x(B, a.L.nx, bx), y = box_y(B, a.L.ny, a.L.periodic != 0, by);
    double rho, ux, uy, eta;
    node_fields<ST>(a, x, y, rho, ux, uy, eta);
    fields[idx] = rho - 1.0;  // density deviation: the pressure force uses p - p0
    fields[n + idx] = ux;
    fields[2 * n + idx] = uy;
    fields[3 * n + idx] = eta;
}

// Eq. (15) and the diffuse-interface drag of Eq. (17) for bead b, summed over the box
// without its one-node border (the border only feeds the gradient stencil; a wrapped
// direction has no border).  One block; fixed-order sums.  out[8]: A, V0x, V0y, eps_v,
// viscous force (x, y), pressure force (x, y).
__device__ inline double phi_at_node(const StepArgs& a, double Rx, double Ry, int x, int y) {
    const double dx = min_image((double)x + 0.5 - Rx, a.L.nx);
    const double dy = y_image((double)y + 0.5 - Ry, a.L.ny, a.L.periodic != 0);
    const double r2 = dist2(dx, dy);
    if (r2 >= a.fib.rc2) return 0.0;
    return phi_f64(sqrt(r2), a.fib.a, a.fib.xi);
}

__global__ void __launch_bounds__(kStatsBlock)
particle_stats_kernel(StepArgs a, int b, NodeBox B, const double* __restrict__ fields,
                      double* __restrict__ out) {
    __shared__ double scratch[kStatsBlock / 64];
    const int tid = threadIdx.x;
    const int nx = a.L.nx, ny = a.L.ny;
    const bool per = a.L.periodic != 0;
    const double Rx = a.fib.bs->R[b][0], Ry = a.fib.bs->R[b][1];
    const int n = B.cw * B.ch;
    const double* drho = fields;
    const double* vx = fields + n;
    const double* vy = fields + 2 * n;
    const double* eta = fields + 3 * n;
    const int bx0 = B.wrap_x ? 0 : 1, bw = B.wrap_x ? B.cw : B.cw - 2;
    const int by0 = B.wrap_y ? 0 : 1, bh = B.wrap_y ? B.ch : B.ch - 2;
    const int total = bw * bh;
    auto nbr = [&](int bx, int by, int ex, int ey) -> int {
        const int xx = B.wrap_x ? imod(bx + ex, B.cw) : bx + ex;
        const int yy = B.wrap_y ? imod(by + ey, B.ch) : by + ey;
        return yy * B.cw + xx;
    };
    // pass 1: A and the phi-weighted velocity
    double A = 0.0, mx = 0.0, my = 0.0;
    for (int t = tid; t < total; t += blockDim.x) {
        const int bx = bx0 + t % bw, by = by0 + t / bw;
        const double ph = phi_at_node(a, Rx, Ry, box_x(B, nx, bx), box_y(B, ny, per, by));
        const int i = by * B.cw + bx;
        A += ph;
        mx += ph * vx[i];
        my += ph * vy[i];
    }
    A = block_sum(A, scratch);
    mx = block_sum(mx, scratch);
    my = block_sum(my, scratch);
    const double V0x = mx / A, V0y = my / A;
    // pass 2: residual flow and forces; gradients by the isotropic D2Q9 stencil
    const int EXs[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int EYs[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    double e = 0.0, fvx = 0.0, fvy = 0.0, fpx = 0.0, fpy = 0.0;
    for (int t = tid; t < total; t += blockDim.x) {
        const int bx = bx0 + t % bw, by = by0 + t / bw;
        const int x = box_x(B, nx, bx), y = box_y(B, ny, per, by);
        const int i = by * B.cw + bx;
        const double ph = phi_at_node(a, Rx, Ry, x, y);
        const double dvx = vx[i] - V0x, dvy = vy[i] - V0y;
        e += ph * (dvx * dvx + dvy * dvy);
        double gpx = 0.0, gpy = 0.0, gxx = 0.0, gyx = 0.0, gxy = 0.0, gyy = 0.0;
        for (int k = 1; k < 9; ++k) {
            const double wk = k < 5 ? 1.0 / 9.0 : 1.0 / 36.0;
            const int ex = EXs[k], ey = EYs[k];
            const double pn = phi_at_node(a, Rx, Ry, imod(x + ex, nx),
                                          per ? imod(y + ey, ny) : y + ey);
            const int j = nbr(bx, by, ex, ey);
            gpx += wk * ex * pn;
            gpy += wk * ey * pn;
            gxx += wk * ex * vx[j];   // d_x v_x
            gyx += wk * ey * vx[j];   // d_y v_x
            gxy += wk * ex * vy[j];   // d_x v_y
            gyy += wk * ey * vy[j];   // d_y v_y
        }
        gpx *= 3.0; gpy *= 3.0; gxx *= 3.0; gyx *= 3.0; gxy *= 3.0; gyy *= 3.0;
        if (gpx == 0.0 && gpy == 0.0) continue;
        const double sxx = eta[i] * 2.0 * gxx;
        const double syy = eta[i] * 2.0 * gyy;
        const double sxy = eta[i] * (gyx + gxy);
        fvx -= sxx * gpx + sxy * gpy;
        fvy -= sxy * gpx + syy * gpy;
        fpx += drho[i] / 3.0 * gpx;  // (p - p0) grad phi: p0 adds nothing to the sum
        fpy += drho[i] / 3.0 * gpy;
    }
    e = block_sum(e, scratch);
    fvx = block_sum(fvx, scratch);
    fvy = block_sum(fvy, scratch);
    fpx = block_sum(fpx, scratch);
    fpy = block_sum(fpy, scratch);
    if (tid == 0) {
        out[0] = A;
        out[1] = V0x;
        out[2] = V0y;
        out[3] = e / A;
        out[4] = fvx;
        out[5] = fvy;
        out[6] = fpx;
        out[7] = fpy;
    }
}

// Plain copy, one 16-byte vector per thread, non-temporal loads and stores in 256-thread
// blocks: the fastest of the copy shapes measured on MI355X (1 GiB: 6.68 TB/s; streaming
// stores alone 6.36, plain 6.26, four vectors per thread 5.63, 512- and 1024-thread blocks
// 2-5 % slower, grid-stride loops 20-35 % slower), so it stands for the bandwidth a kernel
// can reach; its counters also calibrate traffic.
typedef float copy_vec __attribute__((ext_vector_type(4)));
__global__ void copy_kernel(const copy_vec* __restrict__ src, copy_vec* __restrict__ dst,
                            size_t n) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// -------------------------------------------------------------------- launchers ----

template <class T>
struct same_type {
    using type = T;
};

// One launch of kernel k; with events, hipExtLaunchKernel stamps them with the dispatch's
// own start and end, without extra packets in the queue around the kernel.
template <typename... P>
static hipError_t launch_k(void (*k)(P...), dim3 grid, dim3 block, hipStream_t st,
                           hipEvent_t t0, hipEvent_t t1, typename same_type<P>::type... args) {
    void* argv[] = {(void*)&args...};
    if (t0 || t1) return hipExtLaunchKernel((const void*)k, grid, block, argv, 0, st, t0, t1, 0);
    return hipLaunchKernel((const void*)k, grid, block, argv, 0, st);
}

// Dynamic LDS (unused by the kernel) that leaves room for `blocks` resident blocks of it
// per compute unit on the current device, not more: midway between the shares of `blocks`
// and `blocks + 1` of the device's LDS per compute unit, so that the allocation granule
// does not change the count; within the per-block limit; 0 if the device does not report
// them.
static size_t lds_for_blocks(int blocks) {
    static int per_cu[64], per_block[64];  // per device; 0: not asked yet, -1: unknown
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (per_cu[dev] == 0) {
        int c = 0, b = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                  dev) != hipSuccess || c <= 0)
            c = -1;
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess || b <= 0)
            b = -1;
        per_block[dev] = b;
        per_cu[dev] = c;
    }
    if (per_cu[dev] <= 0 || per_block[dev] <= 0) return 0;
    const int mid = (per_cu[dev] / blocks + per_cu[dev] / (blocks + 1)) / 2;
    return (size_t)std::min(mid, per_block[dev]);
}

// Resident fluid-kernel waves per compute unit (the fluid kernel has no LDS of its own, so
// only registers would limit it).  At 8192 x 2048 with the 40-bead fiber, split steps with
// the fluid kernel held to 8 / 7 / 5 / 4 blocks of two waves per compute unit took 390.3 /
// 388.2 / 386.3 / 387.7 us in float64, against 406.4 us unheld; with 6 / 5 / 4 blocks of
// four waves 104.8-106.3 / 108.3-113.3 / 115.5 us in float16 deviations against
// 106.9-107.1, and with 6 / 5 blocks 194.4 / 194.2 us in float32 against 195.7: fewer
// concurrent row streams beside the fiber tiles.  (The whole-step kernel's own 15.5 KB of
// LDS holds it to 10 blocks; fewer gained it at most 0.6 %.)
template <int ST>
constexpr int fluid_waves_per_cu() {
    return ST == FPD_F64 ? 10 : 24;
}

template <int ST, int BC>
static void (*step_kernel_for(int spt))(StepArgs) {
    switch (spt) {
        case 1: return step_kernel<ST, 1, BC>;
        case 2: return step_kernel<ST, 2, BC>;
        case 4: return step_kernel<ST, 4, BC>;
    }
    return nullptr;
}

template <int ST>
static hipError_t launch_step_t(const StepArgs& a, dim3 block, int spt, hipStream_t st,
                                hipEvent_t t0, hipEvent_t t1) {
    void (*k)(StepArgs) = a.L.periodic ? step_kernel_for<ST, kPeriodic>(spt)
                                       : step_kernel_for<ST, kWalls>(spt);
    if (!k) return hipErrorInvalidValue;
    return launch_k(k, dim3(a.n_tiles), block, st, t0, t1, a);
}

hipError_t launch_step(int storage, const StepArgs& a, dim3 block, int spt, hipStream_t st,
                       hipEvent_t t0, hipEvent_t t1) {
    switch (storage) {
        case FPD_F64: return launch_step_t<FPD_F64>(a, block, spt, st, t0, t1);
        case FPD_F32: return launch_step_t<FPD_F32>(a, block, spt, st, t0, t1);
        case FPD_F16DEV: return launch_step_t<FPD_F16DEV>(a, block, spt, st, t0, t1);
        case FPD_BF16DEV: return launch_step_t<FPD_BF16DEV>(a, block, spt, st, t0, t1);
    }
    return hipErrorInvalidValue;
}

template <int ST, int BC>
static void (*part_kernel_for(int spt, int part))(StepArgs) {
    const bool fl = part == kPartFluid;
    switch (spt) {
        case 1: return fl ? fluid_kernel<ST, 1, BC> : fiber_kernel<ST, 1, BC>;
        case 2: return fl ? fluid_kernel<ST, 2, BC> : fiber_kernel<ST, 2, BC>;
        case 4: return fl ? fluid_kernel<ST, 4, BC> : fiber_kernel<ST, 4, BC>;
    }
    return nullptr;
}

template <int ST>
static hipError_t launch_part_t(const StepArgs& a, dim3 block, int spt, int part,
                                hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
    void (*k)(StepArgs) = a.L.periodic ? part_kernel_for<ST, kPeriodic>(spt, part)
                                       : part_kernel_for<ST, kWalls>(spt, part);
    if (!k) return hipErrorInvalidValue;
    const int blocks = part == kPartFluid ? a.n_tiles : a.part_gw * a.part_gh;
    size_t lds = 0;
    if (part == kPartFluid) {
        const int waves = ((int)(block.x * block.y) + 63) / 64;
        lds = lds_for_blocks(std::max(1, fluid_waves_per_cu<ST>() / waves));
    }
    void* argv[] = {(void*)&a};
    if (t0 || t1)
        return hipExtLaunchKernel((const void*)k, dim3(blocks), block, argv, lds, st, t0, t1, 0);
    return hipLaunchKernel((const void*)k, dim3(blocks), block, argv, lds, st);
}

hipError_t launch_step_part(int storage, const StepArgs& a, dim3 block, int spt, int part,
                            hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
    if (part != kPartFluid && part != kPartFiber) return hipErrorInvalidValue;
    if (a.part_gw < 1 || a.part_gh < 1 || a.part_gw > a.tiles_x ||
        a.part_gh > a.n_tiles / a.tiles_x)
        return hipErrorInvalidValue;
    switch (storage) {
        case FPD_F64: return launch_part_t<FPD_F64>(a, block, spt, part, st, t0, t1);
        case FPD_F32: return launch_part_t<FPD_F32>(a, block, spt, part, st, t0, t1);
        case FPD_F16DEV: return launch_part_t<FPD_F16DEV>(a, block, spt, part, st, t0, t1);
        case FPD_BF16DEV: return launch_part_t<FPD_BF16DEV>(a, block, spt, part, st, t0, t1);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_bead(int storage, const StepArgs& a, int do_velocity, int win_out,
                       hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
    if (a.fib.n <= 0) return hipSuccess;
    void (*k)(StepArgs, int, int) = nullptr;
    switch (storage) {
        case FPD_F64: k = bead_kernel<FPD_F64>; break;
        case FPD_F32: k = bead_kernel<FPD_F32>; break;
        case FPD_F16DEV: k = bead_kernel<FPD_F16DEV>; break;
        case FPD_BF16DEV: k = bead_kernel<FPD_BF16DEV>; break;
        default: return hipErrorInvalidValue;
    }
    return launch_k(k, dim3(a.fib.n), dim3(kBeadBlock), st, t0, t1, a, do_velocity, win_out);
}

// Forces F^n, F/A and bond strains of every simulation of a batch, one block per
// simulation (the same arithmetic the lattice tiles use alone).
__global__ void __launch_bounds__(kBeadThreads) batch_forces_kernel(BatchArgs b) {
    __shared__ Bonds B;
    const int s = blockIdx.x;
    if (s >= b.counts[0]) return;
    const StepArgs a = load_args(b.args, 2 * s + b.gpar);
    const Fiber& fib = a.fib;
    if (fib.n <= 0) return;
    BeadState* bs = fib.bs;
    fill_bonds(bs, fib.n, B);
    for (int t = threadIdx.x; t < fib.n; t += blockDim.x) {
        double F[2];
        bead_force(B, fib.chain_len, t, fib.ks_l02, fib.l0, fib.kb, fib.fext, F);
        ev_force(fib, a.L.nx, a.L.ny, a.L.periodic != 0, t, F);
        own_bead(fib, B, t, F, F[0] / bs->A[t], F[1] / bs->A[t]);
    }
    if (a.rec) record_ends(a);  // positions of the step's start, as for one simulation
}

template <int ST, int BC>
static hipError_t launch_batch_lattice(const BatchArgs& b, dim3 grid, dim3 block, int spt,
                                       hipStream_t st) {
    switch (spt) {
        case 1: hipLaunchKernelGGL((batch_step_kernel<ST, 1, BC>), grid, block, 0, st, b); break;
        case 2: hipLaunchKernelGGL((batch_step_kernel<ST, 2, BC>), grid, block, 0, st, b); break;
        case 4: hipLaunchKernelGGL((batch_step_kernel<ST, 4, BC>), grid, block, 0, st, b); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int ST>
static hipError_t launch_batch_t(const BatchArgs& b, dim3 block, int spt, const int counts[3],
                                 bool any_periodic, hipStream_t st) {
    if (counts[0] <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_forces_kernel, dim3(counts[0]), dim3(kBeadThreads), 0, st, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (counts[1] > 0) {
        const dim3 grid(counts[1]);
        e = any_periodic ? launch_batch_lattice<ST, kAnyBoundary>(b, grid, block, spt, st)
                         : launch_batch_lattice<ST, kWalls>(b, grid, block, spt, st);
        if (e != hipSuccess) return e;
    }
    if (counts[2] > 0)
        hipLaunchKernelGGL((batch_bead_kernel<ST>), dim3(counts[2]), dim3(kBatchBeadBlock), 0, st,
                           b);
    return hipGetLastError();
}

hipError_t launch_batch_step(int storage, const BatchArgs& b, dim3 block, int spt,
                             const int counts[3], bool any_periodic, hipStream_t st) {
    switch (storage) {
        case FPD_F64: return launch_batch_t<FPD_F64>(b, block, spt, counts, any_periodic, st);
        case FPD_F32: return launch_batch_t<FPD_F32>(b, block, spt, counts, any_periodic, st);
        case FPD_F16DEV: return launch_batch_t<FPD_F16DEV>(b, block, spt, counts, any_periodic, st);
        case FPD_BF16DEV: return launch_batch_t<FPD_BF16DEV>(b, block, spt, counts, any_periodic, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_record(const StepArgs& a, hipStream_t st) {
    if (!a.rec || a.fib.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(record_kernel, dim3(1), dim3(kBeadThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_ev(const StepArgs& a, hipStream_t st) {
    if (a.fib.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ev_kernel, dim3(1), dim3(kBeadThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_forces(const StepArgs& a, hipStream_t st) {
    if (a.fib.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(forces_kernel, dim3(1), dim3(kBeadThreads), 0, st, a);
    return hipGetLastError();
}

static dim3 site_grid(const Lattice& L) { return dim3((L.nx + 127) / 128, L.ny); }

hipError_t launch_unstream(int storage, const Lattice& L, double u_wall, const double* f64,
                           void* dst, hipStream_t st) {
    const dim3 grid = site_grid(L), block(128);
    switch (storage) {
        case FPD_F64: hipLaunchKernelGGL((unstream_kernel<FPD_F64>), grid, block, 0, st, L, u_wall, f64, (double*)dst); break;
        case FPD_F32: hipLaunchKernelGGL((unstream_kernel<FPD_F32>), grid, block, 0, st, L, u_wall, f64, (float*)dst); break;
        case FPD_F16DEV: hipLaunchKernelGGL((unstream_kernel<FPD_F16DEV>), grid, block, 0, st, L, u_wall, f64, (_Float16*)dst); break;
        case FPD_BF16DEV: hipLaunchKernelGGL((unstream_kernel<FPD_BF16DEV>), grid, block, 0, st, L, u_wall, f64, (uint16_t*)dst); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stream_out(int storage, const Lattice& L, double u_wall, const void* src,
                             double* f64, hipStream_t st) {
    const dim3 grid = site_grid(L), block(128);
    switch (storage) {
        case FPD_F64: hipLaunchKernelGGL((stream_out_kernel<FPD_F64>), grid, block, 0, st, L, u_wall, (const double*)src, f64); break;
        case FPD_F32: hipLaunchKernelGGL((stream_out_kernel<FPD_F32>), grid, block, 0, st, L, u_wall, (const float*)src, f64); break;
        case FPD_F16DEV: hipLaunchKernelGGL((stream_out_kernel<FPD_F16DEV>), grid, block, 0, st, L, u_wall, (const _Float16*)src, f64); break;
        case FPD_BF16DEV: hipLaunchKernelGGL((stream_out_kernel<FPD_BF16DEV>), grid, block, 0, st, L, u_wall, (const uint16_t*)src, f64); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init_eq(const Lattice& L, double u_wall, int init_flow, double* f64,
                          hipStream_t st) {
    hipLaunchKernelGGL(init_eq_kernel, site_grid(L), dim3(128), 0, st, L, u_wall, init_flow, f64);
    return hipGetLastError();
}

hipError_t launch_init_state(int storage, const Lattice& L, double u_wall, int init_flow,
                             void* dst, hipStream_t st) {
    const dim3 grid = site_grid(L), block(128);
    switch (storage) {
        case FPD_F64: hipLaunchKernelGGL((init_state_kernel<FPD_F64>), grid, block, 0, st, L, u_wall, init_flow, (double*)dst); break;
        case FPD_F32: hipLaunchKernelGGL((init_state_kernel<FPD_F32>), grid, block, 0, st, L, u_wall, init_flow, (float*)dst); break;
        case FPD_F16DEV: hipLaunchKernelGGL((init_state_kernel<FPD_F16DEV>), grid, block, 0, st, L, u_wall, init_flow, (_Float16*)dst); break;
        case FPD_BF16DEV: hipLaunchKernelGGL((init_state_kernel<FPD_BF16DEV>), grid, block, 0, st, L, u_wall, init_flow, (uint16_t*)dst); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 8;
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                       (unsigned long long*)p, n);
    return hipGetLastError();
}

hipError_t launch_fiber_setup(BeadState* bs, const double* R, int n, double ev_k, double ev_d,
                              hipStream_t st) {
    hipLaunchKernelGGL(fiber_setup_kernel, dim3(1), dim3(kBeadThreads), 0, st, bs, R, n, ev_k,
                       ev_d);
    return hipGetLastError();
}

hipError_t launch_beads_out(const BeadState* bs, int n, double* R, unsigned* health,
                            hipStream_t st) {
    hipLaunchKernelGGL(beads_out_kernel, dim3(1), dim3(kBeadThreads), 0, st, bs, n, R, health);
    return hipGetLastError();
}

hipError_t launch_fields(int storage, const StepArgs& a, double* rho, double* ux, double* uy,
                         double* eta, hipStream_t st) {
    const dim3 grid = site_grid(a.L), block(128);
    switch (storage) {
        case FPD_F64: hipLaunchKernelGGL((fields_kernel<FPD_F64>), grid, block, 0, st, a, rho, ux, uy, eta); break;
        case FPD_F32: hipLaunchKernelGGL((fields_kernel<FPD_F32>), grid, block, 0, st, a, rho, ux, uy, eta); break;
        case FPD_F16DEV: hipLaunchKernelGGL((fields_kernel<FPD_F16DEV>), grid, block, 0, st, a, rho, ux, uy, eta); break;
        case FPD_BF16DEV: hipLaunchKernelGGL((fields_kernel<FPD_BF16DEV>), grid, block, 0, st, a, rho, ux, uy, eta); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_particle_stats(int storage, const StepArgs& a, int bead, const NodeBox& B,
                                 double* fields, double* out, hipStream_t st) {
    const int n = B.cw * B.ch;
    const dim3 grid((n + 127) / 128), block(128);
    switch (storage) {
        case FPD_F64: hipLaunchKernelGGL((box_fields_kernel<FPD_F64>), grid, block, 0, st, a, B, fields); break;
        case FPD_F32: hipLaunchKernelGGL((box_fields_kernel<FPD_F32>), grid, block, 0, st, a, B, fields); break;
        case FPD_F16DEV: hipLaunchKernelGGL((box_fields_kernel<FPD_F16DEV>), grid, block, 0, st, a, B, fields); break;
        case FPD_BF16DEV: hipLaunchKernelGGL((box_fields_kernel<FPD_BF16DEV>), grid, block, 0, st, a, B, fields); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(particle_stats_kernel, dim3(1), dim3(kStatsBlock), 0, st, a, bead, B,
                       (const double*)fields, out);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 16;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const copy_vec*)src, (copy_vec*)dst, n);
    return hipGetLastError();
}

}  // namespace fpd

namespace fpd {

__global__ void health_gather_kernel(BeadState* const* states, unsigned* out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = states[i] ? states[i]->health : 0u;
}

hipError_t health_gather(BeadState* const* states, unsigned* out, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(health_gather_kernel, dim3((n + 255) / 256), dim3(256), 0, st, states, out, n);
    return hipGetLastError();
}

}  // namespace fpd
