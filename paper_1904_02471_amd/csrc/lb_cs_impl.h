// lb_cs_impl.h -- device code of the collision-streaming D2Q9 step, shared
// by the single-simulation kernel (lb_cs.hip) and the batched kernel
// (lb_batch.hip), so that both evaluate the same rounded expressions.
//
// One launch advances every node by one time step of the CS evolution
// equation (Section 2): f_k(x + e_k, t + 1) = f_k - omega (f_k - f_eq_k),
// omega = dt / tau, with the second-order equilibrium of Section 2.
//
// Storage and mapping
//   * Structure of arrays: plane k holds population k, rows of `pitch`
//     elements, x contiguous; 64 lanes of a wave read 64 consecutive x.
//   * Pull scheme with two buffers: the buffer after step n holds the
//     post-collision values of step n at their source node; a node gathers
//     its 9 incoming values from the neighbours (x - e_k), collides in
//     registers and writes 9 values at its own position.  Each stored value
//     is read exactly once per step: 9 loads + 9 stores per node.
//   * Stored values are shifted, g_k = f_k - w_k rho0, which keeps the
//     small deviations from the reference state in the mantissa (FP32 and
//     FP16 storage); all arithmetic in FP32 (FP64 for double storage).
//   * One workgroup per row, threads striding over x: the periodic x-wrap and
//     the +-1 misaligned x-gathers stay inside one workgroup, so no cache line
//     is shared between workgroups on different XCDs.
//   * Fixed-value x ends: the buffers carry one ghost column on each side
//     (xoff = 1); the step writes the end equilibria into the ghost entries
//     that the next step pulls from.

#pragma once

#include <type_traits>

#include "lb_diag.h"
#include "lb_internal.h"

namespace lbm {

constexpr int kCsThreads = 256;

__device__ __forceinline__ float cs_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double cs_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Per-simulation constants of the collision, in the arithmetic type.
template <typename CT>
struct CsConsts {
    CT w0, w1, w5, a1, a5, b1, b5, omega, rho0;
    __device__ __forceinline__ explicit CsConsts(const Params<CT> &p)
        : w0(p.cs_w0), w1(p.cs_w1), w5(p.cs_w5), a1(p.cs_a1), a5(p.cs_a5), b1(CT(0.5)), b5(CT(0.125)),
          omega(p.omega), rho0(p.rho0)
    {
    }
};

// Moments of one node, for the collision and the diagnostics.
template <typename CT>
struct CsMoments {
    CT drho, rho, jx, jy, ux, uy;
};

// Collision of one node: g[k] are the pulled (pre-collision) shifted values,
// o[k] receives the post-collision values.  Every path of the library (the
// scalar and vector row kernels, the batched kernel) evaluates this same
// sequence of rounded operations.
//
// Second-order equilibrium, shifted, written as
//   w_k drho + a_k (e_k . j) + rho (b_k (e_k . u)^2 - w_k 1.5 u^2),
// a = 3 w, b = 4.5 w: the first-order term takes j itself (rho * (j / rho)
// would carry the quotient's rounding into the momentum every step), and
// with the constants' exact sums the mass and momentum of the equilibrium
// equal the node's up to unbiased rounding.
template <typename CT>
__device__ __forceinline__ CsMoments<CT> cs_collide(const CT (&g)[9], CT (&o)[9], const CsConsts<CT> &c)
{
    CsMoments<CT> m;
    m.drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    m.rho = c.rho0 + m.drho;
    m.jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    m.jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const CT inv = CT(1) / m.rho;
    m.ux = m.jx * inv;
    m.uy = m.jy * inv;
    const CT ux = m.ux, uy = m.uy, jx = m.jx, jy = m.jy, rho = m.rho, drho = m.drho;
    const CT usq = CT(1.5) * cs_fma(ux, ux, uy * uy);
    auto relax = [&](CT gk, CT w, CT a, CT b, CT ej, CT eu) -> CT {
        const CT sec = rho * cs_fma(b * eu, eu, -(w * usq));
        const CT geq = cs_fma(w, drho, cs_fma(a, ej, sec));
        return cs_fma(c.omega, geq - gk, gk);
    };
    {
        const CT geq0 = cs_fma(c.w0, drho, -(rho * (c.w0 * usq)));
        o[0] = cs_fma(c.omega, geq0 - g[0], g[0]);
    }
    o[1] = relax(g[1], c.w1, c.a1, c.b1, jx, ux);
    o[2] = relax(g[2], c.w1, c.a1, c.b1, jy, uy);
    o[3] = relax(g[3], c.w1, c.a1, c.b1, -jx, -ux);
    o[4] = relax(g[4], c.w1, c.a1, c.b1, -jy, -uy);
    o[5] = relax(g[5], c.w5, c.a5, c.b5, jx + jy, ux + uy);
    o[6] = relax(g[6], c.w5, c.a5, c.b5, jy - jx, uy - ux);
    o[7] = relax(g[7], c.w5, c.a5, c.b5, -jx - jy, -ux - uy);
    o[8] = relax(g[8], c.w5, c.a5, c.b5, jx - jy, ux - uy);
    return m;
}

// Diagnostics of one node (input state of the step); qx, qy: the probe
// pattern at the node, ax[x] ay[y] and bx[x] by[y].
template <typename CT>
__device__ __forceinline__ void cs_diag_node_q(DiagAcc &acc, const CsMoments<CT> &m, bool probe, CT qx, CT qy)
{
    acc.v[0] += (double)m.drho;
    acc.v[1] += (double)m.jx;
    acc.v[2] += (double)m.jy;
    acc.v[3] += (double)(CT(0.5) * m.rho * (m.ux * m.ux + m.uy * m.uy));
    if (probe) acc.v[4] += (double)(m.ux * qx + m.uy * qy);
}

template <typename CT>
__device__ __forceinline__ void cs_diag_node(DiagAcc &acc, const CsMoments<CT> &m, const DiagArgs<CT> &d, int x,
                                             CT pay, CT pby)
{
    const bool probe = d.ax != nullptr;
    cs_diag_node_q(acc, m, probe, probe ? d.ax[x] * pay : CT(0), probe ? d.bx[x] * pby : CT(0));
}

// Random bits of the stochastic FP16 rounding: 13 per population, from one
// counter-based word per node and its xorshift successors (populations 2i
// and 2i+1 take the top and the bottom 13 bits of word i), drawn in the
// order 0..8 in every path, so results do not depend on the path.
template <typename T>
struct CsRand {
    uint32_t s = 0;
    bool lo = false;
    __device__ __forceinline__ CsRand(int node, unsigned salt)
    {
        if constexpr (std::is_same<T, __half>::value) s = mix32((uint32_t)node, salt);
    }
    __device__ __forceinline__ uint32_t next()
    {
        if constexpr (std::is_same<T, __half>::value) {
            uint32_t r;
            if (lo) {
                r = s & 0x1fffu;
                s = xorshift32(s);
            } else {
                r = s >> 19;
            }
            lo = !lo;
            return r;
        }
        return 0u;
    }
};

template <typename T>
__device__ __forceinline__ typename Arith<T>::type to_ct(T v);
template <> __device__ __forceinline__ float to_ct<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_ct<__half>(__half v) { return __half2float(v); }
template <> __device__ __forceinline__ double to_ct<double>(double v) { return v; }

// A chunk of W consecutive stored values, loaded and stored as one access:
// 16 bytes (4 FP32 or 2 FP64 values) or, for FP16, 8 bytes (4 values, which
// keeps the per-thread node count and register use at the FP32 level).
template <typename T>
struct Chunk {
    static constexpr int B = sizeof(T) == 2 ? 8 : 16;  // bytes
    static constexpr int W = B / (int)sizeof(T);
    static constexpr int NW = B / 4;                     // 32-bit words
    uint32_t w[NW];
    __device__ __forceinline__ void load(const T *p)
    {
        if constexpr (NW == 4) {
            const uint4 q = *reinterpret_cast<const uint4 *>(p);
            w[0] = q.x;
            w[1] = q.y;
            w[2] = q.z;
            w[3] = q.w;
        } else {
            const uint2 q = *reinterpret_cast<const uint2 *>(p);
            w[0] = q.x;
            w[1] = q.y;
        }
    }
    __device__ __forceinline__ void store(T *p) const
    {
        if constexpr (NW == 4)
            *reinterpret_cast<uint4 *>(p) = make_uint4(w[0], w[1], w[2], w[3]);
        else
            *reinterpret_cast<uint2 *>(p) = make_uint2(w[0], w[1]);
    }
    // the same store, marked non-temporal (the written lines are not kept
    // in the caches for reuse)
    __device__ __forceinline__ void store_nt(T *p) const
    {
        typedef uint32_t V4 __attribute__((ext_vector_type(4)));
        typedef uint32_t V2 __attribute__((ext_vector_type(2)));
        if constexpr (NW == 4)
            __builtin_nontemporal_store(V4{w[0], w[1], w[2], w[3]}, reinterpret_cast<V4 *>(p));
        else
            __builtin_nontemporal_store(V2{w[0], w[1]}, reinterpret_cast<V2 *>(p));
    }
    __device__ __forceinline__ T get(int j) const
    {
        T v;
        __builtin_memcpy(&v, reinterpret_cast<const char *>(w) + j * sizeof(T), sizeof(T));
        return v;
    }
    __device__ __forceinline__ void set(int j, T v) { __builtin_memcpy(reinterpret_cast<char *>(w) + j * sizeof(T), &v, sizeof(T)); }
    // last element of the chunk held by the previous lane of the wave
    __device__ __forceinline__ T prev_lane_last() const
    {
        Chunk t;
        constexpr int w0 = (B - (int)sizeof(T)) / 4;
#pragma unroll
        for (int i = w0; i < NW; ++i) t.w[i] = (uint32_t)__shfl_up((int)w[i], 1, 64);
        return t.get(W - 1);
    }
    // first element of the chunk held by the next lane of the wave
    __device__ __forceinline__ T next_lane_first() const
    {
        Chunk t;
        constexpr int w1 = ((int)sizeof(T) + 3) / 4;
#pragma unroll
        for (int i = 0; i < w1; ++i) t.w[i] = (uint32_t)__shfl_down((int)w[i], 1, 64);
        return t.get(0);
    }
};

// One row y of the step (all threads of a 256-thread workgroup); with DIAG
// the diagnostics of the row's input state go to partial[diag_block].
// REF (FP16 storage only, periodic): the stored values are the departures
// from the reference equilibrium of their node (cs_ref_pop), scaled by
// kRefScale; a pulled value is unscaled and gets the shift of its source
// node added, a stored one the shift of its own node removed and is scaled.
template <typename T, bool FIXED, bool DIAG, bool REF = false>
__device__ __forceinline__ void cs_row(const T *__restrict__ src, T *__restrict__ dst,
                                       const Params<typename Arith<T>::type> &p,
                                       const DiagArgs<typename Arith<T>::type> &d, int y, int diag_block)
{
    static_assert(!REF || (std::is_same<T, __half>::value && !FIXED), "reference shift: FP16, periodic");
    using CT = typename Arith<T>::type;
    const int Nx = p.Nx;
    const int ym = (y == 0) ? p.Ny - 1 : y - 1;
    const int yp = (y == p.Ny - 1) ? 0 : y + 1;
    const long long P = p.plane;
    const T *r0 = src + (long long)y * p.pitch + p.xoff;   // row y
    const T *rs = src + (long long)ym * p.pitch + p.xoff;  // row y-1: sources of N, NE, NW
    const T *rn = src + (long long)yp * p.pitch + p.xoff;  // row y+1: sources of S, SW, SE
    T *orow = dst + (long long)y * p.pitch + p.xoff;

    const CsConsts<CT> c(p);
    DiagAcc acc;
    CT pay = CT(0), pby = CT(0);
    if (DIAG && d.ax) {
        pay = d.ay[y];
        pby = d.by[y];
    }

    for (int x = threadIdx.x; x < Nx; x += kCsThreads) {
        int xm, xp;
        if (FIXED) {
            xm = x - 1;  // ghost column at -1 / Nx lives in memory
            xp = x + 1;
        } else {
            xm = (x == 0) ? Nx - 1 : x - 1;
            xp = (x == Nx - 1) ? 0 : x + 1;
        }
        // gather: population k arrives from x - e_k
        CT g[9], out9[9];
        g[0] = ld(r0 + x);
        g[1] = ld(r0 + 1 * P + xm);  // E  from (x-1, y)
        g[2] = ld(rs + 2 * P + x);   // N  from (x, y-1)
        g[3] = ld(r0 + 3 * P + xp);  // W  from (x+1, y)
        g[4] = ld(rn + 4 * P + x);   // S  from (x, y+1)
        g[5] = ld(rs + 5 * P + xm);  // NE from (x-1, y-1)
        g[6] = ld(rs + 6 * P + xp);  // NW from (x+1, y-1)
        g[7] = ld(rn + 7 * P + xp);  // SW from (x+1, y+1)
        g[8] = ld(rn + 8 * P + xm);  // SE from (x-1, y+1)
        if constexpr (REF) {
            const uint32_t *u0 = p.ref + (long long)y * p.pitch, *us = p.ref + (long long)ym * p.pitch,
                           *un = p.ref + (long long)yp * p.pitch;
            const uint32_t src_u[9] = {u0[x], u0[xm], us[x], u0[xp], un[x], us[xm], us[xp], un[xp], un[xm]};
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                float ux, uy;
                ref_unpack(src_u[k], ux, uy);
                g[k] = __builtin_fmaf(g[k], kRefInvScale, cs_ref_pop(k, ux, uy, p.ref_c));
            }
        }
        const CsMoments<CT> m = cs_collide(g, out9, c);
        if constexpr (REF) {
            float ux, uy;
            ref_unpack(p.ref[(long long)y * p.pitch + x], ux, uy);
#pragma unroll
            for (int k = 0; k < 9; ++k) out9[k] = (out9[k] - cs_ref_pop(k, ux, uy, p.ref_c)) * kRefScale;
        }
        CsRand<T> rnd(y * Nx + x, p.salt);
#pragma unroll
        for (int k = 0; k < 9; ++k) store_state(orow + k * P + x, out9[k], rnd.next());

        if (FIXED) {
            // the next step pulls E, NE, SE into x = 0 from column -1 and W,
            // NW, SW into x = Nx-1 from column Nx: keep the end equilibria there
            if (x == 0) {
                store_from(orow + 1 * P - 1, p.ghost_l[1]);
                store_from(orow + 5 * P - 1, p.ghost_l[5]);
                store_from(orow + 8 * P - 1, p.ghost_l[8]);
            }
            if (x == Nx - 1) {
                store_from(orow + 3 * P + Nx, p.ghost_r[3]);
                store_from(orow + 6 * P + Nx, p.ghost_r[6]);
                store_from(orow + 7 * P + Nx, p.ghost_r[7]);
            }
        }
        if (DIAG) cs_diag_node(acc, m, d, x, pay, pby);
    }
    if (DIAG) block_diag_store(acc, d.partial, diag_block);
}

// Vector form of a periodic row, for Nx a multiple of the chunk width W
// (the row pitch and the plane size are then multiples of W too, and every
// chunk is aligned).  Each thread loads one chunk of W consecutive x from
// each of the 9 source rows, takes the x - 1 neighbours
// of the E, NE, SE planes and the x + W neighbours of the W, NW, SW planes
// from the adjacent lanes of the wave (the wave's first and last lanes load
// them), collides its W nodes with cs_collide and stores whole chunks: the
// same values as cs_row, with full-width memory accesses.  Any workgroup
// size that is a multiple of 64 (up to 1024) works; with one chunk per
// thread all loads of a row are in flight at once.  NT: the output chunks
// are stored non-temporally (for states far larger than the last-level
// cache, where the next step's reads cannot hit the written lines anyway).
template <typename T, bool DIAG, bool REF = false, bool NT = false>
__device__ __forceinline__ void cs_row_vec(const T *__restrict__ src, T *__restrict__ dst,
                                           const Params<typename Arith<T>::type> &p,
                                           const DiagArgs<typename Arith<T>::type> &d, int y, int diag_block)
{
    using CT = typename Arith<T>::type;
    constexpr int W = Chunk<T>::W;
    static_assert(!REF || std::is_same<T, __half>::value, "reference shift: FP16 storage");
    static_assert(!std::is_same<T, __half>::value || W % 2 == 0, "FP16 chunks convert node pairs");
    const int Nx = p.Nx, nch = Nx / W;
    const int ym = (y == 0) ? p.Ny - 1 : y - 1;
    const int yp = (y == p.Ny - 1) ? 0 : y + 1;
    const long long P = p.plane;
    const T *r0 = src + (long long)y * p.pitch;
    const T *rs = src + (long long)ym * p.pitch;
    const T *rn = src + (long long)yp * p.pitch;
    T *orow = dst + (long long)y * p.pitch;
    const int lane = threadIdx.x & 63;

    const CsConsts<CT> c(p);
    DiagAcc acc;
    CT pay = CT(0), pby = CT(0);
    if (DIAG && d.ax) {
        pay = d.ay[y];
        pby = d.by[y];
    }

    for (int v = threadIdx.x; v < nch; v += blockDim.x) {
        const int x = v * W;
        Chunk<T> in[9];
        in[0].load(r0 + x);
        in[1].load(r0 + 1 * P + x);
        in[2].load(rs + 2 * P + x);
        in[3].load(r0 + 3 * P + x);
        in[4].load(rn + 4 * P + x);
        in[5].load(rs + 5 * P + x);
        in[6].load(rs + 6 * P + x);
        in[7].load(rn + 7 * P + x);
        in[8].load(rn + 8 * P + x);
        // the probe pattern of the chunk's nodes, loaded with the chunk
        CT qx[W], qy[W];
#pragma unroll
        for (int j = 0; j < W; ++j) qx[j] = qy[j] = CT(0);
        if (DIAG && d.ax) {
#pragma unroll
            for (int j = 0; j < W; ++j) {
                qx[j] = d.ax[x + j] * pay;
                qy[j] = d.bx[x + j] * pby;
            }
        }
        // neighbours across the chunk edges (lanes of one wave hold
        // consecutive chunks of the row)
        T l1 = in[1].prev_lane_last(), l5 = in[5].prev_lane_last(), l8 = in[8].prev_lane_last();
        T r3 = in[3].next_lane_first(), r6 = in[6].next_lane_first(), r7 = in[7].next_lane_first();
        if (lane == 0) {
            const int xm = (x == 0) ? Nx - 1 : x - 1;
            l1 = r0[1 * P + xm];
            l5 = rs[5 * P + xm];
            l8 = rn[8 * P + xm];
        }
        if (lane == 63 || v == nch - 1) {
            const int xp = (x + W == Nx) ? 0 : x + W;
            r3 = r0[3 * P + xp];
            r6 = rs[6 * P + xp];
            r7 = rn[7 * P + xp];
        }
        // REF: reference velocities of x-1 .. x+W in rows y (c), y-1 (s), y+1 (n)
        uint32_t rc[W + 2], rs_[W + 2], rn_[W + 2];
        if constexpr (REF) {
            const uint32_t *u0 = p.ref + (long long)y * p.pitch, *us = p.ref + (long long)ym * p.pitch,
                           *un = p.ref + (long long)yp * p.pitch;
            const int xm = (x == 0) ? Nx - 1 : x - 1, xp = (x + W == Nx) ? 0 : x + W;
            auto row = [&](const uint32_t *u, uint32_t *o) {
                const uint4 q = *reinterpret_cast<const uint4 *>(u + x);  // W = 4 nodes, 16 bytes
                o[1] = q.x;
                o[2] = q.y;
                o[3] = q.z;
                o[4] = q.w;
                uint32_t l = (uint32_t)__shfl_up((int)q.w, 1, 64), r = (uint32_t)__shfl_down((int)q.x, 1, 64);
                if (lane == 0) l = u[xm];
                if (lane == 63 || v == nch - 1) r = u[xp];
                o[0] = l;
                o[W + 1] = r;
            };
            row(u0, rc);
            row(us, rs_);
            row(un, rn_);
        }
        Chunk<T> out[9];
        half2_bits held[9];  // FP16: the even node's values awaiting their pair
#pragma unroll
        for (int j = 0; j < W; ++j) {
            CT g[9], o[9];
            g[0] = to_ct<T>(in[0].get(j));
            g[1] = to_ct<T>(j > 0 ? in[1].get(j - 1) : l1);
            g[2] = to_ct<T>(in[2].get(j));
            g[3] = to_ct<T>(j < W - 1 ? in[3].get(j + 1) : r3);
            g[4] = to_ct<T>(in[4].get(j));
            g[5] = to_ct<T>(j > 0 ? in[5].get(j - 1) : l5);
            g[6] = to_ct<T>(j < W - 1 ? in[6].get(j + 1) : r6);
            g[7] = to_ct<T>(j < W - 1 ? in[7].get(j + 1) : r7);
            g[8] = to_ct<T>(j > 0 ? in[8].get(j - 1) : l8);
            if constexpr (REF) {
                // sources x+j-e_k: offsets j (x), j+1 (x+1), j+2 (x+2) in the windows
                const uint32_t su[9] = {rc[j + 1], rc[j], rs_[j + 1], rc[j + 2], rn_[j + 1],
                                        rs_[j],    rs_[j + 2], rn_[j + 2], rn_[j]};
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    float ux, uy;
                    ref_unpack(su[k], ux, uy);
                    g[k] = __builtin_fmaf(g[k], kRefInvScale, cs_ref_pop(k, ux, uy, p.ref_c));
                }
            }
            const CsMoments<CT> m = cs_collide(g, o, c);
            if constexpr (REF) {
                float ux, uy;
                ref_unpack(rc[j + 1], ux, uy);
#pragma unroll
                for (int k = 0; k < 9; ++k) o[k] = (o[k] - cs_ref_pop(k, ux, uy, p.ref_c)) * kRefScale;
            }
            CsRand<T> rnd(y * Nx + x + j, p.salt);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                if constexpr (std::is_same<T, __half>::value) {
                    // FP16: nodes in pairs, into the two halves of one word
                    if (j & 1)
                        out[k].w[j >> 1] = __builtin_bit_cast(uint32_t, sr16_into(held[k], o[k], rnd.next(), true));
                    else
                        held[k] = sr16_into(half2_bits{}, o[k], rnd.next(), false);
                } else {
                    out[k].set(j, o[k]);
                }
            }
            if (DIAG) cs_diag_node_q(acc, m, d.ax != nullptr, qx[j], qy[j]);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            if constexpr (NT)
                out[k].store_nt(orow + k * P + x);
            else
                out[k].store(orow + k * P + x);
        }
    }
    if (DIAG) block_diag_store(acc, d.partial, diag_block);
}

// Workgroup size of the single-simulation vector launch: one chunk per
// thread, at least 256 threads (the batched launch uses 256, so for rows of
// up to 256 chunks the two sum their diagnostics in the same order).
template <typename T>
__host__ __device__ __forceinline__ int cs_vec_threads(int Nx)
{
    const int nch = Nx / Chunk<T>::W;
    const int t = (nch + 63) / 64 * 64;
    return t < kCsThreads ? kCsThreads : (t > 1024 ? 1024 : t);
}

// Whether the vector row form applies to a simulation.
template <typename T, typename CT>
__host__ __device__ __forceinline__ bool cs_vec_ok(const Params<CT> &p)
{
    return !p.fixed_x && p.xoff == 0 && p.Nx % Chunk<T>::W == 0 && p.pitch % Chunk<T>::W == 0;
}

}  // namespace lbm
