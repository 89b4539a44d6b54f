// The fused stream-collide sweep (Sec. 2.1 and 2.3): one thread per cell
// loads the 19 deviations of its cell, collides them with LBGK and pushes
// the post-collision values to the neighbours; populations that would enter
// a wall are bounced back (Eq. lbm:bounce_back), those that would enter a
// body are bounced back with the moving-wall term of Sec. 2.3, and the
// momentum exchange of those links (Eq. hydroF) is summed in the sweep
// itself, per wave of 64 consecutive cells and per body, into one record.
#pragma once
#include "geometry.h"

namespace lbm {

// Owners of the 18 neighbours of a near-body cell, loaded before any is
// used so that their latencies overlap (a neighbour across a wall reads the
// cell itself, which is fluid).
__device__ __forceinline__ void neighbour_owners(const BoxDesc &B, int cell, int i, int j, int k, Owners &owner) {
    int idx[19];
#pragma unroll
    for (int a = 1; a < 19; ++a) {
        int ti, tj, tk;
        idx[a] = neighbour_rt(a, i, j, k, B.nx, B.ny, B.nz, B.per, ti, tj, tk) ? ti + B.nx * (tj + B.ny * tk) : cell;
    }
#pragma unroll
    for (int a = 1; a < 19; ++a) owner.set(a, B.flags[idx[a]] & kOwnerMask);
}

// Moving bounce-back of the link (cell, A) into body `owner`: returns the
// reflected value and writes the link's momentum-exchange contribution to
// its scratch record (summed by the wave in body_links).
template <typename S, int A>
__device__ __forceinline__ typename Storage<S>::C bounce_moving(const BoxDesc &B, int cell, int owner,
                                                                int ti, int tj, int tk,
                                                                typename Storage<S>::C v,
                                                                typename Storage<S>::C rho, int slot) {
    using C = typename Storage<S>::C;
    constexpr int O = opp(A);
    const DevBody &bd = B.bodies[owner - 1];
    double r[3], u[3];
    int d[3];
    lever_arm(bd, ti, tj, tk, B.nx, B.ny, B.nz, B.per, r, d);
    wall_velocity(bd, r, u);
    const double eu = (double)ex(O) * u[0] + (double)ey(O) * u[1] + (double)ez(O) * u[2];
    const double mw = 6.0 * wgt(A) * (double)rho * eu;
    const double val = (double)v + mw;
    if (slot >= 0 && slot < B.link_cap) {
        const double sc = 2.0 * (double)v + mw;
        const double t0 = ex(A) * sc, t1 = ey(A) * sc, t2 = ez(A) * sc;
        LinkRec rec;
        rec.f[0] = t0;
        rec.f[1] = t1;
        rec.f[2] = t2;
        rec.t[0] = r[1] * t2 - r[2] * t1;
        rec.t[1] = r[2] * t0 - r[0] * t2;
        rec.t[2] = r[0] * t1 - r[1] * t0;
        constexpr int cw = two_w36(A);
        constexpr int e0 = ex(A) * cw, e1 = ey(A) * cw, e2 = ez(A) * cw;
        const int d0 = 2 * d[0] + 1, d1 = 2 * d[1] + 1, d2 = 2 * d[2] + 1;
        rec.s[0] = d1 * e2 - d2 * e1;
        rec.s[1] = d2 * e0 - d0 * e2;
        rec.s[2] = d0 * e1 - d1 * e0;
        rec.a = A;
        B.link_rec[slot] = rec;
    }
    return (C)val;
}

// owner.get(A): the body behind the link (cell, A), 0 for fluid; only
// near-body cells look it up.  slot: the cell's next link.
template <typename S, int A>
__device__ __forceinline__ void push_one(const BoxDesc &B, S *dst, long long stride, int cell, int i,
                                         int j, int k, const Owners &owner, typename Storage<S>::C v,
                                         typename Storage<S>::C rho, int &slot) {
    using St = Storage<S>;
    int ti, tj, tk;
    if (!neighbour<A>(i, j, k, B.nx, B.ny, B.nz, B.per, ti, tj, tk)) {
        St::store(dst, (size_t)opp(A) * stride + cell, v, B.scale);
        return;
    }
    if (const int o = owner.get(A)) {
        St::store(dst, (size_t)opp(A) * stride + cell, bounce_moving<S, A>(B, cell, o, ti, tj, tk, v, rho, slot),
                  B.scale);
        ++slot;
        return;
    }
    St::store(dst, (size_t)A * stride + (ti + B.nx * (tj + B.ny * tk)), v, B.scale);
}

template <typename S, int A>
struct PushAll {
    static __device__ __forceinline__ void run(const BoxDesc &B, S *dst, long long stride, int cell, int i,
                                               int j, int k, const Owners &owner,
                                               const typename Storage<S>::C *f, typename Storage<S>::C rho,
                                               int &slot) {
        push_one<S, A>(B, dst, stride, cell, i, j, k, owner, f[A], rho, slot);
        PushAll<S, A + 1>::run(B, dst, stride, cell, i, j, k, owner, f, rho, slot);
    }
};
template <typename S>
struct PushAll<S, 19> {
    static __device__ __forceinline__ void run(const BoxDesc &, S *, long long, int, int, int, int,
                                               const Owners &, const typename Storage<S>::C *,
                                               typename Storage<S>::C, int &) {}
};

// Momentum exchange of the wave's near-body cells (Eq. hydroF), body by
// body.  Called by every lane of a wave that holds at least one near-body
// cell, after the pushes, with the cell's links [lfirst, lend) (an empty
// range elsewhere).  A wave covers 64 consecutive cells of its box, and the
// links are numbered in cell order, so the wave's links are one contiguous
// range [l0, l1): lane q takes links l0 + q, l0 + q + 64, ... (coalesced
// loads of the scratch records, a pass or two), the wave adds the lanes in
// a fixed tree (wave_sum), and lane 0 writes the sums to the record that
// the mapping reserved for (this wave, body b): record grp_pos[l0 + n] for
// the wave's n-th body in ascending order.  The sums come out the same bit
// for bit however the sweep is launched.  The populations are no longer
// live here, which keeps the sweep within its register budget.
__device__ __forceinline__ void body_links(const BoxDesc &B, int lfirst, int lend) {
    int l0 = lfirst, l1 = lend;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        l0 = min(l0, __shfl_xor(l0, o, 64));
        l1 = max(l1, __shfl_xor(l1, o, 64));
    }
    l0 = __builtin_amdgcn_readfirstlane(l0);
    l1 = min(__builtin_amdgcn_readfirstlane(l1), B.link_cap);
    if (l0 >= l1) return;
    const int lane = (int)threadIdx.x & 63;
    unsigned wm = 0;
    for (int l = l0 + lane; l < l1; l += 64) wm |= 1u << B.link_body[l];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wm |= __shfl_xor(wm, o, 64);
    wm = __builtin_amdgcn_readfirstlane(wm);
    for (int q = 0; wm; ++q) {
        const int b = __builtin_ctz(wm);
        wm &= wm - 1;
        double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int ia[6] = {0, 0, 0, 0, 0, 0};
        for (int l = l0 + lane; l < l1; l += 64) {
            if (B.link_body[l] != b) continue;
            const LinkRec rec = B.link_rec[l];
            const int cw = two_w36(rec.a);
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                acc[v] += rec.f[v];
                acc[3 + v] += rec.t[v];
                ia[v] += rec.s[v];
            }
            ia[3] += ex(rec.a) * cw;
            ia[4] += ey(rec.a) * cw;
            ia[5] += ez(rec.a) * cw;
        }
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            acc[v] = wave_sum(acc[v]);
            ia[v] = wave_sum_int(ia[v]);
        }
        if (lane == 0) {
            const int l = l0 + q;
            if (l < B.link_cap) {
                const int pos = B.grp_pos[l];
                if (pos >= 0 && pos < B.link_cap) {
                    ForceRec rec;
#pragma unroll
                    for (int v = 0; v < 3; ++v) {
                        rec.f[v] = acc[v];
                        rec.t[v] = acc[3 + v];
                        rec.s[v] = ia[v];
                        rec.g[v] = ia[3 + v];
                    }
                    rec.body = b;
                    rec.pad = 0;
                    B.frec[pos] = rec;
                }
            }
        }
    }
}

// LBGK collision in deviation form: dF~ = dF + omega (dF_eq - dF),
// dF_eq = w [drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)].  Opposite directions
// share the even part drho + rho (4.5 (e.u)^2 - 1.5 u.u) and differ in the
// sign of the odd part 3 rho e.u, which is taken as 3 e.j (j = rho u, the
// momentum summed from the populations): the same number in exact
// arithmetic, but rho (j / rho) rounds away from j, and in float that
// rounding does not average out.  It leaks momentum into the fluid in a way
// correlated with the flow (on the 256x128x128 swimmer it drives a mean
// drift of 1e-11 per step, twice the swimming speed, in 20 periods); with
// e.j the float run's per-period swimming velocity stays within 1.3e-6 of
// the double run's.  Every rounding is spelled out (automatic contraction
// off, fused multiply-adds written as such), so that the collision gives
// the same bits in every kernel and code path that inlines it.
template <typename C>
__device__ __forceinline__ C fmac(C a, C b, C c) {
    if constexpr (sizeof(C) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

// e_A . u with the zero components left out
template <typename C, int A>
__device__ __forceinline__ C edot(C ux, C uy, C uz) {
#pragma clang fp contract(off)
    C s = C(0);
    bool first = true;
    auto add = [&](int e, C u) {
        if (e == 0) return;
        const C t = e > 0 ? u : -u;
        s = first ? t : s + t;
        first = false;
    };
    add(ex(A), ux);
    add(ey(A), uy);
    add(ez(A), uz);
    return s;
}

template <typename C, int A>
__device__ __forceinline__ void relax_pair(C *f, C drho, C rho, C ux, C uy, C uz, C jx, C jy, C jz, C usq15,
                                           C omega) {
#pragma clang fp contract(off)
    constexpr int O = opp(A);
    const C eu = edot<C, A>(ux, uy, uz);
    const C even = fmac(rho, fmac(C(4.5) * eu, eu, -usq15), drho);
    const C odd = C(3) * edot<C, A>(jx, jy, jz);
    const C fa = C(wgt(A)) * (even + odd);
    const C fo = C(wgt(A)) * (even - odd);
    f[A] = fmac(omega, fa - f[A], f[A]);
    f[O] = fmac(omega, fo - f[O], f[O]);
}

template <typename C>
__device__ __forceinline__ C collide(C *f, C omega) {
#pragma clang fp contract(off)
    C drho = f[0];
#pragma unroll
    for (int a = 1; a < 19; ++a) drho += f[a];
    C jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
    C jy = (f[3] - f[4]) + (f[7] - f[8]) + (f[10] - f[9]) + (f[15] - f[16]) + (f[17] - f[18]);
    C jz = (f[5] - f[6]) + (f[11] - f[12]) + (f[14] - f[13]) + (f[15] - f[16]) + (f[18] - f[17]);
    const C rho = C(1) + drho;
    const C inv = C(1) / rho;
    const C ux = jx * inv, uy = jy * inv, uz = jz * inv;
    const C usq15 = C(1.5) * fmac(ux, ux, fmac(uy, uy, uz * uz));
    f[0] = fmac(omega, C(wgt(0)) * (drho - rho * usq15) - f[0], f[0]);
    relax_pair<C, 1>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 3>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 5>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 7>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 9>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 11>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 13>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 15>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 17>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    return rho;
}

// The collision with the test-only uniform body force g (Guo's scheme; not
// part of the method): the equilibrium takes u = (j + g/2) / rho, and each
// direction gains (1 - 1/(2 tau)) w [3 (e - u) + 9 (e.u) e].g.  Used only
// by boxes that set a force (Poiseuille flow, the drag of a sphere array).
template <typename C>
__device__ __forceinline__ C collide_forced(C *f, C omega, const double *gd) {
#pragma clang fp contract(off)
    const C g[3] = {(C)gd[0], (C)gd[1], (C)gd[2]};
    C drho = f[0];
#pragma unroll
    for (int a = 1; a < 19; ++a) drho += f[a];
    C jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
    C jy = (f[3] - f[4]) + (f[7] - f[8]) + (f[10] - f[9]) + (f[15] - f[16]) + (f[17] - f[18]);
    C jz = (f[5] - f[6]) + (f[11] - f[12]) + (f[14] - f[13]) + (f[15] - f[16]) + (f[18] - f[17]);
    jx = jx + C(0.5) * g[0];
    jy = jy + C(0.5) * g[1];
    jz = jz + C(0.5) * g[2];
    const C rho = C(1) + drho;
    const C inv = C(1) / rho;
    const C ux = jx * inv, uy = jy * inv, uz = jz * inv;
    const C usq15 = C(1.5) * fmac(ux, ux, fmac(uy, uy, uz * uz));
    const C pref = C(1) - C(0.5) * omega;
    // sources first, from the pre-collision u
    C src[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        const C eu = (C)ex(a) * ux + (C)ey(a) * uy + (C)ez(a) * uz;
        const C s = (C(3) * ((C)ex(a) - ux) + C(9) * eu * (C)ex(a)) * g[0] +
                    (C(3) * ((C)ey(a) - uy) + C(9) * eu * (C)ey(a)) * g[1] +
                    (C(3) * ((C)ez(a) - uz) + C(9) * eu * (C)ez(a)) * g[2];
        src[a] = pref * C(wgt(a)) * s;
    }
    f[0] = fmac(omega, C(wgt(0)) * (drho - rho * usq15) - f[0], f[0]);
    relax_pair<C, 1>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 3>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 5>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 7>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 9>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 11>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 13>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 15>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
    relax_pair<C, 17>(f, drho, rho, ux, uy, uz, jx, jy, jz, usq15, omega);
#pragma unroll
    for (int a = 0; a < 19; ++a) f[a] = f[a] + src[a];
    return rho;
}

// Time-averaged flow field (the averaged flow fields of Sec. 6): add the
// fluid velocity u = j / rho of this cell's pre-collision state to the box's
// sums, in double, with the moments summed over the directions in ascending
// order.
template <typename C>
__device__ __forceinline__ void flow_sample(const BoxDesc &B, int cell, const C *f) {
#pragma clang fp contract(off)
    double drho = (double)f[0];
    double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 1; a < 19; ++a) {
        const double v = (double)f[a];
        drho += v;
        if (ex(a) == 1) j[0] += v;
        if (ex(a) == -1) j[0] -= v;
        if (ey(a) == 1) j[1] += v;
        if (ey(a) == -1) j[1] -= v;
        if (ez(a) == 1) j[2] += v;
        if (ez(a) == -1) j[2] -= v;
    }
    const double rho = 1.0 + drho;
    const size_t n = (size_t)B.N;
#pragma unroll
    for (int q = 0; q < 3; ++q) B.flow_sum[q * n + cell] += j[q] / rho;
    B.flow_count[cell] += 1;
}

// Interior push: no wall and no body among the neighbours.  off_p / off_m
// are the linear offsets of the +1 / -1 neighbour along each axis (with the
// periodic wrap already applied).
template <typename S, int A>
struct PushFast {
    template <typename P>
    static __device__ __forceinline__ void run(P dst, long long stride, int cell, const int *off_p,
                                               const int *off_m, const typename Storage<S>::C *f, float scale) {
        const int o = (ex(A) > 0 ? off_p[0] : ex(A) < 0 ? off_m[0] : 0) +
                      (ey(A) > 0 ? off_p[1] : ey(A) < 0 ? off_m[1] : 0) +
                      (ez(A) > 0 ? off_p[2] : ez(A) < 0 ? off_m[2] : 0);
        Storage<S>::store(dst + (size_t)A * stride, (size_t)(unsigned)(cell + o), f[A], scale);
        PushFast<S, A + 1>::run(dst, stride, cell, off_p, off_m, f, scale);
    }
};
template <typename S>
struct PushFast<S, 19> {
    template <typename P>
    static __device__ __forceinline__ void run(P, long long, int, const int *, const int *,
                                               const typename Storage<S>::C *, float) {}
};

// Push of a cell on a wall away from bodies: as PushFast, except that a
// population that would leave through a wall is bounced back into slot
// opp(A) of the cell itself (Eq. lbm:bounce_back).  lo_w / hi_w: bit a set
// if the cell is at the low / high end of axis a and that axis has walls.
template <typename S, int A>
struct PushWall {
    template <typename P>
    static __device__ __forceinline__ void run(P dst, long long stride, int cell, const int *off_p,
                                               const int *off_m, unsigned lo_w, unsigned hi_w,
                                               const typename Storage<S>::C *f, float scale) {
        const bool out = (ex(A) > 0 ? (hi_w & 1u) : ex(A) < 0 ? (lo_w & 1u) : 0u) ||
                         (ey(A) > 0 ? (hi_w & 2u) : ey(A) < 0 ? (lo_w & 2u) : 0u) ||
                         (ez(A) > 0 ? (hi_w & 4u) : ez(A) < 0 ? (lo_w & 4u) : 0u);
        const int o = (ex(A) > 0 ? off_p[0] : ex(A) < 0 ? off_m[0] : 0) +
                      (ey(A) > 0 ? off_p[1] : ey(A) < 0 ? off_m[1] : 0) +
                      (ez(A) > 0 ? off_p[2] : ez(A) < 0 ? off_m[2] : 0);
        const size_t at = out ? (size_t)opp(A) * stride + (size_t)cell
                              : (size_t)A * stride + (size_t)(unsigned)(cell + o);
        Storage<S>::store(dst, at, f[A], scale);
        PushWall<S, A + 1>::run(dst, stride, cell, off_p, off_m, lo_w, hi_w, f, scale);
    }
};
template <typename S>
struct PushWall<S, 19> {
    template <typename P>
    static __device__ __forceinline__ void run(P, long long, int, const int *, const int *, unsigned, unsigned,
                                               const typename Storage<S>::C *, float) {}
};

// Interior pushes with the x-shifted directions realigned across lanes.
// The cells of a wave are consecutive, so the push of lane l along +x lands
// on lane l+1's cell: if lane l+1 holds the next cell of the same row, lane
// l+1 stores the value it received from lane l at its own, aligned slot
// (from_left); lane l stores it itself only where no neighbour takes it
// (own_px), that is at the end of a row or a wave or next to a wall or
// near-body cell.  -x works the same way from the right.  Every destination is
// still written exactly once, with the same value.
struct XLanes {
    bool from_left, from_right, own_px, own_mx, fast;
};

template <typename S, int A>
struct PushLanes {
    template <typename P>
    static __device__ __forceinline__ void run(P dst, long long stride, int cell, const int *off_p,
                                               const int *off_m, const typename Storage<S>::C *f, float scale,
                                               const XLanes &x) {
        using St = Storage<S>;
        const int oyz = (ey(A) > 0 ? off_p[1] : ey(A) < 0 ? off_m[1] : 0) +
                        (ez(A) > 0 ? off_p[2] : ez(A) < 0 ? off_m[2] : 0);
        P base = dst + (size_t)A * stride;
        if constexpr (ex(A) == 0) {
            if (x.fast) St::store(base, (size_t)(unsigned)(cell + oyz), f[A], scale);
        } else if constexpr (ex(A) > 0) {
            const auto v = __shfl_up(f[A], 1);
            if (x.from_left) St::store(base, (size_t)(unsigned)(cell + oyz), v, scale);
            if (x.own_px) St::store(base, (size_t)(unsigned)(cell + off_p[0] + oyz), f[A], scale);
        } else {
            const auto v = __shfl_down(f[A], 1);
            if (x.from_right) St::store(base, (size_t)(unsigned)(cell + oyz), v, scale);
            if (x.own_mx) St::store(base, (size_t)(unsigned)(cell + off_m[0] + oyz), f[A], scale);
        }
        PushLanes<S, A + 1>::run(dst, stride, cell, off_p, off_m, f, scale, x);
    }
};
template <typename S>
struct PushLanes<S, 19> {
    template <typename P>
    static __device__ __forceinline__ void run(P, long long, int, const int *, const int *,
                                               const typename Storage<S>::C *, float, const XLanes &) {}
};

// Map a workgroup to its tile.  With xcd_order, the hardware's round-robin
// placement of consecutive workgroups on the 8 XCDs is undone so that each
// XCD sweeps one contiguous slab of tiles (neighbouring rows share its L2).
__device__ __forceinline__ int tile_index(int xcd_order) {
    const int w = blockIdx.x;
    if (!xcd_order) return w;
    const int per = gridDim.x >> 3;
    return (w & 7) * per + (w >> 3);
}

// At least 7 waves per SIMD (72 registers) for the 4- and 2-byte formats,
// 5 for double, one fewer while sampling the flow average: without the hint
// the register allocator settles one register above 72 for the float
// sweep, which costs a wave per SIMD.
template <typename S, int BLOCK, bool NT, bool FLOW, bool FORCE = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 5 : (FLOW ? 6 : 7), 8)))
void sweep_kernel(BoxDesc *boxes, const WorkItem *work, int nwork,
                                                      int xcd_order) {
    using St = Storage<S>;
    using C = typename St::C;
    const int t = tile_index(xcd_order);
    if (t >= nwork) return;
    const WorkItem wk = work[t];
    const BoxDesc &B = boxes[wk.box];
    const int cell = wk.first + (int)threadIdx.x;
    // every lane stays until the interior stores are done: the x-shifted
    // pushes are exchanged between neighbouring lanes
    const bool valid = cell < B.N;
    const uint8_t fl = valid ? B.flags[cell] : kOwnerMask;
    const bool fluid = !(fl & kOwnerMask);  // a body cell has no fluid
    const long long stride = B.stride;
    // the population buffers live in global memory: say so, so that the
    // loads and stores of the interior path are global, not flat
    const global_t<S> *src = (const global_t<S> *)(B.cur ? B.pop1 : B.pop0);
    global_t<S> *dst = (global_t<S> *)(B.cur ? B.pop0 : B.pop1);
    C f[19];
    if (fluid) {
#pragma unroll
        for (int a = 0; a < 19; ++a) f[a] = St::template load<NT>(src, (size_t)a * stride + cell, B.inv_scale);
    } else {
#pragma unroll
        for (int a = 0; a < 19; ++a) f[a] = C(0);
    }
    // coordinates from the tile origin (no integer division)
    int i = wk.i0 + (int)threadIdx.x, j = wk.j0, k = wk.k0;
    while (i >= B.nx) {
        i -= B.nx;
        if (++j == B.ny) {
            j = 0;
            ++k;
        }
    }
    if constexpr (FLOW) {
        if (valid && fluid && B.flow_every > 0 && B.step % B.flow_every == 0) flow_sample<C>(B, cell, f);
    }
    const C omega = sizeof(C) == 8 ? (C)B.omega : (C)B.omegaf;
    C rho;
    if constexpr (FORCE) rho = collide_forced<C>(f, omega, B.force);
    else rho = collide<C>(f, omega);
    const int nx = B.nx, ny = B.ny, nz = B.nz, per = B.per;
    const int sy = nx, sz = nx * ny;
    const bool at_lo[3] = {i == 0, j == 0, k == 0};
    const bool at_hi[3] = {i == nx - 1, j == ny - 1, k == nz - 1};
    const int span[3] = {1, sy, sz};
    const int len[3] = {nx, ny, nz};
    int off_p[3], off_m[3];
    bool wall = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool p = (per >> a) & 1;
        off_p[a] = at_hi[a] ? (1 - len[a]) * span[a] : span[a];
        off_m[a] = at_lo[a] ? (len[a] - 1) * span[a] : -span[a];
        wall |= !p && (at_lo[a] || at_hi[a]);
    }
    const bool fast = valid && fluid && !wall && !(fl & kNearBit);
    if constexpr (sizeof(S) >= 4) {
        // 4- and 8-byte storage: realign the x-shifted pushes across lanes
        // (2% faster on the 256x128x128 box; the 2-byte formats gain nothing)
        const int lane = (int)threadIdx.x & 63;
        XLanes x;
        x.fast = fast;
        const bool left_fast = __shfl_up((int)fast, 1) != 0, right_fast = __shfl_down((int)fast, 1) != 0;
        const bool left_row = lane >= 1 && i != 0, right_row = lane <= 62 && i != nx - 1;
        x.from_left = valid && left_row && left_fast;
        x.from_right = valid && right_row && right_fast;
        x.own_px = fast && !(right_row && right_fast);
        x.own_mx = fast && !(left_row && left_fast);
        if (fast) St::store(dst, (size_t)cell, f[0], B.scale);
        PushLanes<S, 1>::run(dst, stride, cell, off_p, off_m, f, B.scale, x);
    } else {
        // 2-byte storage: each lane pushes its own values
        if (fast) {
            St::store(dst, (size_t)cell, f[0], B.scale);
            PushFast<S, 1>::run(dst, stride, cell, off_p, off_m, f, B.scale);
        }
    }
    // the other fluid cells: on a wall (PushWall) or next to a body (the
    // general path, PushAll).  Every lane stays for the wave's
    // momentum-exchange sums.
    const bool general = valid && fluid && !fast;
    const bool near = general && (fl & kNearBit);
    S *gdst = (S *)(B.cur ? B.pop0 : B.pop1);
    int lfirst = 0x7fffffff, lend = -1;   // this cell's links
    if (general && !near) {
        // on a wall, away from bodies
        unsigned lo_w = 0u, hi_w = 0u;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool w = !((per >> a) & 1);
            lo_w |= (w && at_lo[a]) ? 1u << a : 0u;
            hi_w |= (w && at_hi[a]) ? 1u << a : 0u;
        }
        St::store(dst, (size_t)cell, f[0], B.scale);
        PushWall<S, 1>::run(dst, stride, cell, off_p, off_m, lo_w, hi_w, f, B.scale);
    } else if (general) {
        St::store(gdst, (size_t)cell, f[0], B.scale);
        Owners owner;
        int slot = 0;
        if (near) {
            neighbour_owners(B, cell, i, j, k, owner);
            slot = B.link_base[cell];
            lfirst = slot;
        }
        PushAll<S, 1>::run(B, gdst, stride, cell, i, j, k, owner, f, rho, slot);
        if (near) lend = slot;
    }
    if (__any(near)) body_links(B, lfirst, lend);
}

}  // namespace lbm
