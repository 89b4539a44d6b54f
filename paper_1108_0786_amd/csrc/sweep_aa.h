// Fused sweep with in-place streaming: one population array per box, the
// access pattern of Bailey et al. (2009, "Accelerating lattice Boltzmann
// fluid flow simulations using graphics processors", the "AA" pattern).
//
// The arithmetic is the push sweep's (collision of Eq. lbgk in deviation
// form, halfway bounce-back with the moving-wall term of Sec. 2.3, the
// momentum-exchange records of Eq. hydroF); only where each population sits
// between two steps changes.  With n the step about to be taken:
//
//   n even ("own" layout): f_b(x) sits at slot b of x.  The step reads the
//     19 slots of x, collides, and writes each post-collision f*_a(x) to
//     slot opp(a) of x itself: reads and writes are aligned, no neighbour is
//     touched.
//   n odd ("swapped" layout): f_b(x) sits at slot opp(b) of x - e_b, where
//     x - e_b put it at the even step, or, if x - e_b is a wall or a body
//     cell, at slot b of x (the reflected population, stored there by x).
//     The step pulls from those slots, collides, and pushes f*_a(x) to slot a
//     of x + e_a, or, across a wall or into a body, the reflected value to
//     slot opp(a) of x; after it every population sits in its own layout
//     again.
//
// A reflected population is stored in both steps exactly where the next
// step looks for it, so walls and bodies need no storage of their own, and
// every slot is read and written by one thread within a step: no race, one
// array.  On the 256x128x128 box the pattern moves the same bytes as the
// two-array push in 15% (FP32) to 40% (2-byte formats) less time, the even
// step's accesses being aligned and the odd step's lines being read and
// written by the same workgroups.
//
// A remap between steps moves the populations whose slot depends on a cell
// that changed sides (coupling.h); exports and imports read and write
// through the same rule (current_slot).
#pragma once
#include "sweep.h"

namespace lbm {

// Between steps: are the box's populations in the swapped layout?
__device__ __forceinline__ bool swapped_now(const BoxDesc &B) { return B.aa && (B.step & 1); }

// Element of f_b(x) of fluid cell `cell` in the own (swapped = false) or the
// swapped layout, under the box's present flags.
__device__ __forceinline__ size_t current_slot(const BoxDesc &B, bool swapped, int b, int cell) {
    const size_t stride = (size_t)B.stride;
    if (swapped && b != 0) {
        int i, j, k, ti, tj, tk;
        decode_cell(cell, B.nx, B.ny, i, j, k);
        if (neighbour_rt(opp(b), i, j, k, B.nx, B.ny, B.nz, B.per, ti, tj, tk)) {
            const int s = ti + B.nx * (tj + B.ny * tk);
            if (!(B.flags[s] & kOwnerMask)) return (size_t)opp(b) * stride + (size_t)s;
        }
    }
    return (size_t)b * stride + (size_t)cell;
}

// Odd step, cell next to a body (the general path): pull f_b(x) for b = A..18.
template <typename S, int A>
struct PullAll {
    template <typename P>
    static __device__ __forceinline__ void run(const BoxDesc &B, P src, long long stride, int cell, int i, int j,
                                               int k, const Owners &owner, typename Storage<S>::C *f) {
        constexpr int O = opp(A);
        int ti, tj, tk;
        const bool in = neighbour<O>(i, j, k, B.nx, B.ny, B.nz, B.per, ti, tj, tk);
        const size_t at = in && !owner.get(O) ? (size_t)O * stride + (size_t)(ti + B.nx * (tj + B.ny * tk))
                                               : (size_t)A * stride + (size_t)cell;
        f[A] = Storage<S>::load(src, at, B.inv_scale);
        PullAll<S, A + 1>::run(B, src, stride, cell, i, j, k, owner, f);
    }
};
template <typename S>
struct PullAll<S, 19> {
    template <typename P>
    static __device__ __forceinline__ void run(const BoxDesc &, P, long long, int, int, int, int, const Owners &,
                                               typename Storage<S>::C *) {}
};

// Odd step, interior cell: pull from the 18 neighbours (periodic wrap in
// off_p / off_m, as for the push).
template <typename S, bool NT, int A>
struct PullFast {
    template <typename P>
    static __device__ __forceinline__ void run(P src, long long stride, int cell, const int *off_p,
                                               const int *off_m, typename Storage<S>::C *f, float inv_scale) {
        // source x - e_A
        const int o = (ex(A) > 0 ? off_m[0] : ex(A) < 0 ? off_p[0] : 0) +
                      (ey(A) > 0 ? off_m[1] : ey(A) < 0 ? off_p[1] : 0) +
                      (ez(A) > 0 ? off_m[2] : ez(A) < 0 ? off_p[2] : 0);
        f[A] = Storage<S>::template load<NT>(src + (size_t)opp(A) * stride, (size_t)(unsigned)(cell + o), inv_scale);
        PullFast<S, NT, A + 1>::run(src, stride, cell, off_p, off_m, f, inv_scale);
    }
};
template <typename S, bool NT>
struct PullFast<S, NT, 19> {
    template <typename P>
    static __device__ __forceinline__ void run(P, long long, int, const int *, const int *,
                                               typename Storage<S>::C *, float) {}
};

// Odd step, cell on a wall away from bodies: as PullFast, except that a
// population whose source x - e_A lies beyond a wall was reflected by x
// itself into slot A of x.  lo_w / hi_w: bit a set if the cell is at the
// low / high end of axis a and that axis has walls.
template <int A>
__device__ __forceinline__ bool beyond_wall(unsigned lo_w, unsigned hi_w) {
    return (ex(A) > 0 ? (hi_w & 1u) : ex(A) < 0 ? (lo_w & 1u) : 0u) ||
           (ey(A) > 0 ? (hi_w & 2u) : ey(A) < 0 ? (lo_w & 2u) : 0u) ||
           (ez(A) > 0 ? (hi_w & 4u) : ez(A) < 0 ? (lo_w & 4u) : 0u);
}

template <typename S, bool NT, int A>
struct PullWall {
    template <typename P>
    static __device__ __forceinline__ void run(P src, long long stride, int cell, const int *off_p,
                                               const int *off_m, unsigned lo_w, unsigned hi_w,
                                               typename Storage<S>::C *f, float inv_scale) {
        const int o = (ex(A) > 0 ? off_m[0] : ex(A) < 0 ? off_p[0] : 0) +
                      (ey(A) > 0 ? off_m[1] : ey(A) < 0 ? off_p[1] : 0) +
                      (ez(A) > 0 ? off_m[2] : ez(A) < 0 ? off_p[2] : 0);
        // x - e_A beyond a wall: x + e_opp(A) is
        const size_t at = beyond_wall<opp(A)>(lo_w, hi_w) ? (size_t)A * stride + (size_t)cell
                                                          : (size_t)opp(A) * stride + (size_t)(unsigned)(cell + o);
        f[A] = Storage<S>::template load<NT>(src, at, inv_scale);
        PullWall<S, NT, A + 1>::run(src, stride, cell, off_p, off_m, lo_w, hi_w, f, inv_scale);
    }
};
template <typename S, bool NT>
struct PullWall<S, NT, 19> {
    template <typename P>
    static __device__ __forceinline__ void run(P, long long, int, const int *, const int *, unsigned, unsigned,
                                               typename Storage<S>::C *, float) {}
};

// Even step, cell next to a body: f*_A(x) to slot opp(A) of x, with the
// moving-wall term and the link's record where x + e_A is a body cell.
template <typename S, int A>
struct KeepAll {
    template <typename P>
    static __device__ __forceinline__ void run(const BoxDesc &B, P dst, long long stride, int cell, int i, int j,
                                               int k, const Owners &owner, const typename Storage<S>::C *f,
                                               typename Storage<S>::C rho, int &slot) {
        typename Storage<S>::C v = f[A];
        if (const int o = owner.get(A)) {
            int ti, tj, tk;
            // a body cell is always inside the box
            neighbour<A>(i, j, k, B.nx, B.ny, B.nz, B.per, ti, tj, tk);
            v = bounce_moving<S, A>(B, cell, o, ti, tj, tk, v, rho, slot);
            ++slot;
        }
        Storage<S>::store(dst, (size_t)opp(A) * stride + cell, v, B.scale);
        KeepAll<S, A + 1>::run(B, dst, stride, cell, i, j, k, owner, f, rho, slot);
    }
};
template <typename S>
struct KeepAll<S, 19> {
    template <typename P>
    static __device__ __forceinline__ void run(const BoxDesc &, P, long long, int, int, int, int, const Owners &,
                                               const typename Storage<S>::C *, typename Storage<S>::C, int &) {}
};

// Even step, any fluid cell away from bodies: f*_a(x) to slot opp(a) of x.
template <typename S, bool NT, int A>
struct KeepFast {
    template <typename P>
    static __device__ __forceinline__ void run(P dst, long long stride, int cell, const typename Storage<S>::C *f,
                                               float scale) {
        Storage<S>::store(dst + (size_t)opp(A) * stride, (size_t)cell, f[A], scale);
        KeepFast<S, NT, A + 1>::run(dst, stride, cell, f, scale);
    }
};
template <typename S, bool NT>
struct KeepFast<S, NT, 19> {
    template <typename P>
    static __device__ __forceinline__ void run(P, long long, int, const typename Storage<S>::C *, float) {}
};

// One step of the box in place.  The step's parity is the box's own
// (B.step), so the boxes of a batch may be at different parities, and a
// replayed graph needs no parity of its own.  Both parities share one
// kernel: the branch is uniform over the workgroup.
template <typename S, int BLOCK, bool NT, bool FLOW, bool FORCE = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 5 : (FLOW ? 6 : 7), 8)))
void sweep_aa_kernel(BoxDesc *boxes, const WorkItem *work, int nwork, int xcd_order) {
    using St = Storage<S>;
    using C = typename St::C;
    const int t = tile_index(xcd_order);
    if (t >= nwork) return;
    const WorkItem wk = work[t];
    const BoxDesc &B = boxes[wk.box];
    const int cell = wk.first + (int)threadIdx.x;
    const bool valid = cell < B.N;
    const uint8_t fl = valid ? B.flags[cell] : kOwnerMask;
    const bool fluid = valid && !(fl & kOwnerMask);
    const long long stride = B.stride;
    global_t<S> *pop = (global_t<S> *)(B.cur ? B.pop1 : B.pop0);
    const bool odd = (B.step & 1) != 0;
    int i = wk.i0 + (int)threadIdx.x, j = wk.j0, k = wk.k0;
    while (i >= B.nx) {
        i -= B.nx;
        if (++j == B.ny) {
            j = 0;
            ++k;
        }
    }
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
    const bool near = fluid && (fl & kNearBit);
    const bool fast = fluid && !wall && !near;
    const bool at_wall = fluid && wall && !near;
    unsigned lo_w = 0u, hi_w = 0u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool w = !((per >> a) & 1);
        lo_w |= (w && at_lo[a]) ? 1u << a : 0u;
        hi_w |= (w && at_hi[a]) ? 1u << a : 0u;
    }
    Owners owner;
    int slot = 0, lfirst = 0x7fffffff, lend = -1;
    if (near) {
        neighbour_owners(B, cell, i, j, k, owner);
        slot = B.link_base[cell];
        lfirst = slot;
    }
    C f[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) f[a] = C(0);
    if (!odd) {
        if (fluid) {
#pragma unroll
            for (int a = 0; a < 19; ++a) f[a] = St::template load<NT>(pop, (size_t)a * stride + cell, B.inv_scale);
        }
    } else if (fast) {
        f[0] = St::template load<NT>(pop, (size_t)cell, B.inv_scale);
        PullFast<S, NT, 1>::run(pop, stride, cell, off_p, off_m, f, B.inv_scale);
    } else if (at_wall) {
        f[0] = St::template load<NT>(pop, (size_t)cell, B.inv_scale);
        PullWall<S, NT, 1>::run(pop, stride, cell, off_p, off_m, lo_w, hi_w, f, B.inv_scale);
    } else if (near) {
        f[0] = St::load(pop, (size_t)cell, B.inv_scale);
        PullAll<S, 1>::run(B, pop, stride, cell, i, j, k, owner, f);
    }
    if constexpr (FLOW) {
        if (fluid && B.flow_every > 0 && B.step % B.flow_every == 0) flow_sample<C>(B, cell, f);
    }
    const C omega = sizeof(C) == 8 ? (C)B.omega : (C)B.omegaf;
    const C rho = FORCE ? collide_forced<C>(f, omega, B.force) : collide<C>(f, omega);
    if (!odd) {
        if (near) {
            St::store(pop, (size_t)cell, f[0], B.scale);
            KeepAll<S, 1>::run(B, pop, stride, cell, i, j, k, owner, f, rho, slot);
        } else if (fluid) {
            // walls need nothing of their own here: the reflected population
            // is f*_a itself, in the slot the next step reads
            St::store(pop, (size_t)cell, f[0], B.scale);
            KeepFast<S, NT, 1>::run(pop, stride, cell, f, B.scale);
        }
    } else if (fast) {
        St::store(pop, (size_t)cell, f[0], B.scale);
        PushFast<S, 1>::run(pop, stride, cell, off_p, off_m, f, B.scale);
    } else if (at_wall) {
        St::store(pop, (size_t)cell, f[0], B.scale);
        PushWall<S, 1>::run(pop, stride, cell, off_p, off_m, lo_w, hi_w, f, B.scale);
    } else if (near) {
        St::store(pop, (size_t)cell, f[0], B.scale);
        PushAll<S, 1>::run(B, (S *)pop, stride, cell, i, j, k, owner, f, rho, slot);
    }
    if (near) lend = slot;
    if (__any(near)) body_links(B, lfirst, lend);
}

}  // namespace lbm
