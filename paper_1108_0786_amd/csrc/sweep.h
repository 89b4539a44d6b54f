// The fused stream-collide sweep (Sec. 2.1 and 2.3): one thread per cell
// loads the 19 deviations of its cell, collides them with LBGK and pushes
// the post-collision values to the neighbours; populations that would enter
// a wall are bounced back (Eq. lbm:bounce_back), those that would enter a
// body are bounced back with the moving-wall term of Sec. 2.3, and for those
// the link's post-collision value and density are recorded for the
// momentum-exchange sum (Eq. hydroF).
#pragma once
#include "geometry.h"

namespace lbm {

struct WorkItem {
    int box;
    int first;   // first cell of the block's tile
};

template <typename S>
struct SweepArgs {
    BoxDesc *boxes;
    const WorkItem *work;
};

template <typename S, int A>
__device__ __forceinline__ void push_one(const BoxDesc &B, S *dst, size_t N, int cell, int i,
                                         int j, int k, uint8_t fl,
                                         typename Storage<S>::C v,
                                         typename Storage<S>::C rho, int &nlink) {
    using St = Storage<S>;
    using C = typename St::C;
    int ti, tj, tk;
    if (!neighbour<A>(i, j, k, B.nx, B.ny, B.nz, B.per, ti, tj, tk)) {
        St::store(dst, (size_t)opp(A) * N + cell, v, B.scale);
        return;
    }
    const int tcell = ti + B.nx * (tj + B.ny * tk);
    if (fl & kNearBit) {
        const int owner = B.flags[tcell] & kOwnerMask;
        if (owner) {
            const DevBody &bd = B.bodies[owner - 1];
            double r[3], u[3];
            int d[3];
            lever_arm(bd, ti, tj, tk, B.nx, B.ny, B.nz, B.per, r, d);
            wall_velocity(bd, r, u);
            constexpr int O = opp(A);
            const double eu = (double)ex(O) * u[0] + (double)ey(O) * u[1] + (double)ez(O) * u[2];
            const double val = (double)v + 6.0 * wgt(A) * (double)rho * eu;
            St::store(dst, (size_t)O * N + cell, (C)val, B.scale);
            const int slot = B.link_base[cell] + nlink;
            ++nlink;
            if (slot >= 0 && slot < B.link_cap) B.link_val[slot] = make_double2((double)v, (double)rho);
            return;
        }
    }
    St::store(dst, (size_t)A * N + tcell, v, B.scale);
}

template <typename S, int A>
struct PushAll {
    static __device__ __forceinline__ void run(const BoxDesc &B, S *dst, size_t N, int cell, int i,
                                               int j, int k, uint8_t fl,
                                               const typename Storage<S>::C *f,
                                               typename Storage<S>::C rho, int &nlink) {
        push_one<S, A>(B, dst, N, cell, i, j, k, fl, f[A], rho, nlink);
        PushAll<S, A + 1>::run(B, dst, N, cell, i, j, k, fl, f, rho, nlink);
    }
};
template <typename S>
struct PushAll<S, 19> {
    static __device__ __forceinline__ void run(const BoxDesc &, S *, size_t, int, int, int, int,
                                               uint8_t, const typename Storage<S>::C *,
                                               typename Storage<S>::C, int &) {}
};

// LBGK collision in deviation form: dF~ = dF + omega (dF_eq - dF),
// dF_eq = w [drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)].
template <typename C>
__device__ __forceinline__ C collide(C *f, C omega) {
    C drho = f[0];
#pragma unroll
    for (int a = 1; a < 19; ++a) drho += f[a];
    C jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
    C jy = (f[3] - f[4]) + (f[7] - f[8]) + (f[10] - f[9]) + (f[15] - f[16]) + (f[17] - f[18]);
    C jz = (f[5] - f[6]) + (f[11] - f[12]) + (f[14] - f[13]) + (f[15] - f[16]) + (f[18] - f[17]);
    const C rho = C(1) + drho;
    const C inv = C(1) / rho;
    const C ux = jx * inv, uy = jy * inv, uz = jz * inv;
    const C usq15 = C(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        const C eu = C(ex(a)) * ux + C(ey(a)) * uy + C(ez(a)) * uz;
        const C feq = C(wgt(a)) * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - usq15));
        f[a] = f[a] + omega * (feq - f[a]);
    }
    return rho;
}

template <typename S, int BLOCK>
__global__ __launch_bounds__(BLOCK) void sweep_kernel(BoxDesc *boxes, const WorkItem *work) {
    using St = Storage<S>;
    using C = typename St::C;
    const WorkItem wk = work[blockIdx.x];
    const BoxDesc &B = boxes[wk.box];
    const int cell = wk.first + (int)threadIdx.x;
    if (cell >= B.N) return;
    const uint8_t fl = B.flags[cell];
    if (fl & kOwnerMask) return;  // inside a body: no fluid
    const size_t N = (size_t)B.N;
    const S *src = (const S *)(B.cur ? B.pop1 : B.pop0);
    S *dst = (S *)(B.cur ? B.pop0 : B.pop1);
    C f[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) f[a] = St::load(src, (size_t)a * N + cell, B.inv_scale);
    const C omega = sizeof(C) == 8 ? (C)B.omega : (C)B.omegaf;
    const C rho = collide<C>(f, omega);
    int i, j, k;
    decode_cell(cell, B.nx, B.ny, i, j, k);
    St::store(dst, (size_t)cell, f[0], B.scale);
    int nlink = 0;
    PushAll<S, 1>::run(B, dst, N, cell, i, j, k, fl, f, rho, nlink);
}

}  // namespace lbm
