// Hand-written reverse mode of the coupled step (flags held fixed).
//
// Forward step n, per fluid cell x and link (x, alpha, b) into body b:
//   dF~ = dF + omega (dF_eq(drho, j) - dF)                 (Eq. collide)
//   dF'(y, alpha) = dF~(x, alpha)                            (fluid neighbour y)
//   dF'(x, opp)   = dF~(x, alpha)                            (wall)
//   dF'(x, opp)   = dF~(x, alpha) + M,  M = 6 w rho e_opp.u  (moving wall, Sec. 2.3)
//   u = V_b + Omega_b x r,  r = lever arm of the body cell
//   F_b += e_alpha s,  T_b += r x e_alpha s,  s = 2 dF~ + M  (Eq. hydroF)
//   V' = V + (F + F_dri + F_osci)/m,  D' = D + V',  Omega' = Omega + I^-1 T.
// The reverse sweep pulls the adjoint of dF' back through these maps:
//   lam~(x, alpha) = lam'(y, alpha) | lam'(x, opp) | lam'(x, opp) + 2 lam_s,
//   lam_s = e_alpha . (lam_F + lam_T x r),   lam_M = lam'(x, opp) + lam_s,
//   lam_rho += 6 w (e_opp.u) lam_M,  lam_u = 6 w rho e_opp lam_M,
// and through the collision, with dF_eq = w [drho + 3 e.j + (4.5 (e.j)^2 - 1.5 j.j)/rho]:
//   lam(x, beta) = (1 - omega) lam~_beta + omega (g_rho + e_beta . g_j) + lam_rho,
//   g_rho = sum_a lam~_a w_a [1 - (4.5 (e_a.j)^2 - 1.5 j.j)/rho^2],
//   g_j   = sum_a lam~_a w_a [3 e_a + (9 (e_a.j) e_a - 3 j)/rho].
// Each link also returns its share of the body adjoints: lam_V += lam_u,
// lam_Omega += r x lam_u, lam_D += -(lam_u x Omega) - (t x lam_T), t = e_alpha s.
#pragma once
#include "coupling.h"

namespace lbm {

// body adjoint state of one body
struct AdjBody {
    double lD[3], lV[3], lO[3];     // adjoints of D, V, Omega at the current reverse step
    double lF[3], lT[3];            // adjoints of the hydrodynamic force / torque of step n
    double muV[3];                  // adjoint of V^{n+1} including its use in D^{n+1}
    double lDs[3], lVs[3];          // spring contributions to lam_D^n, lam_V^n
    // with the two-step force mean: the plain adjoints of the force and torque
    // of step n+1 (the hydrodynamic sums of step n move the bodies at steps n
    // and n+1, half each)
    double lFn[3], lTn[3];
};

// body state of one step kept for the reverse pass
struct BodyHist {
    double D[3], V[3], O[3], q[4];
};

struct AdjLinkRec {
    double v[9];                    // lam_V (3), lam_Omega (3), lam_D (3)
    double pad;
};

struct AdjArgs {
    const void *state;              // dF^n of the step being reversed (storage type)
    const double *lam_next;         // adjoint of dF^{n+1}, 19 * stride doubles
    double *lam;                    // adjoint of dF^n (output)
    const BodyHist *hist;           // body states at step n, nb entries
    AdjBody *adj;                   // body adjoints (lam_F, lam_T read here)
    AdjLinkRec *lrec;               // one record per link (output)
};

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// lever arm of cell (i,j,k) from a body state in the history
__device__ __forceinline__ void hist_lever(const DevBody &bd, const BodyHist &h, int i, int j, int k,
                                           const BoxDesc &B, double r[3]) {
    const double X[3] = {bd.anchor[0] + h.D[0], bd.anchor[1] + h.D[1], bd.anchor[2] + h.D[2]};
    int d[3];
    lever_arm_at(X, i, j, k, B.nx, B.ny, B.nz, B.per, r, d);
}

// The cell's state that every direction of the reverse sweep reads.
struct AdjCell {
    double drho, rho, omega, jj, j[3];
    int cell, i, j_, k, near;
    size_t stride;
};

// Reverse of the push of direction A out of fluid cell x: lam~_A(x) (to
// lt[A * 256], the thread's column of an LDS table) from the adjoint of the
// step's output, and for a link into a body its share of the body adjoints
// (scratch record) and of lam_rho.  A is a template argument so that the
// cell's 19 populations stay in registers.
template <int A>
__device__ __forceinline__ void adj_pull(const BoxDesc &B, const AdjArgs &args, const AdjCell &c, const double *f,
                                         double *lt, double &lrho, int &nlink) {
    constexpr int o = opp(A);
    int ti, tj, tk;
    if (!neighbour<A>(c.i, c.j_, c.k, B.nx, B.ny, B.nz, B.per, ti, tj, tk)) {
        lt[A * 256] = args.lam_next[(size_t)o * c.stride + c.cell];
        return;
    }
    const int tcell = ti + B.nx * (tj + B.ny * tk);
    const int owner = c.near ? (B.flags[tcell] & kOwnerMask) : 0;
    if (!owner) {
        lt[A * 256] = args.lam_next[(size_t)A * c.stride + tcell];
        return;
    }
    // link into body owner-1
    const int b = owner - 1;
    const BodyHist &h = args.hist[b];
    const AdjBody &ab = args.adj[b];
    double r[3];
    hist_lever(B.bodies[b], h, ti, tj, tk, B, r);
    double Oxr[3];
    cross3(h.O, r, Oxr);
    const double u[3] = {h.V[0] + Oxr[0], h.V[1] + Oxr[1], h.V[2] + Oxr[2]};
    const double e[3] = {(double)ex(A), (double)ey(A), (double)ez(A)};
    const double eou = -(e[0] * u[0] + e[1] * u[1] + e[2] * u[2]);
    // forward post-collision value of this population
    const double eu_f = (e[0] * c.j[0] + e[1] * c.j[1] + e[2] * c.j[2]);
    const double feq = wgt(A) * (c.drho + 3.0 * eu_f + (4.5 * eu_f * eu_f - 1.5 * c.jj) / c.rho);
    const double ft = f[A] + c.omega * (feq - f[A]);
    const double M = 6.0 * wgt(A) * c.rho * eou;
    const double s = 2.0 * ft + M;
    double lTxr[3];
    cross3(ab.lT, r, lTxr);
    const double ls = e[0] * (ab.lF[0] + lTxr[0]) + e[1] * (ab.lF[1] + lTxr[1]) + e[2] * (ab.lF[2] + lTxr[2]);
    const double ln = args.lam_next[(size_t)o * c.stride + c.cell];
    lt[A * 256] = ln + 2.0 * ls;
    const double lM = ln + ls;
    lrho += 6.0 * wgt(A) * eou * lM;
    const double lu[3] = {-6.0 * wgt(A) * c.rho * e[0] * lM, -6.0 * wgt(A) * c.rho * e[1] * lM,
                          -6.0 * wgt(A) * c.rho * e[2] * lM};
    const int slot = B.link_base[c.cell] + nlink;
    ++nlink;
    if (slot >= 0 && slot < B.link_cap) {
        AdjLinkRec rec;
        double rxl[3], luxO[3], txl[3];
        cross3(r, lu, rxl);
        cross3(lu, h.O, luxO);
        const double t[3] = {e[0] * s, e[1] * s, e[2] * s};
        cross3(t, ab.lT, txl);
        for (int q = 0; q < 3; ++q) {
            rec.v[q] = lu[q];
            rec.v[3 + q] = rxl[q];
            rec.v[6 + q] = -luxO[q] - txl[q];
        }
        rec.pad = 0.0;
        args.lrec[slot] = rec;
    }
}

template <int A>
struct AdjPullAll {
    static __device__ __forceinline__ void run(const BoxDesc &B, const AdjArgs &args, const AdjCell &c,
                                               const double *f, double *lt, double &lrho, int &nlink) {
        adj_pull<A>(B, args, c, f, lt, lrho, nlink);
        AdjPullAll<A + 1>::run(B, args, c, f, lt, lrho, nlink);
    }
};
template <>
struct AdjPullAll<19> {
    static __device__ __forceinline__ void run(const BoxDesc &, const AdjArgs &, const AdjCell &, const double *,
                                               double *, double &, int &) {}
};

template <typename S>
__global__ __launch_bounds__(256) void adjoint_sweep_kernel(const BoxDesc *boxes, AdjArgs args) {
    const BoxDesc &B = boxes[0];
    const int cell = blockIdx.x * 256 + (int)threadIdx.x;
    if (cell >= B.N) return;
    const size_t stride = (size_t)B.stride;
    const uint8_t fl = B.flags[cell];
    if (fl & kOwnerMask) {
#pragma unroll
        for (int a = 0; a < 19; ++a) args.lam[(size_t)a * stride + cell] = 0.0;
        return;
    }
    // forward quantities at x
    double f[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) f[a] = load_dev<S>(args.state, (size_t)a * stride + cell, B.inv_scale);
    AdjCell c;
    double drho = 0.0, j[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        drho += f[a];
        j[0] += ex(a) * f[a];
        j[1] += ey(a) * f[a];
        j[2] += ez(a) * f[a];
    }
    c.drho = drho;
    c.rho = 1.0 + drho;
    c.omega = B.omega;
    c.jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
    for (int q = 0; q < 3; ++q) c.j[q] = j[q];
    c.cell = cell;
    c.stride = stride;
    c.near = (fl & kNearBit) != 0;
    decode_cell(cell, B.nx, B.ny, c.i, c.j_, c.k);
    // the 19 pulled adjoints wait in LDS for the collision adjoint (as a
    // private array the compiler keeps them in scratch memory)
    __shared__ double lt_sh[19 * 256];
    double *lt = lt_sh + threadIdx.x;
    lt[0] = args.lam_next[cell];
    double lrho = 0.0;
    int nlink = 0;
    AdjPullAll<1>::run(B, args, c, f, lt, lrho, nlink);
    const double rho = c.rho, jj = c.jj, omega = c.omega;
    // collision adjoint
    double grho = 0.0, gj[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        const double e[3] = {(double)ex(a), (double)ey(a), (double)ez(a)};
        const double ej = e[0] * j[0] + e[1] * j[1] + e[2] * j[2];
        const double w = wgt(a) * lt[a * 256];
        grho += w * (1.0 - (4.5 * ej * ej - 1.5 * jj) / (rho * rho));
#pragma unroll
        for (int q = 0; q < 3; ++q) gj[q] += w * (3.0 * e[q] + (9.0 * ej * e[q] - 3.0 * j[q]) / rho);
    }
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        const double egj = ex(a) * gj[0] + ey(a) * gj[1] + ez(a) * gj[2];
        args.lam[(size_t)a * stride + cell] = (1.0 - omega) * lt[a * 256] + omega * (grho + egj) + lrho;
    }
}

// Driving forces of Eqs. FB1-FB3 at step n and their derivatives with
// respect to the amplitude and the phase lag (x components, per body).
__device__ void drive_grad(const BoxDesc &B, const DevDrive *drives, long long n, double dFa[kMaxBodies],
                           double dFp[kMaxBodies]) {
    for (int b = 0; b < B.nb; ++b) dFa[b] = dFp[b] = 0.0;
    for (int e = 0; e < B.nd; ++e) {
        const DevDrive &dv = drives[e];
        const double om = 2.0 * M_PI / dv.period;
        double sl = -sin(om * (double)n), sr = sin(om * (double)n - dv.phase_lag);
        double pr = -dv.amplitude * cos(om * (double)n - dv.phase_lag);
        if (dv.gate && om * (double)n < dv.phase_lag) sr = pr = 0.0;
        if (dv.off_left >= 0 && n >= dv.off_left) sl = 0.0;
        if (dv.off_right >= 0 && n >= dv.off_right) sr = pr = 0.0;
        dFa[dv.left] += sl;
        dFa[dv.right] += sr;
        dFa[dv.middle] -= sl + sr;
        dFp[dv.right] += pr;
        dFp[dv.middle] -= pr;
    }
}

// Body adjoint, one workgroup: finish the reverse of step n+1 (if `finish`)
// with the link records of its sweep, then begin the reverse of step n (if
// n >= 0): adjoints of the hydrodynamic force and torque for the sweep of
// step n, spring contributions, and the parameter gradients.  The body
// adjoints, body tables, the step's history and the gradient are staged in
// LDS by the whole workgroup first (one round of loads), so that the serial
// part works from LDS, and stored back at the end.
__global__ __launch_bounds__(kCoupleThreads) void adjoint_body_kernel(const BoxDesc *boxes, AdjBody *adj,
                                                                      const BodyHist *hist_np1,
                                                                      const BodyHist *hist_n, const AdjLinkRec *lrec,
                                                                      long long n, int finish, double *grad) {
    __shared__ double sums[kMaxBodies][9];
    __shared__ int gsum[kMaxBodies][3];
    __shared__ AdjBody s_adj[kMaxBodies];
    __shared__ DevBody s_body[kMaxBodies];
    __shared__ BodyHist s_hist[kMaxBodies];
    __shared__ DevSpring s_spring[kMaxSprings];
    __shared__ DevDrive s_drive[kMaxDrives];
    __shared__ double s_grad[3];
    const BoxDesc &B = boxes[0];
    const int nb = B.nb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    copy_words(s_adj, adj, (int)sizeof(AdjBody) * nb);
    copy_words(s_body, B.bodies, (int)sizeof(DevBody) * nb);
    copy_words(s_hist, hist_n, (int)sizeof(BodyHist) * nb);
    copy_words(s_spring, B.springs, (int)sizeof(DevSpring) * B.ns);
    copy_words(s_drive, B.drives, (int)sizeof(DevDrive) * B.nd);
    if (threadIdx.x < 3) s_grad[threadIdx.x] = grad[threadIdx.x];
    __syncthreads();
    if (finish) {
        const int L = min(B.link_count, B.link_cap);
        // one pass over the links per kBodiesPerPass bodies: every thread
        // loads its links l, l + 256, ... four at a time (owner, direction and
        // record together) and adds each into its body's sums; the lanes and
        // then the four waves are added in a fixed order, so the sums do not
        // depend on timing
        constexpr int kBodiesPerPass = 4;
        __shared__ double wred[kCoupleThreads / 64][kBodiesPerPass][9];
        __shared__ int gred[kCoupleThreads / 64][kBodiesPerPass][3];
        for (int b0 = 0; b0 < nb; b0 += kBodiesPerPass) {
            double acc[kBodiesPerPass][9];
            int g[kBodiesPerPass][3];
#pragma unroll
            for (int k = 0; k < kBodiesPerPass; ++k) {
#pragma unroll
                for (int q = 0; q < 9; ++q) acc[k][q] = 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q) g[k][q] = 0;
            }
            for (int l0 = threadIdx.x; l0 < L; l0 += 4 * kCoupleThreads) {
                int lb[4], ld[4];
                AdjLinkRec rec[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int l = l0 + u * kCoupleThreads;
                    const bool ok = l < L;
                    lb[u] = ok ? B.link_body[l] : -1;
                    ld[u] = ok ? B.link_dir[l] : 0;
                    if (ok) rec[u] = lrec[l];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int cw = two_w36(ld[u]);
#pragma unroll
                    for (int k = 0; k < kBodiesPerPass; ++k) {
                        if (lb[u] != b0 + k) continue;
#pragma unroll
                        for (int q = 0; q < 9; ++q) acc[k][q] += rec[u].v[q];
                        g[k][0] += ex(ld[u]) * cw;
                        g[k][1] += ey(ld[u]) * cw;
                        g[k][2] += ez(ld[u]) * cw;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < kBodiesPerPass; ++k) {
#pragma unroll
                for (int q = 0; q < 9; ++q) acc[k][q] = wave_sum(acc[k][q]);
#pragma unroll
                for (int q = 0; q < 3; ++q) g[k][q] = wave_sum_int(g[k][q]);
                if (lane == 0) {
#pragma unroll
                    for (int q = 0; q < 9; ++q) wred[wave][k][q] = acc[k][q];
#pragma unroll
                    for (int q = 0; q < 3; ++q) gred[wave][k][q] = g[k][q];
                }
            }
            __syncthreads();
            const int t = threadIdx.x;
            if (t < kBodiesPerPass * 12) {
                const int k = t / 12, q = t % 12;
                if (b0 + k < nb) {
                    if (q < 9) {
                        double v = wred[0][k][q];
                        for (int w = 1; w < kCoupleThreads / 64; ++w) v = v + wred[w][k][q];
                        sums[b0 + k][q] = v;
                    } else {
                        int v = gred[0][k][q - 9];
                        for (int w = 1; w < kCoupleThreads / 64; ++w) v += gred[w][k][q - 9];
                        gsum[b0 + k][q - 9] = v;
                    }
                }
            }
            __syncthreads();
        }
        if ((int)threadIdx.x < nb) {
            const int b = threadIdx.x;
            AdjBody &ab = s_adj[b];
            const double G[3] = {gsum[b][0] / 36.0, gsum[b][1] / 36.0, gsum[b][2] / 36.0};
            double GxlT[3];
            cross3(G, ab.lT, GxlT);
            for (int q = 0; q < 3; ++q) {
                const double lV = ab.muV[q] + ab.lVs[q] + sums[b][q];
                const double lO = ab.lO[q] + sums[b][3 + q];
                const double lD = ab.lD[q] + ab.lDs[q] + sums[b][6 + q] - GxlT[q];
                ab.lV[q] = lV;
                ab.lO[q] = lO;
                ab.lD[q] = lD;
            }
        }
        __syncthreads();
    }
    // per-body tables of thread 0 in LDS: indexed by body numbers read at run
    // time, private arrays would live in scratch memory
    __shared__ double dFa[kMaxBodies], dFp[kMaxBodies], lF[kMaxBodies][3];
    if (n >= 0 && threadIdx.x == 0) {
        // begin step n: adjoints of F^n, T^n; springs; parameters
        drive_grad(B, s_drive, n, dFa, dFp);
        for (int b = 0; b < nb; ++b) {
            AdjBody &ab = s_adj[b];
            const DevBody &bd = s_body[b];
            for (int q = 0; q < 3; ++q) {
                ab.muV[q] = ab.lV[q] + ab.lD[q];
                lF[b][q] = bd.kinematic == 1 ? 0.0 : ab.muV[q] / bd.mass;
                ab.lF[q] = lF[b][q];
                ab.lDs[q] = ab.lVs[q] = 0.0;
            }
            // T enters Omega' = Omega + R diag(1/I) R^T T: lam_T = R diag(1/I) R^T lam_Omega
            const double w = s_hist[b].q[0], x = s_hist[b].q[1], y = s_hist[b].q[2], z = s_hist[b].q[3];
            const double R[3][3] = {
                {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
            double bt[3];
            for (int p = 0; p < 3; ++p)
                bt[p] = bd.kinematic != 0 ? 0.0
                                     : (R[0][p] * ab.lO[0] + R[1][p] * ab.lO[1] + R[2][p] * ab.lO[2]) / bd.inertia[p];
            for (int p = 0; p < 3; ++p) ab.lT[p] = R[p][0] * bt[0] + R[p][1] * bt[1] + R[p][2] * bt[2];
            if (B.force_avg) {
                // the hydrodynamic force and torque of step n enter the updates of
                // steps n and n+1 with weight 1/2 each
                for (int q = 0; q < 3; ++q) {
                    const double f = ab.lF[q], t = ab.lT[q];
                    ab.lF[q] = 0.5 * (f + ab.lFn[q]);
                    ab.lT[q] = 0.5 * (t + ab.lTn[q]);
                    ab.lFn[q] = f;
                    ab.lTn[q] = t;
                }
            }
            s_grad[0] += lF[b][0] * dFa[b];
            s_grad[1] += lF[b][0] * dFp[b];
        }
        for (int e = 0; e < B.ns; ++e) {
            const DevSpring &sp = s_spring[e];
            const BodyHist &hi = s_hist[sp.i], &hj = s_hist[sp.j];
            const DevBody &bi = s_body[sp.i], &bj = s_body[sp.j];
            double d[3], lf[3];
            for (int q = 0; q < 3; ++q) {
                d[q] = (bi.anchor[q] - bj.anchor[q]) + (hi.D[q] - hj.D[q]);
                lf[q] = lF[sp.i][q] - lF[sp.j][q];
            }
            const double ell = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double c1 = 1.0 - sp.rest_len / ell, c2 = sp.rest_len / (ell * ell * ell);
            const double dl = d[0] * lf[0] + d[1] * lf[1] + d[2] * lf[2];
            // df/dk = -(ell - l0) d / ell
            s_grad[2] += -(ell - sp.rest_len) / ell * dl;
            for (int q = 0; q < 3; ++q) {
                const double gD = -sp.k * (c1 * lf[q] + c2 * d[q] * dl);
                s_adj[sp.i].lDs[q] += gD;
                s_adj[sp.j].lDs[q] -= gD;
                s_adj[sp.i].lVs[q] += -sp.gamma * lf[q];
                s_adj[sp.j].lVs[q] += sp.gamma * lf[q];
            }
        }
    }
    __syncthreads();
    copy_words(adj, s_adj, (int)sizeof(AdjBody) * nb);
    if (threadIdx.x < 3) grad[threadIdx.x] = s_grad[threadIdx.x];
    (void)hist_np1;
}

}  // namespace lbm
