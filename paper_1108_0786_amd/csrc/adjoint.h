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
    DevBody tmp = bd;
    for (int q = 0; q < 3; ++q) tmp.D[q] = h.D[q];
    int d[3];
    lever_arm(tmp, i, j, k, B.nx, B.ny, B.nz, B.per, r, d);
}

template <typename S>
__global__ __launch_bounds__(256) void adjoint_sweep_kernel(const BoxDesc *boxes, AdjArgs args) {
    const BoxDesc &B = boxes[0];
    const int cell = blockIdx.x * 256 + (int)threadIdx.x;
    if (cell >= B.N) return;
    const size_t stride = (size_t)B.stride;
    const uint8_t fl = B.flags[cell];
    if (fl & kOwnerMask) {
        for (int a = 0; a < 19; ++a) args.lam[(size_t)a * stride + cell] = 0.0;
        return;
    }
    // forward quantities at x
    double f[19];
    for (int a = 0; a < 19; ++a) f[a] = load_dev<S>(args.state, (size_t)a * stride + cell, B.inv_scale);
    double drho = 0.0, j[3] = {0, 0, 0};
    for (int a = 0; a < 19; ++a) {
        drho += f[a];
        j[0] += ex(a) * f[a];
        j[1] += ey(a) * f[a];
        j[2] += ez(a) * f[a];
    }
    const double rho = 1.0 + drho;
    const double omega = B.omega;
    const double jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
    int i, jy, kz;
    decode_cell(cell, B.nx, B.ny, i, jy, kz);
    double lt[19];
    lt[0] = args.lam_next[cell];
    double lrho = 0.0;
    int nlink = 0;
    for (int a = 1; a < 19; ++a) {
        const int o = opp(a);
        int ti, tj, tk;
        if (!neighbour_rt(a, i, jy, kz, B.nx, B.ny, B.nz, B.per, ti, tj, tk)) {
            lt[a] = args.lam_next[(size_t)o * stride + cell];
            continue;
        }
        const int tcell = ti + B.nx * (tj + B.ny * tk);
        const int owner = (fl & kNearBit) ? (B.flags[tcell] & kOwnerMask) : 0;
        if (!owner) {
            lt[a] = args.lam_next[(size_t)a * stride + tcell];
            continue;
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
        const double e[3] = {(double)ex(a), (double)ey(a), (double)ez(a)};
        const double eou = -(e[0] * u[0] + e[1] * u[1] + e[2] * u[2]);
        // forward post-collision value of this population
        const double eu_f = (e[0] * j[0] + e[1] * j[1] + e[2] * j[2]);
        const double feq = wgt(a) * (drho + 3.0 * eu_f + (4.5 * eu_f * eu_f - 1.5 * jj) / rho);
        const double ft = f[a] + omega * (feq - f[a]);
        const double M = 6.0 * wgt(a) * rho * eou;
        const double s = 2.0 * ft + M;
        double lTxr[3];
        cross3(ab.lT, r, lTxr);
        const double ls = e[0] * (ab.lF[0] + lTxr[0]) + e[1] * (ab.lF[1] + lTxr[1]) + e[2] * (ab.lF[2] + lTxr[2]);
        const double ln = args.lam_next[(size_t)o * stride + cell];
        lt[a] = ln + 2.0 * ls;
        const double lM = ln + ls;
        lrho += 6.0 * wgt(a) * eou * lM;
        const double lu[3] = {-6.0 * wgt(a) * rho * e[0] * lM, -6.0 * wgt(a) * rho * e[1] * lM,
                              -6.0 * wgt(a) * rho * e[2] * lM};
        const int slot = B.link_base[cell] + nlink;
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
    // collision adjoint
    double grho = 0.0, gj[3] = {0, 0, 0};
    for (int a = 0; a < 19; ++a) {
        const double e[3] = {(double)ex(a), (double)ey(a), (double)ez(a)};
        const double ej = e[0] * j[0] + e[1] * j[1] + e[2] * j[2];
        const double w = wgt(a) * lt[a];
        grho += w * (1.0 - (4.5 * ej * ej - 1.5 * jj) / (rho * rho));
        for (int q = 0; q < 3; ++q) gj[q] += w * (3.0 * e[q] + (9.0 * ej * e[q] - 3.0 * j[q]) / rho);
    }
    for (int a = 0; a < 19; ++a) {
        const double egj = ex(a) * gj[0] + ey(a) * gj[1] + ez(a) * gj[2];
        args.lam[(size_t)a * stride + cell] = (1.0 - omega) * lt[a] + omega * (grho + egj) + lrho;
    }
}

// Driving forces of Eqs. FB1-FB3 at step n and their derivatives with
// respect to the amplitude and the phase lag (x components, per body).
__device__ void drive_grad(const BoxDesc &B, long long n, double dFa[kMaxBodies], double dFp[kMaxBodies]) {
    for (int b = 0; b < B.nb; ++b) dFa[b] = dFp[b] = 0.0;
    for (int e = 0; e < B.nd; ++e) {
        const DevDrive &dv = B.drives[e];
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
// step n, spring contributions, and the parameter gradients.
__global__ __launch_bounds__(kCoupleThreads) void adjoint_body_kernel(const BoxDesc *boxes, AdjBody *adj,
                                                                      const BodyHist *hist_np1,
                                                                      const BodyHist *hist_n, const AdjLinkRec *lrec,
                                                                      long long n, int finish, double *grad) {
    __shared__ double wred[kCoupleThreads / 64][9];
    __shared__ double sums[kMaxBodies][9];
    __shared__ int gsum[kMaxBodies][3];
    const BoxDesc &B = boxes[0];
    const int nb = B.nb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (finish) {
        const int L = min(B.link_count, B.link_cap);
        for (int b = 0; b < nb; ++b) {
            double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            int g[3] = {0, 0, 0};
            for (int l = threadIdx.x; l < L; l += kCoupleThreads) {
                if (B.link_body[l] != b) continue;
                const AdjLinkRec rec = lrec[l];
                for (int q = 0; q < 9; ++q) acc[q] += rec.v[q];
                const int a = B.link_dir[l], cw = two_w36(a);
                g[0] += ex(a) * cw;
                g[1] += ey(a) * cw;
                g[2] += ez(a) * cw;
            }
            for (int q = 0; q < 9; ++q) acc[q] = wave_sum(acc[q]);
            for (int q = 0; q < 3; ++q) g[q] = wave_sum_int(g[q]);
            __syncthreads();
            if (lane == 0)
                for (int q = 0; q < 9; ++q) wred[wave][q] = acc[q];
            if (threadIdx.x == 0)
                for (int q = 0; q < 3; ++q) gsum[b][q] = 0;
            __syncthreads();
            if (lane == 0)
                for (int q = 0; q < 3; ++q) atomicAdd(&gsum[b][q], g[q]);  // integers: order-free
            if (threadIdx.x < 9) {
                double t = wred[0][threadIdx.x];
                for (int w = 1; w < kCoupleThreads / 64; ++w) t = t + wred[w][threadIdx.x];
                sums[b][threadIdx.x] = t;
            }
            __syncthreads();
        }
        if ((int)threadIdx.x < nb) {
            const int b = threadIdx.x;
            AdjBody &ab = adj[b];
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
    if (n < 0) return;
    if (threadIdx.x == 0) {
        // begin step n: adjoints of F^n, T^n; springs; parameters
        double dFa[kMaxBodies], dFp[kMaxBodies];
        drive_grad(B, n, dFa, dFp);
        double lF[kMaxBodies][3];
        for (int b = 0; b < nb; ++b) {
            AdjBody &ab = adj[b];
            const DevBody &bd = B.bodies[b];
            for (int q = 0; q < 3; ++q) {
                ab.muV[q] = ab.lV[q] + ab.lD[q];
                lF[b][q] = bd.kinematic == 1 ? 0.0 : ab.muV[q] / bd.mass;
                ab.lF[q] = lF[b][q];
                ab.lDs[q] = ab.lVs[q] = 0.0;
            }
            // T enters Omega' = Omega + R diag(1/I) R^T T: lam_T = R diag(1/I) R^T lam_Omega
            const double w = hist_n[b].q[0], x = hist_n[b].q[1], y = hist_n[b].q[2], z = hist_n[b].q[3];
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
            grad[0] += lF[b][0] * dFa[b];
            grad[1] += lF[b][0] * dFp[b];
        }
        for (int e = 0; e < B.ns; ++e) {
            const DevSpring &sp = B.springs[e];
            const BodyHist &hi = hist_n[sp.i], &hj = hist_n[sp.j];
            const DevBody &bi = B.bodies[sp.i], &bj = B.bodies[sp.j];
            double d[3], lf[3];
            for (int q = 0; q < 3; ++q) {
                d[q] = (bi.anchor[q] - bj.anchor[q]) + (hi.D[q] - hj.D[q]);
                lf[q] = lF[sp.i][q] - lF[sp.j][q];
            }
            const double ell = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double c1 = 1.0 - sp.rest_len / ell, c2 = sp.rest_len / (ell * ell * ell);
            const double dl = d[0] * lf[0] + d[1] * lf[1] + d[2] * lf[2];
            // df/dk = -(ell - l0) d / ell
            grad[2] += -(ell - sp.rest_len) / ell * dl;
            for (int q = 0; q < 3; ++q) {
                const double gD = -sp.k * (c1 * lf[q] + c2 * d[q] * dl);
                adj[sp.i].lDs[q] += gD;
                adj[sp.j].lDs[q] -= gD;
                adj[sp.i].lVs[q] += -sp.gamma * lf[q];
                adj[sp.j].lVs[q] += sp.gamma * lf[q];
            }
        }
    }
    (void)hist_np1;
}

}  // namespace lbm
