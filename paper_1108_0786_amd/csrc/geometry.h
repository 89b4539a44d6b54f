// Body geometry on the lattice (Sec. 2.3): lever arms from a body to a cell
// centre, the inside test of the object mapping, and the body's velocity at a
// cell.  Every expression is evaluated in a fixed float64 sequence without
// fused multiply-add, so that the inside/outside decision of a cell is
// reproducible bit for bit by any implementation of the same sequence.
#pragma once
#include "common.h"

namespace lbm {

__device__ __forceinline__ int wrap_centered(int d, int L) {
    // d wrapped into [-L/2, L - L/2)
    int h = L / 2;
    int m = (d + h) % L;
    if (m < 0) m += L;
    return m - h;
}

// r = (d + 1/2) - f, with R = floor(X), f = X - R, d = cell - R (wrapped on
// periodic axes); also returns the integer offsets d.
// X: the body position, anchor + D, per axis.
__device__ __forceinline__ void lever_arm_at(const double X3[3], int i, int j, int k, int nx, int ny, int nz,
                                             int per, double r[3], int d[3]) {
#pragma clang fp contract(off)
    const int idx[3] = {i, j, k};
    const int n[3] = {nx, ny, nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double X = X3[a];
        double R = floor(X);
        double f = X - R;
        // R is converted through a clamp so that a non-finite or huge position
        // cannot produce an undefined conversion (such a body maps to nothing)
        int di = idx[a] - (int)fmin(fmax(R, -1073741824.0), 1073741824.0);
        if (per & (1 << a)) di = wrap_centered(di, n[a]);
        d[a] = di;
        r[a] = ((double)di + 0.5) - f;
    }
}

__device__ __forceinline__ void lever_arm(const DevBody &b, int i, int j, int k, int nx, int ny,
                                          int nz, int per, double r[3], int d[3]) {
#pragma clang fp contract(off)
    const double X[3] = {b.anchor[0] + b.D[0], b.anchor[1] + b.D[1], b.anchor[2] + b.D[2]};
    lever_arm_at(X, i, j, k, nx, ny, nz, per, r, d);
}

__device__ __forceinline__ void body_axis(const DevBody &b, double a[3]) {
#pragma clang fp contract(off)
    const double qw = b.q[0], qx = b.q[1], qy = b.q[2], qz = b.q[3];
    a[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    a[1] = 2.0 * (qx * qy + qw * qz);
    a[2] = 2.0 * (qx * qz - qw * qy);
}

// Squared distance from the body's core (centre point or axis segment).
__device__ __forceinline__ double core_dist2(const DevBody &b, const double r[3]) {
#pragma clang fp contract(off)
    if (b.shape == kBodyShapeSphere) return (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    double a[3];
    body_axis(b, a);
    double t = (r[0] * a[0] + r[1] * a[1]) + r[2] * a[2];
    const double h = b.half_len;
    t = fmin(fmax(t, -h), h);
    double sx = r[0] - t * a[0];
    double sy = r[1] - t * a[1];
    double sz = r[2] - t * a[2];
    return (sx * sx + sy * sy) + sz * sz;
}

// Signed distance along the body's x axis (the slab's normal).
__device__ __forceinline__ double axial(const DevBody &b, const double r[3]) {
#pragma clang fp contract(off)
    double a[3];
    body_axis(b, a);
    return (r[0] * a[0] + r[1] * a[1]) + r[2] * a[2];
}

__device__ __forceinline__ bool inside(const DevBody &b, const double r[3]) {
#pragma clang fp contract(off)
    if (b.shape == kBodyShapeSlab) return axial(b, r) > 0.0;
    return core_dist2(b, r) <= b.radius * b.radius;
}

// Distance of a point from the body's surface (the margin of the remap skip).
__device__ __forceinline__ double surface_dist(const DevBody &b, const double r[3]) {
    if (b.shape == kBodyShapeSlab) return fabs(axial(b, r));
    return fabs(sqrt(core_dist2(b, r)) - b.radius);
}

// u_w = V + Omega x r
__device__ __forceinline__ void wall_velocity(const DevBody &b, const double r[3], double u[3]) {
#pragma clang fp contract(off)
    u[0] = b.V[0] + (b.O[1] * r[2] - b.O[2] * r[1]);
    u[1] = b.V[1] + (b.O[2] * r[0] - b.O[0] * r[2]);
    u[2] = b.V[2] + (b.O[0] * r[1] - b.O[1] * r[0]);
}

__device__ __forceinline__ void decode_cell(int c, int nx, int ny, int &i, int &j, int &k) {
    i = c % nx;
    int t = c / nx;
    j = t % ny;
    k = t / ny;
}

// Neighbour of (i,j,k) in direction a; false if it lies beyond a wall.
template <int A>
__device__ __forceinline__ bool neighbour(int i, int j, int k, int nx, int ny, int nz, int per,
                                          int &ti, int &tj, int &tk) {
    ti = i + ex(A);
    tj = j + ey(A);
    tk = k + ez(A);
    if (ex(A) != 0 && (ti < 0 || ti >= nx)) {
        if (!(per & 1)) return false;
        ti = ti < 0 ? ti + nx : ti - nx;
    }
    if (ey(A) != 0 && (tj < 0 || tj >= ny)) {
        if (!(per & 2)) return false;
        tj = tj < 0 ? tj + ny : tj - ny;
    }
    if (ez(A) != 0 && (tk < 0 || tk >= nz)) {
        if (!(per & 4)) return false;
        tk = tk < 0 ? tk + nz : tk - nz;
    }
    return true;
}

__device__ __forceinline__ bool neighbour_rt(int a, int i, int j, int k, int nx, int ny, int nz,
                                             int per, int &ti, int &tj, int &tk) {
    ti = i + ex(a);
    tj = j + ey(a);
    tk = k + ez(a);
    if (ti < 0 || ti >= nx) {
        if (!(per & 1)) return false;
        ti = ti < 0 ? ti + nx : ti - nx;
    }
    if (tj < 0 || tj >= ny) {
        if (!(per & 2)) return false;
        tj = tj < 0 ? tj + ny : tj - ny;
    }
    if (tk < 0 || tk >= nz) {
        if (!(per & 4)) return false;
        tk = tk < 0 ? tk + nz : tk - nz;
    }
    return true;
}

}  // namespace lbm
