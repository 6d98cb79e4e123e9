// gint_device.h -- device helpers shared by the gfx950 kernels: geometry,
// the numerical-atomic-orbital evaluation (PhiOperator role) and small
// search utilities.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "gint_internal.h"

namespace gint {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16x16 matrix-core products on orbital tiles of element type T with 4
// accumulator registers per lane:
//   operands   A[i][k], B[k][j] with i, j = lane & 15, k = lane >> 4
//   result     register v of lane l holds C[row(l >> 4, v)][l & 15]
// (both layouts checked on gfx950 with a lane-layout probe).
template <typename T>
struct MM;
template <>
struct MM<double> {
    typedef d4 acc;
    static __device__ __forceinline__ acc zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc mma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct MM<float> {
    typedef f4 acc;
    static __device__ __forceinline__ acc zero() { return f4{0.0f, 0.0f, 0.0f, 0.0f}; }
    static __device__ __forceinline__ acc mma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

// Make this wave's LDS stores visible to its other lanes' later LDS loads:
// release fence, wave barrier, acquire fence (for exchanges inside one wave
// where some waves of the workgroup may already have exited).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// real spherical harmonics (no Condon-Shortley phase)
#define Y_C00 0.28209479177387814
#define Y_C1 0.4886025119029199
#define Y_C2 1.0925484305920792
#define Y_C20 0.31539156525252005
#define Y_C22 0.5462742152960396

__device__ __forceinline__ void frac_of(const Geo &g, const double *x, double *s)
{
    for (int i = 0; i < 3; ++i)
        s[i] = g.rec[3 * i] * x[0] + g.rec[3 * i + 1] * x[1] + g.rec[3 * i + 2] * x[2];
}

__device__ __forceinline__ void cart_of(const Geo &g, const double *s, double *x)
{
    for (int k = 0; k < 3; ++k)
        x[k] = s[0] * g.lat[k] + s[1] * g.lat[3 + k] + s[2] * g.lat[6 + k];
}

// Batch b -> batch coordinates: tiles of bt[0] x bt[1] x bt[2] batches in
// row-major order, batches row-major inside a tile.
__device__ __forceinline__ void batch_coords(const Geo &g, int b, int *ib)
{
    const int tsz = g.bt[0] * g.bt[1] * g.bt[2];
    const int t = b / tsz, w = b - t * tsz;
    const int m1 = g.nb[1] / g.bt[1], m2 = g.nb[2] / g.bt[2];
    const int t2 = t % m2, t1 = (t / m2) % m1, t0 = t / (m2 * m1);
    const int w2 = w % g.bt[2], w1 = (w / g.bt[2]) % g.bt[1], w0 = w / (g.bt[2] * g.bt[1]);
    ib[0] = t0 * g.bt[0] + w0;
    ib[1] = t1 * g.bt[1] + w1;
    ib[2] = t2 * g.bt[2] + w2;
}

// Batch of workgroup i among n batches starting at b0, XCD-contiguous: XCD x
// (workgroups i = x mod kXcd) takes the x-th contiguous run of batches, so
// the workgroups an XCD runs together share atoms and D blocks in its L2.
// Returns -1 for the padding workgroups of a grid of kXcd * ceil(n / kXcd).
__device__ __forceinline__ int xcd_batch(int i, int b0, int n)
{
    const int run = (n + kXcd - 1) / kXcd;
    const int q = (i % kXcd) * run + i / kXcd;
    return q < n ? b0 + q : -1;
}

// Mesh indices of point q of batch (i0, i1, i2); false outside the mesh.
__device__ __forceinline__ bool batch_point(const Geo &g, const int *ib, int q, int *n)
{
    const int l2 = q % g.bs[2], l1 = (q / g.bs[2]) % g.bs[1], l0 = q / (g.bs[2] * g.bs[1]);
    n[0] = ib[0] * g.bs[0] + l0;
    n[1] = ib[1] * g.bs[1] + l1;
    n[2] = ib[2] * g.bs[2] + l2;
    return q < g.P && n[0] < g.N[0] && n[1] < g.N[1] && n[2] < g.N[2];
}

// r = sum_i n_i a_i / N_i
__device__ __forceinline__ void mesh_cart(const Geo &g, const int *n, double *r)
{
#pragma unroll
    for (int k = 0; k < 3; ++k)
        r[k] = n[0] * g.h[k] + n[1] * g.h[3 + k] + n[2] * g.h[6 + k];
}

// 1/sqrt(x) for x > 0 to full FP64 accuracy: hardware estimate refined by
// two Newton steps.
__device__ __forceinline__ double rsqrt_f64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// First index in [lo, hi) of a[] that is >= key.
__device__ __forceinline__ int lower_bound_i(const int *__restrict__ a, int lo, int hi, int key)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// index of R = (n1, n2, n3) in a caller's list of lattice vectors, -1 if
// absent
__device__ __forceinline__ int hr_lookup(const HRMap &m, int n1, int n2, int n3)
{
    if (n1 < -m.ext[0] || n1 > m.ext[0] || n2 < -m.ext[1] || n2 > m.ext[1] || n3 < -m.ext[2] || n3 > m.ext[2])
        return -1;
    return m.rmap[((n1 + m.ext[0]) * (2 * m.ext[1] + 1) + n2 + m.ext[1]) * (2 * m.ext[2] + 1) + n3 + m.ext[2]];
}

__device__ __forceinline__ void unpack_image(int pk, int *n)
{
    n[0] = (int)(signed char)(pk & 0xff);
    n[1] = (int)(signed char)((pk >> 8) & 0xff);
    n[2] = (int)(signed char)((pk >> 16) & 0xff);
}

// Spline interval and offset for radius rr (left-closed intervals, last
// interval extended to rc).
__device__ __forceinline__ int spline_interval(const DevRadial &R, double rr, double *t)
{
    int iv = (int)(rr * R.inv_dr);
    // the reciprocal can round across a knot: settle on floor(r/dr)
    if (iv * R.dr > rr)
        --iv;
    else if ((iv + 1) * R.dr <= rr)
        ++iv;
    iv = iv > R.nr - 2 ? R.nr - 2 : (iv < 0 ? 0 : iv);
    *t = rr - iv * R.dr;
    return iv;
}

// Folded orbitals of one atom at cartesian point r, for the radials
// k0..k1-1 of its species (radial descriptors in LDS), evaluated in FP64
// and stored as T.  Writes every orbital those radials own: assignment for
// the first listed image, accumulation for further images (several images
// of one atom reach a point only in cells smaller than the cutoff sphere).
// pk0 is the first packed image; further ones are read from img[ioff + i].
// The radial loop is unrolled by U (8: all spline-coefficient loads of an
// image in flight together).  Orbital o goes to row[(o ^ swz) * ST].
template <typename T, int ST = 1, int U = 8>
__device__ __forceinline__ void eval_orbitals(const Geo &g, const DevRadial *__restrict__ rads, int k0, int k1,
                                              double rc, const double *__restrict__ coef, const double *X,
                                              int icnt, int pk0, int ioff, const int *__restrict__ img,
                                              const double *r, T *row, int swz = 0)
{
    const double rc2 = rc * rc;
    for (int i = 0; i < icnt; ++i) {
        const int pk = (i == 0) ? pk0 : img[ioff + i];
        int n[3];
        unpack_image(pk, n);
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            d[k] = r[k] - (X[k] + n[0] * g.lat[k] + n[1] * g.lat[3 + k] + n[2] * g.lat[6 + k]);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const bool inside = r2 < rc2;
        const bool tiny = r2 < kRTiny * kRTiny;
        double ir = 0.0, rr = 0.0;
        if (inside && !tiny) {
            ir = rsqrt_f64(r2);
            rr = r2 * ir;
        }
        const double ux = d[0] * ir, uy = d[1] * ir, uz = d[2] * ir;
        const bool add = i > 0;
        for (int kb = k0; kb < k1; kb += U) {
            double2 c01[U], c23[U];
            double tt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u;
                c01[u] = double2{0.0, 0.0};
                c23[u] = double2{0.0, 0.0};
                tt[u] = 0.0;
                if (k < k1) {
                    const DevRadial R = rads[k];
                    if (inside && rr < R.rc) {
                        const int iv = spline_interval(R, rr, &tt[u]);
                        c01[u] = *reinterpret_cast<const double2 *>(coef + R.coef_off + 4 * iv);
                        c23[u] = *reinterpret_cast<const double2 *>(coef + R.coef_off + 4 * iv + 2);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u;
                if (k >= k1)
                    break;
                const int l = rads[k].l, o = rads[k].orb0;
                const double t = tt[u];
                const double f = c01[u].x + t * (c01[u].y + t * (c23[u].x + t * c23[u].y));
                if (l == 0) {
                    const double v = f * Y_C00;
                    row[(o ^ swz) * ST] = add ? (T)(row[(o ^ swz) * ST] + v) : (T)v;
                } else if (l == 1) {
                    // phi_1m vanishes at the centre (u = 0 there)
                    const double Y[3] = {Y_C1 * uy, Y_C1 * uz, Y_C1 * ux};
#pragma unroll
                    for (int m = 0; m < 3; ++m)
                        row[((o + m) ^ swz) * ST] = add ? (T)(row[((o + m) ^ swz) * ST] + f * Y[m]) : (T)(f * Y[m]);
                } else {
                    // phi_2m vanishes at the centre
                    const double Y[5] = {Y_C2 * ux * uy, Y_C2 * uy * uz, Y_C20 * (2.0 * uz * uz - ux * ux - uy * uy),
                                         Y_C2 * ux * uz, Y_C22 * (ux * ux - uy * uy)};
#pragma unroll
                    for (int m = 0; m < 5; ++m)
                        row[((o + m) ^ swz) * ST] = add ? (T)(row[((o + m) ^ swz) * ST] + f * Y[m]) : (T)(f * Y[m]);
                }
            }
        }
    }
}

// fx += sum_o c_o grad_r phit_o(r) over every orbital of one atom at point r
// (radials k0..k1-1 of its species), summed over the listed images, with
// c_o = wp * crow[o * ST].  One spline evaluation (value and slope) per
// radial serves its 2l+1 orbitals:
//     sum_m c_m grad(f Y_m) = (f' A - l (f/r) A) u + (f/r) G,
//     A = sum_m c_m Y_m(u),  G = sum_m c_m dY_m/du,
// (Y_lm is a homogeneous polynomial of degree l in u, so u . dY/du = l Y).
// At the atom's centre only p orbitals keep a gradient, f'(0) dY/du.
// The radial loop is unrolled by U (spline-coefficient loads in flight
// together).
template <typename T, int ST, int U = 4>
__device__ __forceinline__ void grad_dot_all(const Geo &g, const DevRadial *__restrict__ rads, int k0, int k1,
                                             double rc, const double *__restrict__ coef, const double *X, int icnt,
                                             int pk0, int ioff, const int *__restrict__ img, const double *r,
                                             const T *crow, double wp, double *fx)
{
    const double rc2 = rc * rc;
    for (int i = 0; i < icnt; ++i) {
        const int pk = (i == 0) ? pk0 : img[ioff + i];
        int n[3];
        unpack_image(pk, n);
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            d[k] = r[k] - (X[k] + n[0] * g.lat[k] + n[1] * g.lat[3 + k] + n[2] * g.lat[6 + k]);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(r2 < rc2))
            continue;
        const bool tiny = r2 < kRTiny * kRTiny;
        double ir = 0.0, rr = 0.0;
        if (!tiny) {
            ir = rsqrt_f64(r2);
            rr = r2 * ir;
        }
        const double ux = d[0] * ir, uy = d[1] * ir, uz = d[2] * ir;
        for (int kb = k0; kb < k1; kb += U) {
            double2 c01[U], c23[U];
            double tt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u;
                c01[u] = double2{0.0, 0.0};
                c23[u] = double2{0.0, 0.0};
                tt[u] = 0.0;
                if (k < k1) {
                    const DevRadial R = rads[k];
                    if (rr < R.rc) {
                        const int iv = spline_interval(R, rr, &tt[u]);
                        c01[u] = *reinterpret_cast<const double2 *>(coef + R.coef_off + 4 * iv);
                        c23[u] = *reinterpret_cast<const double2 *>(coef + R.coef_off + 4 * iv + 2);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb + u;
                if (k >= k1)
                    break;
                const int l = rads[k].l, o = rads[k].orb0;
                const double t = tt[u];
                const double f = c01[u].x + t * (c01[u].y + t * (c23[u].x + t * c23[u].y));
                const double fp = c01[u].y + t * (2.0 * c23[u].x + t * 3.0 * c23[u].y);
                double A, G0, G1, G2;
                if (l == 0) {
                    A = Y_C00 * wp * (double)crow[o * ST];
                    G0 = G1 = G2 = 0.0;
                } else if (l == 1) {
                    // m = -1, 0, 1 -> y, z, x
                    const double cy = wp * (double)crow[o * ST], cz = wp * (double)crow[(o + 1) * ST],
                                 cx = wp * (double)crow[(o + 2) * ST];
                    G0 = Y_C1 * cx;
                    G1 = Y_C1 * cy;
                    G2 = Y_C1 * cz;
                    A = G0 * ux + G1 * uy + G2 * uz;
                } else {
                    // m = -2 .. 2 -> xy, yz, 2z^2 - x^2 - y^2, xz, x^2 - y^2
                    const double c0 = wp * (double)crow[o * ST], c1 = wp * (double)crow[(o + 1) * ST],
                                 c2 = wp * (double)crow[(o + 2) * ST], c3 = wp * (double)crow[(o + 3) * ST],
                                 c4 = wp * (double)crow[(o + 4) * ST];
                    G0 = Y_C2 * (c0 * uy + c3 * uz) + ux * (2.0 * Y_C22 * c4 - 2.0 * Y_C20 * c2);
                    G1 = Y_C2 * (c0 * ux + c1 * uz) - uy * (2.0 * Y_C22 * c4 + 2.0 * Y_C20 * c2);
                    G2 = Y_C2 * (c1 * uy + c3 * ux) + uz * (4.0 * Y_C20 * c2);
                    A = 0.5 * (G0 * ux + G1 * uy + G2 * uz);
                }
                if (tiny) {
                    if (l == 1) {
                        fx[0] += fp * G0;
                        fx[1] += fp * G1;
                        fx[2] += fp * G2;
                    }
                    continue;
                }
                const double fr = f * ir;
                const double s = (fp - l * fr) * A;
                fx[0] += s * ux + fr * G0;
                fx[1] += s * uy + fr * G1;
                fx[2] += s * uz + fr * G2;
            }
        }
    }
}

// sum_v wv[v] grad phit_{o_v}(r) for four orbitals o_v = o0 + step v
// (v < 4; zero for o_v >= norb) of one atom at point r, summed over the
// listed images, added to fx.  orb_rad[o] is the radial (index into rads)
// owning orbital o, orb_m[o] its m.  Used where each lane holds exactly the
// orbitals of its MFMA result rows.
__device__ __forceinline__ void grad4_dot(const Geo &g, const DevRadial *__restrict__ rads,
                                          const signed char *__restrict__ orb_rad,
                                          const signed char *__restrict__ orb_m, int norb, double rc,
                                          const double *__restrict__ coef, const double *X, int icnt, int pk0,
                                          int ioff, const int *__restrict__ img, const double *r, int o0, int step,
                                          const double *wv, double *fx)
{
    const double rc2 = rc * rc;
    for (int i = 0; i < icnt; ++i) {
        const int pk = (i == 0) ? pk0 : img[ioff + i];
        int n[3];
        unpack_image(pk, n);
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            d[k] = r[k] - (X[k] + n[0] * g.lat[k] + n[1] * g.lat[3 + k] + n[2] * g.lat[6 + k]);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(r2 < rc2))
            continue;
        const bool tiny = r2 < kRTiny * kRTiny;
        double ir = 0.0, rr = 0.0;
        if (!tiny) {
            ir = rsqrt_f64(r2);
            rr = r2 * ir;
        }
        const double ux = d[0] * ir, uy = d[1] * ir, uz = d[2] * ir;
        // two orbitals at a time (fewer live coefficient registers)
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
        const double wh[2] = {h ? wv[2] : wv[0], h ? wv[3] : wv[1]};
        double2 c01[2], c23[2];
        double tt[2];
        int lv[2], mv[2];
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int o = o0 + step * (2 * h + v);
            c01[v] = double2{0.0, 0.0};
            c23[v] = double2{0.0, 0.0};
            tt[v] = 0.0;
            lv[v] = -1;
            mv[v] = 0;
            if (o < norb) {
                const DevRadial R = rads[orb_rad[o]];
                lv[v] = R.l;
                mv[v] = orb_m[o];
                if (rr < R.rc) {
                    const int iv = spline_interval(R, rr, &tt[v]);
                    c01[v] = *reinterpret_cast<const double2 *>(coef + R.coef_off + 4 * iv);
                    c23[v] = *reinterpret_cast<const double2 *>(coef + R.coef_off + 4 * iv + 2);
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            if (lv[v] < 0)
                continue;
            const double t = tt[v];
            const double f = c01[v].x + t * (c01[v].y + t * (c23[v].x + t * c23[v].y));
            const double fp = c01[v].y + t * (2.0 * c23[v].x + t * 3.0 * c23[v].y);
            const int m = mv[v];
            double Y, G0, G1, G2;
            if (lv[v] == 0) {
                Y = Y_C00;
                G0 = G1 = G2 = 0.0;
            } else if (lv[v] == 1) {
                // m = -1, 0, 1 -> y, z, x
                Y = Y_C1 * (m == -1 ? uy : (m == 0 ? uz : ux));
                G0 = (m == 1) ? Y_C1 : 0.0;
                G1 = (m == -1) ? Y_C1 : 0.0;
                G2 = (m == 0) ? Y_C1 : 0.0;
            } else {
                if (m == -2) {
                    Y = Y_C2 * ux * uy;
                    G0 = Y_C2 * uy;
                    G1 = Y_C2 * ux;
                    G2 = 0.0;
                } else if (m == -1) {
                    Y = Y_C2 * uy * uz;
                    G0 = 0.0;
                    G1 = Y_C2 * uz;
                    G2 = Y_C2 * uy;
                } else if (m == 0) {
                    Y = Y_C20 * (2.0 * uz * uz - ux * ux - uy * uy);
                    G0 = -2.0 * Y_C20 * ux;
                    G1 = -2.0 * Y_C20 * uy;
                    G2 = 4.0 * Y_C20 * uz;
                } else if (m == 1) {
                    Y = Y_C2 * ux * uz;
                    G0 = Y_C2 * uz;
                    G1 = 0.0;
                    G2 = Y_C2 * ux;
                } else {
                    Y = Y_C22 * (ux * ux - uy * uy);
                    G0 = 2.0 * Y_C22 * ux;
                    G1 = -2.0 * Y_C22 * uy;
                    G2 = 0.0;
                }
            }
            if (tiny) {
                // only p orbitals keep a gradient at the centre: f'(0) C1 e_m
                if (lv[v] == 1) {
                    fx[0] += wh[v] * (fp * G0);
                    fx[1] += wh[v] * (fp * G1);
                    fx[2] += wh[v] * (fp * G2);
                }
                continue;
            }
            const double fr = f * ir;
            const double lY = lv[v] * Y;
            fx[0] += wh[v] * (fp * Y * ux + fr * (G0 - lY * ux));
            fx[1] += wh[v] * (fp * Y * uy + fr * (G1 - lY * uy));
            fx[2] += wh[v] * (fp * Y * uz + fr * (G2 - lY * uz));
        }
        }
    }
}

}  // namespace gint
