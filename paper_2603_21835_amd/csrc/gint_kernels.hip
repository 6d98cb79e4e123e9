// gint_kernels.hip -- gfx950 kernels of the real-space grid integration.
//
// Pipeline (Fig. 2 of arXiv:2603.21835: GintInfo -> loop over mesh blocks ->
// PhiOperator -> calculation kernels -> aggregation -> target format):
//
//   spline       clamped cubic spline coefficients of every radial (FP64)
//   wrap/sort    wrap atoms into the cell; order them along a Morton curve
//                and cut the order into groups of 4 spatially close atoms
//   bin          mesh batches x (atom, lattice image) lists (GintInfo/BigGrid)
//   pairs_*      output-stationary contractions: one workgroup owns a pair of
//                atom groups (a 4x4 tile of 16x16 atom-pair blocks) and
//                streams the batches both groups reach; per batch it evaluates
//                the folded orbitals of its <= 8 atoms into LDS (PhiOperator)
//                and runs v_mfma_f64_16x16x4 on them (H^loc, rho, force of
//                Sec. 3.3.1)
//   reductions   fixed-order FP64 sums over chunks / group pairs, then the
//                dense output layouts (conversion to the target format)
#include <hip/hip_runtime.h>

#include <climits>

#include "gint_internal.h"

namespace gint {

typedef double d4 __attribute__((ext_vector_type(4)));

// real spherical harmonics (no Condon-Shortley phase)
#define Y_C00 0.28209479177387814
#define Y_C1 0.4886025119029199
#define Y_C2 1.0925484305920792
#define Y_C20 0.31539156525252005
#define Y_C22 0.5462742152960396

// ---------------------------------------------------------------------------
// Clamped cubic spline, Hermite form: unknown knot slopes k_i with
// k_0 = s0, k_{n-1} = sn and k_{i-1} + 4 k_i + k_{i+1} = 3 (y_{i+1} - y_{i-1})/h,
// solved by the Thomas algorithm; then per interval
// f(t) = y_i + k_i t + c t^2 + d t^3.  One thread per radial.

__global__ void k_spline(int nrad, const DevRadial *__restrict__ rad, const double *__restrict__ knots,
                         const double *__restrict__ s0, const double *__restrict__ sn,
                         double *__restrict__ coef, double *__restrict__ scratch)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrad)
        return;
    const DevRadial R = rad[k];
    const int n = R.nr;
    const double h = R.dr;
    const double *y = knots + R.knot_off;
    double *cp = scratch + 3 * (size_t)R.knot_off;
    double *dp = cp + n;
    double *ks = dp + n;
    for (int i = 1; i <= n - 2; ++i) {
        double rhs = 3.0 * (y[i + 1] - y[i - 1]) / h;
        if (i == 1)
            rhs -= s0[k];
        if (i == n - 2)
            rhs -= sn[k];
        if (i == 1) {
            cp[i] = 0.25;
            dp[i] = rhs * 0.25;
        } else {
            const double den = 4.0 - cp[i - 1];
            cp[i] = 1.0 / den;
            dp[i] = (rhs - dp[i - 1]) / den;
        }
    }
    ks[0] = s0[k];
    ks[n - 1] = sn[k];
    ks[n - 2] = dp[n - 2];
    for (int i = n - 3; i >= 1; --i)
        ks[i] = dp[i] - cp[i] * ks[i + 1];
    double *c = coef + R.coef_off;
    for (int i = 0; i < n - 1; ++i) {
        const double del = (y[i + 1] - y[i]) / h;
        c[4 * i + 0] = y[i];
        c[4 * i + 1] = ks[i];
        c[4 * i + 2] = (3.0 * del - 2.0 * ks[i] - ks[i + 1]) / h;
        c[4 * i + 3] = (ks[i] + ks[i + 1] - 2.0 * del) / (h * h);
    }
}

hipError_t launch_spline(hipStream_t s, int nrad, const DevRadial *rad, const double *knots,
                         const double *s0, const double *sn, double *coef, double *scratch)
{
    hipLaunchKernelGGL(k_spline, dim3((nrad + 63) / 64), dim3(64), 0, s, nrad, rad, knots, s0, sn, coef,
                       scratch);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Geometry helpers

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

__device__ __forceinline__ unsigned int spread10(unsigned int v)
{
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

// Wrap positions into [0,1)^3 fractional; Morton key of the wrapped point.
__global__ void k_wrap(Geo g, const double *__restrict__ pos_in, double *__restrict__ xw_in,
                       unsigned long long *__restrict__ keys)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.natom)
        return;
    double x[3] = {pos_in[3 * i], pos_in[3 * i + 1], pos_in[3 * i + 2]};
    double s[3];
    frac_of(g, x, s);
    unsigned int q[3];
    for (int k = 0; k < 3; ++k) {
        s[k] -= floor(s[k]);
        if (!(s[k] < 1.0) || !(s[k] >= 0.0))
            s[k] = 0.0;
        int qi = (int)(s[k] * 1024.0);
        q[k] = (unsigned int)(qi < 0 ? 0 : (qi > 1023 ? 1023 : qi));
    }
    double w[3];
    cart_of(g, s, w);
    xw_in[3 * i] = w[0];
    xw_in[3 * i + 1] = w[1];
    xw_in[3 * i + 2] = w[2];
    if (keys) {
        const unsigned long long m = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
        keys[i] = (m << 32) | (unsigned long long)i;
    }
}

hipError_t launch_wrap(hipStream_t s, const Geo &g, const double *pos_in, double *xw_in,
                       unsigned long long *keys)
{
    hipLaunchKernelGGL(k_wrap, dim3((g.natom + 255) / 256), dim3(256), 0, s, g, pos_in, xw_in, keys);
    return hipGetLastError();
}

// Bitonic sort of n (power of two) keys in global memory, one stage per launch.
__global__ void k_bitonic_stage(unsigned long long *__restrict__ a, int n, int k, int j)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int l = i ^ j;
    if (l > i) {
        const unsigned long long x = a[i], y = a[l];
        const bool up = (i & k) == 0;
        if ((x > y) == up) {
            a[i] = y;
            a[l] = x;
        }
    }
}

__global__ void k_perm_from_keys(int natom, const unsigned long long *__restrict__ keys, int *__restrict__ perm,
                                 int *__restrict__ inv_perm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natom)
        return;
    const int p = (int)(keys[i] & 0xffffffffull);
    perm[i] = p;
    inv_perm[p] = i;
}

// keys must hold a power-of-two capacity >= natom; the tail is padded here.
__global__ void k_pad_keys(unsigned long long *a, int natom, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natom && i < n)
        a[i] = ULLONG_MAX;
}

hipError_t launch_sort_perm(hipStream_t s, int natom, unsigned long long *keys, int *perm, int *inv_perm)
{
    int n = 1;
    while (n < natom)
        n <<= 1;
    const int nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_pad_keys, dim3(nb), dim3(256), 0, s, keys, natom, n);
    for (int k = 2; k <= n; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_stage, dim3(nb), dim3(256), 0, s, keys, n, k, j);
    hipLaunchKernelGGL(k_perm_from_keys, dim3((natom + 255) / 256), dim3(256), 0, s, natom, keys, perm,
                       inv_perm);
    return hipGetLastError();
}

__global__ void k_gather_internal(int natom, const int *__restrict__ perm, const double *__restrict__ xw_in,
                                  const int *__restrict__ spc_in, double *__restrict__ xw, int *__restrict__ spc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= natom)
        return;
    const int p = perm[i];
    xw[3 * i] = xw_in[3 * p];
    xw[3 * i + 1] = xw_in[3 * p + 1];
    xw[3 * i + 2] = xw_in[3 * p + 2];
    spc[i] = spc_in[p];
}

hipError_t launch_gather_internal(hipStream_t s, int natom, const int *perm, const double *xw_in,
                                  const int *spc_in, double *xw, int *spc)
{
    hipLaunchKernelGGL(k_gather_internal, dim3((natom + 255) / 256), dim3(256), 0, s, natom, perm, xw_in,
                       spc_in, xw, spc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Binning (GintInfo / BigGrid): for every batch, the atoms with at least one
// lattice image whose cutoff sphere reaches the batch's points, and those
// images.  Conservative: exact box test for axis-aligned cells, a bounding
// sphere of the batch's point parallelepiped otherwise.  Entries are in
// increasing internal atom order, images in (n1, n2, n3) loop order.

__device__ __forceinline__ void batch_coords(const Geo &g, int b, int *ib)
{
    ib[2] = b % g.nb[2];
    ib[1] = (b / g.nb[2]) % g.nb[1];
    ib[0] = b / (g.nb[2] * g.nb[1]);
}

template <bool FILL>
__device__ void bin_one_batch(const Geo &g, const Basis &bs, int b, int *ne, int *ni, int *ng, int *ent_atom,
                              int *ent_img, int *img, int *bgrp, int e0, int i0, int g0)
{
    int ib[3];
    batch_coords(g, b, ib);
    // fractional extent of the batch's points along each axis
    double slo[3], shi[3];
    for (int k = 0; k < 3; ++k) {
        const int n0 = ib[k] * g.bs[k];
        int n1 = n0 + g.bs[k] - 1;
        if (n1 > g.N[k] - 1)
            n1 = g.N[k] - 1;
        slo[k] = (double)n0 / g.N[k];
        shi[k] = (double)n1 / g.N[k];
    }
    double sc[3] = {0.5 * (slo[0] + shi[0]), 0.5 * (slo[1] + shi[1]), 0.5 * (slo[2] + shi[2])};
    double c[3];
    cart_of(g, sc, c);
    // bounding radius of the point parallelepiped around its centre
    double rad = 0.0;
    for (int m = 0; m < 8; ++m) {
        double sd[3] = {((m & 1) ? 0.5 : -0.5) * (shi[0] - slo[0]), ((m & 2) ? 0.5 : -0.5) * (shi[1] - slo[1]),
                        ((m & 4) ? 0.5 : -0.5) * (shi[2] - slo[2])};
        double xd[3];
        cart_of(g, sd, xd);
        const double r = sqrt(xd[0] * xd[0] + xd[1] * xd[1] + xd[2] * xd[2]);
        rad = r > rad ? r : rad;
    }
    double blo[3], bhi[3];
    if (g.ortho) {
        for (int k = 0; k < 3; ++k) {
            blo[k] = slo[k] * g.lat[4 * k];
            bhi[k] = shi[k] * g.lat[4 * k];
            if (blo[k] > bhi[k]) {
                const double t = blo[k];
                blo[k] = bhi[k];
                bhi[k] = t;
            }
        }
    }
    double bn[3];
    for (int i = 0; i < 3; ++i)
        bn[i] = sqrt(g.rec[3 * i] * g.rec[3 * i] + g.rec[3 * i + 1] * g.rec[3 * i + 1] +
                     g.rec[3 * i + 2] * g.rec[3 * i + 2]);
    int cnt_e = 0, cnt_i = 0, cnt_g = 0, last_grp = -1;
    for (int a = 0; a < g.natom; ++a) {
        const double rc = bs.sp[bs.spc[a]].rc;
        const double reach = rc + rad + 1e-9;
        const double *X = bs.xw + 3 * a;
        const double dx[3] = {c[0] - X[0], c[1] - X[1], c[2] - X[2]};
        double ds[3];
        frac_of(g, dx, ds);
        int lo[3], hi[3];
        bool empty = false;
        for (int i = 0; i < 3; ++i) {
            lo[i] = (int)ceil(ds[i] - reach * bn[i]);
            hi[i] = (int)floor(ds[i] + reach * bn[i]);
            empty |= lo[i] > hi[i];
        }
        if (empty)
            continue;
        int nimg = 0;
        for (int n0 = lo[0]; n0 <= hi[0]; ++n0)
            for (int n1 = lo[1]; n1 <= hi[1]; ++n1)
                for (int n2 = lo[2]; n2 <= hi[2]; ++n2) {
                    double p[3];
                    for (int k = 0; k < 3; ++k)
                        p[k] = X[k] + n0 * g.lat[k] + n1 * g.lat[3 + k] + n2 * g.lat[6 + k];
                    bool hit;
                    if (g.ortho) {
                        double d2 = 0.0;
                        for (int k = 0; k < 3; ++k) {
                            double e = 0.0;
                            if (p[k] < blo[k])
                                e = blo[k] - p[k];
                            else if (p[k] > bhi[k])
                                e = p[k] - bhi[k];
                            d2 += e * e;
                        }
                        hit = d2 < (rc + 1e-9) * (rc + 1e-9);
                    } else {
                        const double e0 = p[0] - c[0], e1 = p[1] - c[1], e2 = p[2] - c[2];
                        hit = e0 * e0 + e1 * e1 + e2 * e2 < reach * reach;
                    }
                    if (!hit)
                        continue;
                    if (FILL)
                        img[i0 + cnt_i] = (int)(((unsigned)(n0 & 0xff)) | ((unsigned)(n1 & 0xff) << 8) |
                                                ((unsigned)(n2 & 0xff) << 16));
                    ++cnt_i;
                    ++nimg;
                }
        if (nimg == 0)
            continue;
        if (FILL) {
            ent_atom[e0 + cnt_e] = a;
            ent_img[e0 + cnt_e] = i0 + cnt_i - nimg;
        }
        ++cnt_e;
        const int grp = a / kGroup;
        if (grp != last_grp) {
            if (FILL)
                bgrp[g0 + cnt_g] = grp;
            ++cnt_g;
            last_grp = grp;
        }
    }
    *ne = cnt_e;
    *ni = cnt_i;
    *ng = cnt_g;
}

__global__ void k_bin_count(Geo g, Basis bs, int *__restrict__ cnt_e, int *__restrict__ cnt_i,
                            int *__restrict__ cnt_g, long long *__restrict__ cnt_s)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.nbatch)
        return;
    int ne, ni, ng;
    bin_one_batch<false>(g, bs, b, &ne, &ni, &ng, nullptr, nullptr, nullptr, nullptr, 0, 0, 0);
    cnt_e[b] = ne;
    cnt_i[b] = ni;
    cnt_g[b] = ng;
    cnt_s[b] = (long long)ng * (ng + 1) / 2;
}

hipError_t launch_bin_count(hipStream_t s, const Geo &g, const Basis &b, int *cnt_e, int *cnt_i, int *cnt_g,
                            long long *cnt_s)
{
    hipLaunchKernelGGL(k_bin_count, dim3((g.nbatch + 127) / 128), dim3(128), 0, s, g, b, cnt_e, cnt_i, cnt_g,
                       cnt_s);
    return hipGetLastError();
}

__global__ void k_bin_fill(Geo g, Basis bs, const int *__restrict__ bptr, const int *__restrict__ iptr,
                           const int *__restrict__ bgptr, int *__restrict__ ent_atom, int *__restrict__ ent_img,
                           int *__restrict__ img, int *__restrict__ bgrp)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.nbatch)
        return;
    int ne, ni, ng;
    bin_one_batch<true>(g, bs, b, &ne, &ni, &ng, ent_atom, ent_img, img, bgrp, bptr[b], iptr[b], bgptr[b]);
    if (b == g.nbatch - 1)
        ent_img[bptr[b] + ne] = iptr[b] + ni;  // closing offset
}

hipError_t launch_bin_fill(hipStream_t s, const Geo &g, const Basis &b, const int *bptr, const int *iptr,
                           const int *bgptr, int *ent_atom, int *ent_img, int *img, int *bgrp)
{
    hipLaunchKernelGGL(k_bin_fill, dim3((g.nbatch + 127) / 128), dim3(128), 0, s, g, b, bptr, iptr, bgptr,
                       ent_atom, ent_img, img, bgrp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive scan, one workgroup: out[i] = sum_{j<i} in[j], out[n] = total.

template <typename T>
__global__ __launch_bounds__(1024) void k_scan(const T *__restrict__ in, long long n, T *__restrict__ out)
{
    __shared__ T part[1024];
    const int t = threadIdx.x;
    const long long per = (n + 1023) / 1024;
    const long long lo = t * per;
    const long long hi = (lo + per < n) ? lo + per : n;
    T s = 0;
    for (long long i = lo; i < hi; ++i)
        s += in[i];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        T v = (t >= off) ? part[t - off] : (T)0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    T run = (t == 0) ? (T)0 : part[t - 1];
    for (long long i = lo; i < hi; ++i) {
        const T v = in[i];
        out[i] = run;
        run += v;
    }
    if (t == 1023)
        out[n] = part[1023];
}

hipError_t launch_scan_i32(hipStream_t s, const int *in, long long n, int *out)
{
    hipLaunchKernelGGL(k_scan<int>, dim3(1), dim3(1024), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_scan_i64(hipStream_t s, const long long *in, long long n, long long *out)
{
    hipLaunchKernelGGL(k_scan<long long>, dim3(1), dim3(1024), 0, s, in, n, out);
    return hipGetLastError();
}

__global__ void k_fill_i32(int *p, long long n, int v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

hipError_t launch_fill_i32(hipStream_t s, int *p, long long n, int v)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-group batch lists (in increasing batch order), one workgroup per group.

__device__ __forceinline__ bool batch_has_group(const int *bgptr, const int *bgrp, int b, int grp)
{
    int lo = bgptr[b], hi = bgptr[b + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int v = bgrp[mid];
        if (v == grp)
            return true;
        if (v < grp)
            lo = mid + 1;
        else
            hi = mid;
    }
    return false;
}

__global__ __launch_bounds__(256) void k_group_count(Geo g, const int *__restrict__ bgptr,
                                                     const int *__restrict__ bgrp, int *__restrict__ gcnt)
{
    __shared__ int red[256];
    const int grp = blockIdx.x;
    int c = 0;
    for (int b = threadIdx.x; b < g.nbatch; b += 256)
        c += batch_has_group(bgptr, bgrp, b, grp) ? 1 : 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        gcnt[grp] = red[0];
}

hipError_t launch_group_count(hipStream_t s, const Geo &g, const int *bgptr, const int *bgrp, int *gcnt)
{
    hipLaunchKernelGGL(k_group_count, dim3(g.ngroup), dim3(256), 0, s, g, bgptr, bgrp, gcnt);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_group_fill(Geo g, const int *__restrict__ bgptr,
                                                    const int *__restrict__ bgrp, const int *__restrict__ gptr,
                                                    int *__restrict__ gbatch)
{
    __shared__ int wcnt[4];
    const int grp = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int run = gptr[grp];
    for (int base = 0; base < g.nbatch; base += 256) {
        const int b = base + threadIdx.x;
        const bool keep = (b < g.nbatch) && batch_has_group(bgptr, bgrp, b, grp);
        const unsigned long long m = __ballot(keep);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0)
            wcnt[wave] = __popcll(m);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; ++w)
            off += wcnt[w];
        if (keep)
            gbatch[run + off + pre] = b;
        run += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
}

hipError_t launch_group_fill(hipStream_t s, const Geo &g, const int *bgptr, const int *bgrp, const int *gptr,
                             int *gbatch)
{
    hipLaunchKernelGGL(k_group_fill, dim3(g.ngroup), dim3(256), 0, s, g, bgptr, bgrp, gptr, gbatch);
    return hipGetLastError();
}

// Group pairs (A <= B) that share at least one batch.
__global__ void k_pair_mark(Geo g, const int *__restrict__ bgptr, const int *__restrict__ bgrp, int *mark)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.nbatch)
        return;
    const int lo = bgptr[b], hi = bgptr[b + 1];
    for (int i = lo; i < hi; ++i)
        for (int j = i; j < hi; ++j)
            mark[(size_t)bgrp[i] * g.ngroup + bgrp[j]] = 1;
}

hipError_t launch_pair_mark(hipStream_t s, const Geo &g, const int *bgptr, const int *bgrp, int *mark)
{
    hipLaunchKernelGGL(k_pair_mark, dim3((g.nbatch + 255) / 256), dim3(256), 0, s, g, bgptr, bgrp, mark);
    return hipGetLastError();
}

__global__ void k_pair_list(int ngroup, const int *__restrict__ mark, const int *__restrict__ mscan,
                            int *__restrict__ pair_index, int *__restrict__ pairA, int *__restrict__ pairB)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)ngroup * ngroup)
        return;
    if (mark[i]) {
        const int p = mscan[i];
        pair_index[i] = p;
        pairA[p] = (int)(i / ngroup);
        pairB[p] = (int)(i % ngroup);
    } else {
        pair_index[i] = -1;
    }
}

hipError_t launch_pair_list(hipStream_t s, int ngroup, const int *mark, const int *mark_scan, int *pair_index,
                            int *pairA, int *pairB)
{
    const long long n = (long long)ngroup * ngroup;
    hipLaunchKernelGGL(k_pair_list, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ngroup, mark, mark_scan,
                       pair_index, pairA, pairB);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Orbital evaluation (PhiOperator).  The folded orbitals of one atom at one
// mesh point, accumulated over the atom's listed images into a 16-slot LDS
// row (and, with GRAD, three gradient rows).  Angular part: closed-form real
// Y_lm and their analytic tangential gradients; radial part: the spline and
// its derivative.

__device__ __forceinline__ void mesh_point(const Geo &g, int b, int q, double *r, int *gidx)
{
    int ib[3];
    batch_coords(g, b, ib);
    const int l2 = q % g.bs[2];
    const int l1 = (q / g.bs[2]) % g.bs[1];
    const int l0 = q / (g.bs[2] * g.bs[1]);
    const int n0 = ib[0] * g.bs[0] + l0, n1 = ib[1] * g.bs[1] + l1, n2 = ib[2] * g.bs[2] + l2;
    if (q >= g.P || n0 >= g.N[0] || n1 >= g.N[1] || n2 >= g.N[2]) {
        *gidx = -1;
        return;
    }
    *gidx = (n0 * g.N[1] + n1) * g.N[2] + n2;
    const double s[3] = {(double)n0 / g.N[0], (double)n1 / g.N[1], (double)n2 / g.N[2]};
    cart_of(g, s, r);
}

template <bool GRAD>
__device__ void eval_atom(const Geo &g, const Basis &bs, int e, const int *__restrict__ ent_atom,
                          const int *__restrict__ ent_img, const int *__restrict__ img, const double *r,
                          double *row, double *gx, double *gy, double *gz)
{
    const int a = ent_atom[e];
    const DevSpecies S = bs.sp[bs.spc[a]];
    const double X[3] = {bs.xw[3 * a], bs.xw[3 * a + 1], bs.xw[3 * a + 2]};
    const int i1 = ent_img[e + 1];
    for (int im = ent_img[e]; im < i1; ++im) {
        const int pk = img[im];
        const int n0 = (int)(signed char)(pk & 0xff), n1 = (int)(signed char)((pk >> 8) & 0xff),
                  n2 = (int)(signed char)((pk >> 16) & 0xff);
        double d[3];
        for (int k = 0; k < 3; ++k)
            d[k] = r[k] - (X[k] + n0 * g.lat[k] + n1 * g.lat[3 + k] + n2 * g.lat[6 + k]);
        const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(rr < S.rc))
            continue;
        const bool tiny = rr < kRTiny;
        const double ir = tiny ? 0.0 : 1.0 / rr;
        const double ux = d[0] * ir, uy = d[1] * ir, uz = d[2] * ir;
        for (int k = S.rad0; k < S.rad0 + S.nrad; ++k) {
            const DevRadial R = bs.rad[k];
            if (!(rr < R.rc))
                continue;
            int iv = (int)(rr * R.inv_dr);
            // the reciprocal can round across a knot: settle on floor(r/dr)
            if (iv * R.dr > rr)
                --iv;
            else if ((iv + 1) * R.dr <= rr)
                ++iv;
            if (iv > R.nr - 2)
                iv = R.nr - 2;
            if (iv < 0)
                iv = 0;
            const double t = rr - iv * R.dr;
            const double2 c01 = *reinterpret_cast<const double2 *>(bs.coef + R.coef_off + 4 * iv);
            const double2 c23 = *reinterpret_cast<const double2 *>(bs.coef + R.coef_off + 4 * iv + 2);
            const double f = c01.x + t * (c01.y + t * (c23.x + t * c23.y));
            const double fp = c01.y + t * (2.0 * c23.x + t * 3.0 * c23.y);
            const int o = R.orb0;
            if (R.l == 0) {
                row[o] += f * Y_C00;
                if (GRAD && !tiny) {
                    const double q = fp * Y_C00;
                    gx[o] += q * ux;
                    gy[o] += q * uy;
                    gz[o] += q * uz;
                }
            } else if (R.l == 1) {
                if (tiny) {
                    // phi_1m -> 0, grad phi_1m -> f'(0) C1 e_m, e = (y, z, x)
                    if (GRAD) {
                        gy[o + 0] += fp * Y_C1;
                        gz[o + 1] += fp * Y_C1;
                        gx[o + 2] += fp * Y_C1;
                    }
                    continue;
                }
                const double Y[3] = {Y_C1 * uy, Y_C1 * uz, Y_C1 * ux};
                row[o + 0] += f * Y[0];
                row[o + 1] += f * Y[1];
                row[o + 2] += f * Y[2];
                if (GRAD) {
                    const double fr = f * ir;
                    // grad Y(d/|d|) = (grad_u Yhat - l Yhat u)/|d|
                    const double G[3][3] = {{0.0, Y_C1, 0.0}, {0.0, 0.0, Y_C1}, {Y_C1, 0.0, 0.0}};
                    for (int m = 0; m < 3; ++m) {
                        gx[o + m] += fp * Y[m] * ux + fr * (G[m][0] - Y[m] * ux);
                        gy[o + m] += fp * Y[m] * uy + fr * (G[m][1] - Y[m] * uy);
                        gz[o + m] += fp * Y[m] * uz + fr * (G[m][2] - Y[m] * uz);
                    }
                }
            } else {
                if (tiny)
                    continue;  // phi_2m and its gradient vanish at the centre
                const double Y[5] = {Y_C2 * ux * uy, Y_C2 * uy * uz, Y_C20 * (2.0 * uz * uz - ux * ux - uy * uy),
                                     Y_C2 * ux * uz, Y_C22 * (ux * ux - uy * uy)};
                for (int m = 0; m < 5; ++m)
                    row[o + m] += f * Y[m];
                if (GRAD) {
                    const double fr = f * ir;
                    const double G[5][3] = {{Y_C2 * uy, Y_C2 * ux, 0.0},
                                            {0.0, Y_C2 * uz, Y_C2 * uy},
                                            {-2.0 * Y_C20 * ux, -2.0 * Y_C20 * uy, 4.0 * Y_C20 * uz},
                                            {Y_C2 * uz, 0.0, Y_C2 * ux},
                                            {2.0 * Y_C22 * ux, -2.0 * Y_C22 * uy, 0.0}};
                    for (int m = 0; m < 5; ++m) {
                        gx[o + m] += fp * Y[m] * ux + fr * (G[m][0] - 2.0 * Y[m] * ux);
                        gy[o + m] += fp * Y[m] * uy + fr * (G[m][1] - 2.0 * Y[m] * uy);
                        gz[o + m] += fp * Y[m] * uz + fr * (G[m][2] - 2.0 * Y[m] * uz);
                    }
                }
            }
        }
    }
}

// Entry of internal atom `atom` in batch b, or -1.
__device__ __forceinline__ int find_entry(const Bins &bn, int b, int atom)
{
    int lo = bn.bptr[b], hi = bn.bptr[b + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int v = bn.ent_atom[mid];
        if (v == atom)
            return mid;
        if (v < atom)
            lo = mid + 1;
        else
            hi = mid;
    }
    return -1;
}

// Rank of group g in batch b's sorted group list.
__device__ __forceinline__ int group_rank(const Bins &bn, int b, int grp)
{
    int lo = bn.bgptr[b], hi = bn.bgptr[b + 1];
    const int base = lo;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (bn.bgrp[mid] < grp)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo - base;
}

// ---------------------------------------------------------------------------
// Group-pair contractions.
//
// Workgroup = (group pair (A, B), chunk of A's batch list); 4 waves.  Wave w
// owns the row atom I = 4A + w and the blocks (I, J = 4B + j), j = 0..3 (for
// A == B only j >= w).  Per batch the workgroup stages the folded orbitals of
// the <= 8 atoms of A and B at the batch's points into LDS as
// s_phi[slot][point][orbital] (row pitch kRow doubles), then each wave runs
// its blocks on v_mfma_f64_16x16x4:
//
//   operand lane layout (lane l):  A[i][k], B[k][j] with i, j = l & 15, k = l >> 4
//   result lane layout:            C[i][j] with i = (l >> 4) + 4 v, j = l & 15, v < 4
//                                  (checked on gfx950 with a lane-layout probe)
//
//   H     C_IJ += (w phi_I)^T phi_J over the batch points         (16x16 per block)
//   rho   u = S'_IJ phi_J^T, rho_p += sum_a phi_I[a](p) u[a][p]   with S' = D_II for
//         I = J and D_IJ + D_JI^T otherwise (rho = sum over I <= J)
//   force u = S2_IJ phi_J^T with S2 = D + D^T, dE/dR_I -= w_p grad phi_I . u and,
//         for I != J, the mirrored product for dE/dR_J

enum { MODE_H = 0, MODE_RHO = 1, MODE_FORCE = 2 };

template <int MODE>
__global__ __launch_bounds__(256) void k_pairs(Geo g, Bins bn, Basis bs, int nchunk, const double *__restrict__ W,
                                               double wscale, const double *__restrict__ D, int norb,
                                               double *__restrict__ out)
{
    constexpr int PT = (MODE == MODE_FORCE) ? 16 : 32;  // points staged per step
    constexpr int NG = (MODE == MODE_FORCE) ? 3 : 1;    // gradient rows
    __shared__ double s_phi[8][PT][kRow];
    __shared__ double s_grad[NG][(MODE == MODE_FORCE) ? 8 : 1][(MODE == MODE_FORCE) ? PT : 1][kRow];
    __shared__ double s_w[PT];
    __shared__ double s_red[4][PT];
    __shared__ int s_list[256];
    __shared__ int s_wcnt[4];
    __shared__ int s_ent[8];
    __shared__ long long s_slot;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int pair = blockIdx.x / nchunk, chunk = blockIdx.x % nchunk;
    const int A = bn.pairA[pair], B = bn.pairB[pair];
    const bool diag = (A == B);
    const int natom = g.natom;
    const int Iint = A * kGroup + wave;
    const bool Iex = Iint < natom;

    // ---- density-matrix fragments of this wave's blocks (loaded once) ----
    double fa[4][4], fb[4][4];
    if (MODE != MODE_H) {
        const int Iin = Iex ? bs.perm[Iint] : 0;
        const int mu0 = bs.orb0[Iin];
        const int nI = Iex ? bs.orb0[Iin + 1] - mu0 : 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int Jint = B * kGroup + j;
            const bool act = Iex && Jint < natom && (!diag || j >= wave);
            const int Jin = act ? bs.perm[Jint] : 0;
            const int nu0 = bs.orb0[Jin];
            const int nJ = act ? bs.orb0[Jin + 1] - nu0 : 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int kb = 4 * c + lk;
                // fa: S[a = li][b = kb]   (rho: S'; force: S2)
                double v = 0.0;
                if (li < nI && kb < nJ) {
                    const double dij = D[(size_t)(mu0 + li) * norb + nu0 + kb];
                    const double dji = D[(size_t)(nu0 + kb) * norb + mu0 + li];
                    if (MODE == MODE_RHO)
                        v = (diag && j == wave) ? dij : dij + dji;
                    else
                        v = dij + dji;
                }
                fa[j][c] = v;
                // fb (force only): S2_JI[b = li][a = kb] = S2_IJ[kb][li]
                double u = 0.0;
                if (MODE == MODE_FORCE && kb < nI && li < nJ)
                    u = D[(size_t)(mu0 + kb) * norb + nu0 + li] + D[(size_t)(nu0 + li) * norb + mu0 + kb];
                fb[j][c] = u;
            }
        }
    }

    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        acc[j] = d4{0.0, 0.0, 0.0, 0.0};
    double fI[3] = {0.0, 0.0, 0.0};
    double fJ[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        fJ[j][0] = fJ[j][1] = fJ[j][2] = 0.0;

    const int gb0 = bn.gptr[A], gb1 = bn.gptr[A + 1];
    const long long len = gb1 - gb0;
    const int c0 = gb0 + (int)(len * chunk / nchunk);
    const int c1 = gb0 + (int)(len * (chunk + 1) / nchunk);

    for (int base = c0; base < c1; base += 256) {
        // ---- batches of this chunk that group B also reaches (ordered) ----
        bool keep = false;
        int bb = -1;
        if (base + tid < c1) {
            bb = bn.gbatch[base + tid];
            keep = diag || batch_has_group(bn.bgptr, bn.bgrp, bb, B);
        }
        const unsigned long long m = __ballot(keep);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0)
            s_wcnt[wave] = __popcll(m);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; ++w)
            off += s_wcnt[w];
        if (keep)
            s_list[off + pre] = bb;
        const int nlist = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
        __syncthreads();

        for (int it = 0; it < nlist; ++it) {
            const int b = s_list[it];
            if (tid < 8) {
                const int atom = (tid < 4) ? A * kGroup + tid : B * kGroup + (tid - 4);
                s_ent[tid] = (atom < natom && !(diag && tid >= 4)) ? find_entry(bn, b, atom) : -1;
            }
            if (MODE == MODE_RHO && tid == 0) {
                const int n = bn.bgptr[b + 1] - bn.bgptr[b];
                const int pa = group_rank(bn, b, A), pb = group_rank(bn, b, B);
                s_slot = bn.soff[b] + (long long)pa * n - (long long)pa * (pa - 1) / 2 + (pb - pa);
            }
            __syncthreads();
            const bool rowI = Iex && s_ent[wave] >= 0;

            for (int sub = 0; sub < g.P; sub += PT) {
                // ---- stage the folded orbitals (PhiOperator) ----
                {
                    const int s = tid / PT, p = tid % PT;
                    if (s < 8) {
                        double *row = &s_phi[s][p][0];
                        double *gx = (MODE == MODE_FORCE) ? &s_grad[0][s % 8][p % PT][0] : nullptr;
                        double *gy = (MODE == MODE_FORCE) ? &s_grad[NG > 1 ? 1 : 0][s % 8][p % PT][0] : nullptr;
                        double *gz = (MODE == MODE_FORCE) ? &s_grad[NG > 2 ? 2 : 0][s % 8][p % PT][0] : nullptr;
#pragma unroll
                        for (int o = 0; o < kMaxOrb; ++o) {
                            row[o] = 0.0;
                            if (MODE == MODE_FORCE) {
                                gx[o] = 0.0;
                                gy[o] = 0.0;
                                gz[o] = 0.0;
                            }
                        }
                        const int e = s_ent[s];
                        if (e >= 0) {
                            double r[3];
                            int gi;
                            mesh_point(g, b, sub + p, r, &gi);
                            if (gi >= 0)
                                eval_atom<MODE == MODE_FORCE>(g, bs, e, bn.ent_atom, bn.ent_img, bn.img, r, row,
                                                              gx, gy, gz);
                        }
                    }
                    if (MODE != MODE_RHO && tid < PT) {
                        double r[3];
                        int gi;
                        mesh_point(g, b, sub + tid, r, &gi);
                        s_w[tid] = (gi >= 0) ? wscale * W[gi] : 0.0;
                    }
                }
                __syncthreads();

                // ---- contractions on the matrix cores ----
                if (MODE == MODE_H) {
                    if (rowI) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int sj = diag ? j : 4 + j;
                            if ((!diag || j >= wave) && s_ent[sj] >= 0) {
#pragma unroll
                                for (int kk = 0; kk < PT / 4; ++kk) {
                                    const int p = 4 * kk + lk;
                                    const double av = s_w[p] * s_phi[wave][p][li];
                                    const double bv = s_phi[sj][p][li];
                                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[j], 0, 0, 0);
                                }
                            }
                        }
                    }
                } else if (MODE == MODE_RHO) {
#pragma unroll
                    for (int q = 0; q < PT / 16; ++q) {
                        double rp = 0.0;
                        if (rowI) {
                            const int p = 16 * q + li;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const int sj = diag ? j : 4 + j;
                                if ((!diag || j >= wave) && s_ent[sj] >= 0) {
                                    d4 u = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                                    for (int c = 0; c < 4; ++c)
                                        u = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[j][c], s_phi[sj][p][4 * c + lk], u,
                                                                                0, 0, 0);
                                    const double *pI = &s_phi[wave][p][lk];
                                    rp += u[0] * pI[0] + u[1] * pI[4] + u[2] * pI[8] + u[3] * pI[12];
                                }
                            }
                        }
                        rp += __shfl_xor(rp, 16);
                        rp += __shfl_xor(rp, 32);
                        if (lane < 16)
                            s_red[wave][16 * q + lane] = rp;
                    }
                } else {
                    if (rowI) {
                        const int p = li;
                        const double wp = s_w[p];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int sj = diag ? j : 4 + j;
                            if ((!diag || j >= wave) && s_ent[sj] >= 0) {
                                d4 u = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                                for (int c = 0; c < 4; ++c)
                                    u = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[j][c], s_phi[sj][p][4 * c + lk], u, 0,
                                                                            0, 0);
#pragma unroll
                                for (int x = 0; x < 3; ++x) {
                                    const double *gI = &s_grad[x][wave][p][lk];
                                    fI[x] += wp * (u[0] * gI[0] + u[1] * gI[4] + u[2] * gI[8] + u[3] * gI[12]);
                                }
                                if (!(diag && j == wave)) {
                                    d4 u2 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                                    for (int c = 0; c < 4; ++c)
                                        u2 = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[j][c], s_phi[wave][p][4 * c + lk],
                                                                                 u2, 0, 0, 0);
#pragma unroll
                                    for (int x = 0; x < 3; ++x) {
                                        const double *gJ = &s_grad[x][sj][p][lk];
                                        fJ[j][x] +=
                                            wp * (u2[0] * gJ[0] + u2[1] * gJ[4] + u2[2] * gJ[8] + u2[3] * gJ[12]);
                                    }
                                }
                            }
                        }
                    }
                }
                __syncthreads();

                if (MODE == MODE_RHO) {
                    // fixed-order sum over the 4 waves, one partial per batch point
                    if (tid < PT && sub + tid < g.P)
                        out[(size_t)s_slot * g.P + sub + tid] =
                            ((s_red[0][tid] + s_red[1][tid]) + s_red[2][tid]) + s_red[3][tid];
                    __syncthreads();
                }
            }
        }
        __syncthreads();
    }

    // ---- outputs ----
    if (MODE == MODE_H) {
        double *blk = out + (size_t)blockIdx.x * 16 * 256;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!diag || j >= wave) {
                double *o = blk + (size_t)(wave * 4 + j) * 256;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    o[(lk + 4 * v) * 16 + li] = acc[j][v];
            }
        }
    } else if (MODE == MODE_FORCE) {
        // wave sums (fixed butterfly), then slots: A atoms in 0..3, B atoms in 4..7
        __shared__ double s_f[4][5][3];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            double v = fI[x];
            for (int o = 32; o > 0; o >>= 1)
                v += __shfl_xor(v, o);
            if (lane == 0)
                s_f[wave][4][x] = v;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double u = fJ[j][x];
                for (int o = 32; o > 0; o >>= 1)
                    u += __shfl_xor(u, o);
                if (lane == 0)
                    s_f[wave][j][x] = u;
            }
        }
        __syncthreads();
        if (tid < 24) {
            const int slot = tid / 3, x = tid % 3;
            double v = 0.0;
            if (slot < 4) {
                v = s_f[slot][4][x];
                if (diag)
                    v += ((s_f[0][slot][x] + s_f[1][slot][x]) + s_f[2][slot][x]) + s_f[3][slot][x];
            } else if (!diag) {
                const int j = slot - 4;
                v = ((s_f[0][j][x] + s_f[1][j][x]) + s_f[2][j][x]) + s_f[3][j][x];
            }
            out[(size_t)blockIdx.x * 24 + tid] = -v;
        }
    }
}

hipError_t launch_pairs_H(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int npair, int nchunk,
                          const double *W, double wscale, double *Hblk)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pairs<MODE_H>, dim3(npair * nchunk), dim3(256), 0, s, g, bn, b, nchunk, W, wscale,
                       (const double *)nullptr, 0, Hblk);
    return hipGetLastError();
}

hipError_t launch_pairs_rho(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int npair, int nchunk,
                            const double *D, int norb, double *rho_part)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pairs<MODE_RHO>, dim3(npair * nchunk), dim3(256), 0, s, g, bn, b, nchunk,
                       (const double *)nullptr, 0.0, D, norb, rho_part);
    return hipGetLastError();
}

hipError_t launch_pairs_force(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int npair, int nchunk,
                              const double *W, double wscale, const double *D, int norb, double *Fpart)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pairs<MODE_FORCE>, dim3(npair * nchunk), dim3(256), 0, s, g, bn, b, nchunk, W, wscale, D,
                       norb, Fpart);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions and output layouts.

// Dense symmetric H from the canonical (upper) atom-pair blocks, summing the
// chunks in order.  H[mu][nu] and H[nu][mu] read the same stored value.
__global__ void k_H_convert(Geo g, Bins bn, Basis bs, int norb, int nchunk, const double *__restrict__ Hblk,
                            double *__restrict__ H)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)norb * norb)
        return;
    const int mu = (int)(idx / norb), nu = (int)(idx % norb);
    const int Iin = bs.orb_atom[mu], Jin = bs.orb_atom[nu];
    int a = mu - bs.orb0[Iin], c = nu - bs.orb0[Jin];
    int ii = bs.inv_perm[Iin], jj = bs.inv_perm[Jin];
    if (ii > jj || (ii == jj && a > c)) {
        int t = ii;
        ii = jj;
        jj = t;
        t = a;
        a = c;
        c = t;
    }
    const int gA = ii / kGroup, gB = jj / kGroup;
    const int p = bn.pair_index[(size_t)gA * g.ngroup + gB];
    double v = 0.0;
    if (p >= 0) {
        const int blk = (ii % kGroup) * 4 + (jj % kGroup);
        for (int ch = 0; ch < nchunk; ++ch)
            v += Hblk[((size_t)(p * nchunk + ch) * 16 + blk) * 256 + a * 16 + c];
    }
    H[idx] = v;
}

hipError_t launch_H_convert(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int norb, int nchunk,
                            const double *Hblk, double *H)
{
    const long long n = (long long)norb * norb;
    hipLaunchKernelGGL(k_H_convert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, bn, b, norb, nchunk,
                       Hblk, H);
    return hipGetLastError();
}

// rho(r_g) = fixed-order sum of the batch's group-pair partials.
__global__ void k_rho_reduce(Geo g, Bins bn, const double *__restrict__ part, double *__restrict__ rho)
{
    const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long ng = (long long)g.N[0] * g.N[1] * g.N[2];
    if (gi >= ng)
        return;
    const int n2 = (int)(gi % g.N[2]);
    const int n1 = (int)((gi / g.N[2]) % g.N[1]);
    const int n0 = (int)(gi / ((long long)g.N[2] * g.N[1]));
    const int b = ((n0 / g.bs[0]) * g.nb[1] + n1 / g.bs[1]) * g.nb[2] + n2 / g.bs[2];
    const int q = ((n0 % g.bs[0]) * g.bs[1] + n1 % g.bs[1]) * g.bs[2] + n2 % g.bs[2];
    double v = 0.0;
    for (long long k = bn.soff[b]; k < bn.soff[b + 1]; ++k)
        v += part[(size_t)k * g.P + q];
    rho[gi] = v;
}

hipError_t launch_rho_reduce(hipStream_t s, const Geo &g, const Bins &bn, const double *rho_part, double *rho)
{
    const long long n = (long long)g.N[0] * g.N[1] * g.N[2];
    hipLaunchKernelGGL(k_rho_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, bn, rho_part, rho);
    return hipGetLastError();
}

// dE/dR per atom: fixed-order sum over the group pairs and chunks that hold
// the atom (as row group A or column group B).
__global__ __launch_bounds__(256) void k_force_reduce(Geo g, Bins bn, Basis bs, int npair, int nchunk,
                                                      const double *__restrict__ Fpart, double *__restrict__ dEdR)
{
    __shared__ double red[3][256];
    const int ii = blockIdx.x;
    const int grp = ii / kGroup, sl = ii % kGroup;
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < npair * nchunk; k += 256) {
        const int p = k / nchunk;
        const int A = bn.pairA[p], B = bn.pairB[p];
        int slot = -1;
        if (A == grp)
            slot = sl;
        else if (B == grp)
            slot = 4 + sl;
        if (slot >= 0)
            for (int x = 0; x < 3; ++x)
                v[x] += Fpart[(size_t)k * 24 + slot * 3 + x];
    }
    for (int x = 0; x < 3; ++x)
        red[x][threadIdx.x] = v[x];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int x = 0; x < 3; ++x)
                red[x][threadIdx.x] += red[x][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 3)
        dEdR[3 * bs.perm[ii] + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_force_reduce(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int npair, int nchunk,
                               const double *Fpart, double *dEdR)
{
    hipLaunchKernelGGL(k_force_reduce, dim3(g.natom), dim3(256), 0, s, g, bn, b, npair, nchunk, Fpart, dEdR);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact work counts: n_g = orbitals of the atoms with an image strictly
// inside their cutoff at mesh point g; per-block partial sums of n_g, n_g^2.

__global__ __launch_bounds__(256) void k_support_count(Geo g, Bins bn, Basis bs, double *__restrict__ sums)
{
    __shared__ double r1[256], r2[256];
    double s1 = 0.0, s2 = 0.0;
    const long long total = (long long)g.nbatch * g.P;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const int b = (int)(t / g.P), q = (int)(t % g.P);
        double r[3];
        int gi;
        mesh_point(g, b, q, r, &gi);
        if (gi < 0)
            continue;
        int n = 0;
        for (int e = bn.bptr[b]; e < bn.bptr[b + 1]; ++e) {
            const int a = bn.ent_atom[e];
            const DevSpecies S = bs.sp[bs.spc[a]];
            bool in = false;
            for (int im = bn.ent_img[e]; im < bn.ent_img[e + 1] && !in; ++im) {
                const int pk = bn.img[im];
                const int n0 = (int)(signed char)(pk & 0xff), n1 = (int)(signed char)((pk >> 8) & 0xff),
                          n2 = (int)(signed char)((pk >> 16) & 0xff);
                double d2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double dk =
                        r[k] - (bs.xw[3 * a + k] + n0 * g.lat[k] + n1 * g.lat[3 + k] + n2 * g.lat[6 + k]);
                    d2 += dk * dk;
                }
                in = sqrt(d2) < S.rc;
            }
            if (in)
                n += S.norb;
        }
        s1 += n;
        s2 += (double)n * n;
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sums[2 * blockIdx.x] = r1[0];
        sums[2 * blockIdx.x + 1] = r2[0];
    }
}

hipError_t launch_support_count(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, double *sums,
                                int nblocks)
{
    hipLaunchKernelGGL(k_support_count, dim3(nblocks), dim3(256), 0, s, g, bn, b, sums);
    return hipGetLastError();
}

}  // namespace gint
