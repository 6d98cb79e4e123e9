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

#include <algorithm>
#include <climits>
#include <hipcub/hipcub.hpp>

#include "gint_device.h"

namespace gint {

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
// Atom wrapping and Morton ordering

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
                            int *__restrict__ cnt_g)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.nbatch)
        return;
    int ne, ni, ng;
    bin_one_batch<false>(g, bs, b, &ne, &ni, &ng, nullptr, nullptr, nullptr, nullptr, 0, 0, 0);
    cnt_e[b] = ne;
    cnt_i[b] = ni;
    cnt_g[b] = ng;
}

hipError_t launch_bin_count(hipStream_t s, const Geo &g, const Basis &b, int *cnt_e, int *cnt_i, int *cnt_g)
{
    hipLaunchKernelGGL(k_bin_count, dim3((g.nbatch + 127) / 128), dim3(128), 0, s, g, b, cnt_e, cnt_i, cnt_g);
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
// Exclusive scan out[i] = sum_{j<i} in[j], out[n] = total, in three passes
// over tiles of kScanTile elements (1024 threads x 4 consecutive elements):
// tile sums; an exclusive scan of the tile sums (one workgroup); each tile
// scanned and offset by its tile's sum.  tmp holds the tile sums
// (ceil(n / kScanTile) ints).

constexpr int kScanTile = 4096;

// inclusive scan over the 1024 threads of a workgroup; returns the exclusive
// prefix of this thread, *total the workgroup's sum
__device__ __forceinline__ int block_scan_excl(int v, int *s_w, int *total)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        s_w[w] = x;
    __syncthreads();
    if (w == 0) {
        int u = lane < 16 ? s_w[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int y = __shfl_up(u, o);
            if (lane >= o)
                u += y;
        }
        if (lane < 16)
            s_w[16 + lane] = u;  // inclusive prefix of the wave sums
    }
    __syncthreads();
    *total = s_w[31];
    const int before = w > 0 ? s_w[16 + w - 1] : 0;
    return before + x - v;
}

__global__ __launch_bounds__(1024) void k_scan_tiles(const int *__restrict__ in, long long n, int *__restrict__ tsum)
{
    __shared__ int s_w[32];
    const long long base = (long long)blockIdx.x * kScanTile + 4 * (long long)threadIdx.x;
    int v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < n)
            v += in[base + k];
    int total;
    (void)block_scan_excl(v, s_w, &total);
    if (threadIdx.x == 0)
        tsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(int *__restrict__ tsum, int ntile, int *__restrict__ total_out)
{
    __shared__ int s_w[32];
    int carry = 0;
    for (int c = 0; c < ntile; c += 1024) {
        const int i = c + threadIdx.x;
        const int v = i < ntile ? tsum[i] : 0;
        int total;
        const int ex = block_scan_excl(v, s_w, &total);
        if (i < ntile)
            tsum[i] = carry + ex;
        carry += total;
        __syncthreads();  // s_w reused by the next chunk
    }
    if (threadIdx.x == 0)
        *total_out = carry;
}

__global__ __launch_bounds__(1024) void k_scan_apply(const int *__restrict__ in, long long n,
                                                     const int *__restrict__ toff, int *__restrict__ out)
{
    __shared__ int s_w[32];
    const long long base = (long long)blockIdx.x * kScanTile + 4 * (long long)threadIdx.x;
    int v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        sum += v[k];
    }
    int total;
    int run = toff[blockIdx.x] + block_scan_excl(sum, s_w, &total);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < n) {
            out[base + k] = run;
            run += v[k];
        }
}

int scan_tmp_ints(long long n) { return (int)((n + kScanTile - 1) / kScanTile) + 1; }

hipError_t launch_scan_i32(hipStream_t s, const int *in, long long n, int *out, int *tmp)
{
    const long long nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 0)
        return launch_fill_i32(s, out, 1, 0);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(1024), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, (int)nt, out + n);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(1024), 0, s, in, n, tmp, out);
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

// Per-group batch lists, in increasing batch order.  The batches are cut
// into chunks of kGroupChunk; workgroup (group, chunk) counts, then fills,
// the chunk's batches that hold the group, so the counts scanned in
// (group, chunk) order give every workgroup its output offset.
constexpr int kGroupChunk = 4096;

int group_chunks(const Geo &g) { return (g.nbatch + kGroupChunk - 1) / kGroupChunk; }

template <bool FILL>
__global__ __launch_bounds__(256) void k_group_lists(Geo g, int nchunk, const int *__restrict__ bgptr,
                                                     const int *__restrict__ bgrp, int *__restrict__ cnt,
                                                     const int *__restrict__ off, int *__restrict__ gbatch,
                                                     int *__restrict__ gptr)
{
    __shared__ int wcnt[4];
    const int grp = blockIdx.x / nchunk, ch = blockIdx.x % nchunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b0 = ch * kGroupChunk, b1 = min(b0 + kGroupChunk, g.nbatch);
    int run = FILL ? off[blockIdx.x] : 0;
    for (int base = b0; base < b1; base += 256) {
        const int b = base + threadIdx.x;
        const bool keep = (b < b1) && batch_has_group(bgptr, bgrp, b, grp);
        const unsigned long long m = __ballot(keep);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0)
            wcnt[wave] = __popcll(m);
        __syncthreads();
        int o = 0;
        for (int w = 0; w < wave; ++w)
            o += wcnt[w];
        if (FILL && keep)
            gbatch[run + o + pre] = b;
        run += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (!FILL)
            cnt[blockIdx.x] = run;
        else {
            if (ch == 0)
                gptr[grp] = off[blockIdx.x];
            if (blockIdx.x == gridDim.x - 1)
                gptr[g.ngroup] = off[gridDim.x];
        }
    }
}

hipError_t launch_group_count(hipStream_t s, const Geo &g, const int *bgptr, const int *bgrp, int *cnt)
{
    const int nc = group_chunks(g);
    hipLaunchKernelGGL(k_group_lists<false>, dim3(g.ngroup * nc), dim3(256), 0, s, g, nc, bgptr, bgrp, cnt, nullptr,
                       nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_group_fill(hipStream_t s, const Geo &g, const int *bgptr, const int *bgrp, const int *off,
                             int *gbatch, int *gptr)
{
    const int nc = group_chunks(g);
    hipLaunchKernelGGL(k_group_lists<true>, dim3(g.ngroup * nc), dim3(256), 0, s, g, nc, bgptr, bgrp, nullptr, off,
                       gbatch, gptr);
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
// Mesh point q of batch b: cartesian position and flat mesh index (-1 if
// outside the mesh).

__device__ __forceinline__ void mesh_point(const Geo &g, int b, int q, double *r, int *gidx)
{
    int ib[3], n[3];
    batch_coords(g, b, ib);
    if (!batch_point(g, ib, q, n)) {
        *gidx = -1;
        return;
    }
    *gidx = (n[0] * g.N[1] + n[1]) * g.N[2] + n[2];
    mesh_cart(g, n, r);
}

// Maximum of an int array (one workgroup).
// max of n non-negative ints: per-workgroup maxima combined with an integer
// atomic max into *out, zeroed first (the result does not depend on the
// order of the atomics)
__global__ __launch_bounds__(256) void k_max_i32(const int *__restrict__ a, long long n, int *__restrict__ out)
{
    __shared__ int red[256];
    int m = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        m = a[i] > m ? a[i] : m;
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            red[threadIdx.x] = red[threadIdx.x + o] > red[threadIdx.x] ? red[threadIdx.x + o] : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(out, red[0]);
}

hipError_t launch_max_i32(hipStream_t s, const int *a, long long n, int *out)
{
    const hipError_t e = launch_fill_i32(s, out, 1, 0);
    if (e != hipSuccess)
        return e;
    const long long nblk = std::min<long long>(256, std::max<long long>(1, (n + 1023) / 1024));
    hipLaunchKernelGGL(k_max_i32, dim3((unsigned)nblk), dim3(256), 0, s, a, n, out);
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

namespace gint {

// ---------------------------------------------------------------------------
// Lists for the point-stationary H path.

// Atom-pair blocks (ia <= ja) of each batch: n_b (n_b + 1) / 2.
__global__ void k_block_count(int nbatch, const int *__restrict__ bptr, int *__restrict__ cnt)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbatch)
        return;
    const int n = bptr[b + 1] - bptr[b];
    cnt[b] = n * (n + 1) / 2;
}

hipError_t launch_block_count(hipStream_t s, int nbatch, const int *bptr, int *cnt)
{
    hipLaunchKernelGGL(k_block_count, dim3((nbatch + 255) / 256), dim3(256), 0, s, nbatch, bptr, cnt);
    return hipGetLastError();
}

// Entry indices of each atom in increasing batch order: one workgroup per
// atom scans its group's batch list and compacts in order.
// With FILL false it only counts them into acnt (the count and fill passes
// visit the same batches in the same way).
template <bool FILL>
__global__ __launch_bounds__(256) void k_atom_fill(const int *__restrict__ gptr, const int *__restrict__ gbatch,
                                                   const int *__restrict__ bptr, const int *__restrict__ ent_atom,
                                                   const int *__restrict__ aptr, int *__restrict__ aent,
                                                   int *__restrict__ abat, int *__restrict__ acnt)
{
    __shared__ int wcnt[4];
    const int ii = blockIdx.x, grp = ii / kGroup;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int run = FILL ? aptr[ii] : 0;
    for (int base = gptr[grp]; base < gptr[grp + 1]; base += 256) {
        const int k = base + threadIdx.x;
        int e = -1, b = -1;
        if (k < gptr[grp + 1]) {
            b = gbatch[k];
            const int lo = bptr[b], hi = bptr[b + 1];
            const int f = lower_bound_i(ent_atom, lo, hi, ii);
            if (f < hi && ent_atom[f] == ii)
                e = f;
        }
        const unsigned long long m = __ballot(e >= 0);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0)
            wcnt[wave] = __popcll(m);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; ++w)
            off += wcnt[w];
        if (FILL && e >= 0) {
            aent[run + off + pre] = e;
            abat[run + off + pre] = b;
        }
        run += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
    if (!FILL && threadIdx.x == 0)
        acnt[ii] = run;
}

hipError_t launch_atom_count(hipStream_t s, int natom, const int *gptr, const int *gbatch, const int *bptr,
                             const int *ent_atom, int *acnt)
{
    hipLaunchKernelGGL(k_atom_fill<false>, dim3(natom), dim3(256), 0, s, gptr, gbatch, bptr, ent_atom, nullptr,
                       nullptr, nullptr, acnt);
    return hipGetLastError();
}

hipError_t launch_atom_fill(hipStream_t s, int natom, const int *gptr, const int *gbatch, const int *bptr,
                            const int *ent_atom, const int *aptr, int *aent, int *abat)
{
    hipLaunchKernelGGL(k_atom_fill<true>, dim3(natom), dim3(256), 0, s, gptr, gbatch, bptr, ent_atom, aptr, aent,
                       abat, nullptr);
    return hipGetLastError();
}

// Partners of atom I whose H block (I, J) atom I owns: every J that can share
// a mesh batch with I (some images within rc_I + rc_J + 2 * batch radius),
// with each unordered pair owned by exactly one of its atoms (circulant rule
// on the internal order: J - I mod natom in [0, natom/2), ties to the
// smaller index).  Listed in increasing J.
__device__ __forceinline__ bool owns_pair(int I, int J, int natom)
{
    const int d = ((J - I) % natom + natom) % natom;
    if (d == 0)
        return true;
    if (2 * d < natom)
        return true;
    return 2 * d == natom && I < J;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_partners(Geo g, Basis bs, double brad, const int *__restrict__ pptr,
                                                  int *__restrict__ pcnt, int *__restrict__ plist)
{
    __shared__ int wcnt[4];
    const int I = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double *XI = bs.xw + 3 * I;
    const double rcI = bs.sp[bs.spc[I]].rc;
    double bn[3];
    for (int i = 0; i < 3; ++i)
        bn[i] = sqrt(g.rec[3 * i] * g.rec[3 * i] + g.rec[3 * i + 1] * g.rec[3 * i + 1] +
                     g.rec[3 * i + 2] * g.rec[3 * i + 2]);
    int run = FILL ? pptr[I] : 0;
    for (int base = 0; base < g.natom; base += 256) {
        const int J = base + threadIdx.x;
        bool keep = false;
        if (J < g.natom && owns_pair(I, J, g.natom)) {
            const double reach = rcI + bs.sp[bs.spc[J]].rc + 2.0 * brad + 1e-6;
            const double dx[3] = {XI[0] - bs.xw[3 * J], XI[1] - bs.xw[3 * J + 1], XI[2] - bs.xw[3 * J + 2]};
            double ds[3];
            frac_of(g, dx, ds);
            int lo[3], hi[3];
            for (int i = 0; i < 3; ++i) {
                lo[i] = (int)floor(ds[i] - reach * bn[i]);
                hi[i] = (int)ceil(ds[i] + reach * bn[i]);
            }
            for (int n0 = lo[0]; n0 <= hi[0] && !keep; ++n0)
                for (int n1 = lo[1]; n1 <= hi[1] && !keep; ++n1)
                    for (int n2 = lo[2]; n2 <= hi[2] && !keep; ++n2) {
                        double d2 = 0.0;
                        for (int k = 0; k < 3; ++k) {
                            const double v = dx[k] - (n0 * g.lat[k] + n1 * g.lat[3 + k] + n2 * g.lat[6 + k]);
                            d2 += v * v;
                        }
                        keep = d2 < reach * reach;
                    }
        }
        const unsigned long long m = __ballot(keep);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0)
            wcnt[wave] = __popcll(m);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; ++w)
            off += wcnt[w];
        if (FILL && keep)
            plist[run + off + pre] = J;
        run += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
    if (!FILL && threadIdx.x == 0)
        pcnt[I] = run;
}

hipError_t launch_partners(hipStream_t s, const Geo &g, const Basis &b, double brad, const int *pptr, int *pcnt,
                           int *plist)
{
    if (plist)
        hipLaunchKernelGGL(k_partners<true>, dim3(g.natom), dim3(256), 0, s, g, b, brad, pptr, pcnt, plist);
    else
        hipLaunchKernelGGL(k_partners<false>, dim3(g.natom), dim3(256), 0, s, g, b, brad, pptr, pcnt, plist);
    return hipGetLastError();
}

}  // namespace gint

namespace gint {

// ---------------------------------------------------------------------------
// Block lists of the owned atom pairs, for the H reduction.
//
// For owned pair p = (I, J) (I the owner, J = plist[p]) the list holds, in
// increasing batch order, one code per batch that both atoms reach: the
// index q of block (min(ia, ja), max(ia, ja)) among the H block partials, as
// q when ia <= ja (the block is H_IJ) or -(q + 1) when it is H_JI.  One wave
// per pair intersects the two atoms' batch-sorted entry lists 64 at a time:
// each lane looks its batch up in the other window (a binary search over
// lanes), and both windows then advance past the smaller window maximum, so
// every common batch is met exactly once.  Both forms write the list's
// length to lcnt; the filling form writes the list at lptr[p].

namespace {
__device__ __forceinline__ int upper_bound_i(const int *__restrict__ a, int lo, int hi, int key)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int tri_block(int lo, int hi, int n) { return lo * n - lo * (lo - 1) / 2 + (hi - lo); }
}  // namespace

template <bool FILL>
__global__ __launch_bounds__(256) void k_pair_blocks(int natom, int npair, const int *__restrict__ aptr,
                                                     const int *__restrict__ aent, const int *__restrict__ abat,
                                                     const int *__restrict__ bptr, const int *__restrict__ boff,
                                                     const int *__restrict__ pptr, const int *__restrict__ plist,
                                                     int *__restrict__ lcnt, const int *__restrict__ lptr,
                                                     int *__restrict__ list)
{
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= npair)
        return;
    const int I = upper_bound_i(pptr, 0, natom + 1, p) - 1;
    const int J = plist[p];
    const int a0 = aptr[I], nA = aptr[I + 1] - a0;
    const int c0 = aptr[J], nB = aptr[J + 1] - c0;
    int ia0 = 0, ib0 = 0, run = 0;
    const int out0 = FILL ? lptr[p] : 0;
    while (ia0 < nA && ib0 < nB) {
        const int ka = ia0 + lane, kb = ib0 + lane;
        const int av = ka < nA ? abat[a0 + ka] : INT_MAX;
        const int bv = kb < nB ? abat[c0 + kb] : INT_MAX;
        const int la = min(63, nA - 1 - ia0), lb = min(63, nB - 1 - ib0);
        const int m = min(__shfl(av, la), __shfl(bv, lb));
        // lanes of the B window holding values < av
        int pos = 0;
#pragma unroll
        for (int st = 32; st >= 1; st >>= 1) {
            const int v = __shfl(bv, pos + st - 1);
            if (v < av)
                pos += st;
        }
        const int hit_b = __shfl(bv, min(pos, 63));
        const bool hit = av <= m && pos < 64 && hit_b == av;
        const unsigned long long mh = __ballot(hit);
        if (FILL) {
            const int ebv = kb < nB ? aent[c0 + kb] : 0;
            const int eb = __shfl(ebv, min(pos, 63));
            if (hit) {
                const int b = av;
                const int base = bptr[b], nb = bptr[b + 1] - base;
                const int ia = aent[a0 + ka] - base, ja = eb - base;
                const int q = boff[b] + (ia <= ja ? tri_block(ia, ja, nb) : tri_block(ja, ia, nb));
                list[out0 + run + __popcll(mh & ((1ull << lane) - 1ull))] = ia <= ja ? q : -(q + 1);
            }
        }
        run += __popcll(mh);
        ia0 += __popcll(__ballot(av <= m));
        ib0 += __popcll(__ballot(bv <= m));
    }
    if (lane == 0)
        lcnt[p] = run;
}

// Upper bound of every owned pair's block count (the smaller of the two
// atoms' entry counts): the fill pass writes each list at its bound's offset
__global__ __launch_bounds__(256) void k_pair_ub(int natom, int npair, const int *__restrict__ aptr,
                                                 const int *__restrict__ pptr, const int *__restrict__ plist,
                                                 int *__restrict__ ub)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npair)
        return;
    const int I = upper_bound_i(pptr, 0, natom + 1, p) - 1;
    const int J = plist[p];
    ub[p] = min(aptr[I + 1] - aptr[I], aptr[J + 1] - aptr[J]);
}

// Each pair's list (cnt[p] entries from src + uptr[p]) to dst + lptr[p], one
// wave per pair
__global__ __launch_bounds__(256) void k_list_compact(int npair, const int *__restrict__ uptr,
                                                      const int *__restrict__ lptr, const int *__restrict__ cnt,
                                                      const int *__restrict__ src, int *__restrict__ dst)
{
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= npair)
        return;
    const int lane = threadIdx.x & 63;
    const int *a = src + uptr[p];
    int *b = dst + lptr[p];
    for (int k = lane; k < cnt[p]; k += 64)
        b[k] = a[k];
}

hipError_t launch_pair_ub(hipStream_t s, int natom, int npair, const int *aptr, const int *pptr, const int *plist,
                          int *ub)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pair_ub, dim3((npair + 255) / 256), dim3(256), 0, s, natom, npair, aptr, pptr, plist, ub);
    return hipGetLastError();
}

hipError_t launch_list_compact(hipStream_t s, int npair, const int *uptr, const int *lptr, const int *cnt,
                               const int *src, int *dst)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_list_compact, dim3((npair + 3) / 4), dim3(256), 0, s, npair, uptr, lptr, cnt, src, dst);
    return hipGetLastError();
}

hipError_t launch_pair_blocks(hipStream_t s, int natom, int npair, const int *aptr, const int *aent,
                              const int *abat, const int *bptr, const int *boff, const int *pptr, const int *plist,
                              int *lcnt, const int *lptr, int *list)
{
    if (npair <= 0)
        return hipSuccess;
    const unsigned nblk = (unsigned)((npair + 3) / 4);
    if (list)
        hipLaunchKernelGGL(k_pair_blocks<true>, dim3(nblk), dim3(256), 0, s, natom, npair, aptr, aent, abat, bptr,
                           boff, pptr, plist, lcnt, lptr, list);
    else
        hipLaunchKernelGGL(k_pair_blocks<false>, dim3(nblk), dim3(256), 0, s, natom, npair, aptr, aent, abat, bptr,
                           boff, pptr, plist, lcnt, lptr, list);
    return hipGetLastError();
}


// Owner atom of every owned pair, and where each slab's blocks start in the
// pair's block list: lsl[p (nslab + 1) + s] = first list entry whose block
// index is >= slab_q[s] (slab_q[nslab] is past every block).  Lists hold
// block indices q (or -(q + 1), transposed blocks) in increasing q.
__global__ __launch_bounds__(256) void k_pair_slabs(int natom, int npair, const int *__restrict__ pptr,
                                                    const int *__restrict__ lptr, const int *__restrict__ list,
                                                    int nslab, const int *__restrict__ slab_q, int *__restrict__ pown,
                                                    int *__restrict__ lsl)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npair)
        return;
    int lo = 0, hi = natom + 1;  // last atom I with pptr[I] <= p
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pptr[mid] <= p)
            lo = mid + 1;
        else
            hi = mid;
    }
    pown[p] = lo - 1;
    const int l0 = lptr[p], l1 = lptr[p + 1];
    for (int si = 0; si <= nslab; ++si) {
        const int q = slab_q[si];
        int a = l0, z = l1;
        while (a < z) {
            const int mid = (a + z) >> 1;
            const int c = list[mid];
            if ((c >= 0 ? c : -c - 1) < q)
                a = mid + 1;
            else
                z = mid;
        }
        lsl[(size_t)p * (nslab + 1) + si] = a;
    }
}

hipError_t launch_pair_slabs(hipStream_t s, int natom, int npair, const int *pptr, const int *lptr, const int *list,
                             int nslab, const int *slab_q, int *pown, int *lsl)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pair_slabs, dim3((npair + 255) / 256), dim3(256), 0, s, natom, npair, pptr, lptr, list, nslab,
                       slab_q, pown, lsl);
    return hipGetLastError();
}

// Cost of every item (list entries of its reduction: ptr[i stride + span] -
// ptr[i stride]), with the item index as the value, for a heaviest-first
// launch order
__global__ void k_item_cost(int n, int stride, int span, const int *__restrict__ ptr, int *__restrict__ cost,
                            int *__restrict__ idx)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    cost[i] = ptr[(size_t)i * stride + span] - ptr[(size_t)i * stride];
    idx[i] = i;
}

hipError_t launch_item_order(hipStream_t s, void *tmp, size_t &tmp_bytes, int n, int stride, int span, const int *ptr,
                             int *cost, int *cost2, int *idx, int *order)
{
    if (!tmp)
        return hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tmp_bytes, cost, cost2, idx, order,
                                                            n > 0 ? n : 1, 0, 32, s);
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_item_cost, dim3((n + 255) / 256), dim3(256), 0, s, n, stride, span, ptr, cost, idx);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // stable: pairs of equal cost keep their index order
    return hipcub::DeviceRadixSort::SortPairsDescending(tmp, tmp_bytes, cost, cost2, idx, order, n, 0, 32, s);
}

}  // namespace gint
