// gint_dphi.hip -- the moving-basis matrix of Sec. 2.3 (Ehrenfest dynamics,
// D_K equation) on the uniform mesh, at the Gamma point:
//
//     DK_c,mu,nu = < phit_mu | W | d phit_nu / d tau_K >_c      (K = atom of nu)
//                = -dV sum_g W_g phit_mu(r_g) d/dr_c phit_nu(r_g),
//
// (an orbital centred on tau_K depends on it only through r - tau_K; the sum
// over lattice vectors of the D_K equation at k = 0 folds the orbital).
// With W = 1 its two orientations give the derivatives of the mesh overlap
// S_grid; with W = V it carries the grid force, dE/dR_I =
// sum_{mu on I, nu} (D + D^T)_mu,nu DK_V[nu][mu].
//
// Pair-stationary: one workgroup per owned atom pair (I, J) walks the
// batches the two atoms share (the pair's block list of the H reduction, in
// batch order), each wave taking every fourth batch.  Per batch a wave
// evaluates phit and grad phit of both atoms at the batch's points (one lane
// per (atom, point), one spline evaluation per radial) into its own LDS
// region and contracts them on the FP64 matrix cores into six 16 x 16
// accumulators that stay in registers for the whole list:
//     G^c_IJ += sum_p (w_p phit_I(p)) d_c phit_J(p)^T,
//     G^c_JI += sum_p (w_p phit_J(p)) d_c phit_I(p)^T   (I != J).
// The four waves' sums are added in a fixed order and written once: no
// partials in HBM, no atomics, repeatable bits.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gint_device.h"

namespace gint {

namespace {

constexpr int kDKWaves = 4;
constexpr int kDKVals = 4;  // w phit, d_x phit, d_y phit, d_z phit

// phit and its cartesian gradient for every orbital of one atom at point r,
// summed over the listed images (radials k0..k1-1 of its species, radial
// descriptors in LDS).  Value v of orbital o goes to out[v * vstride +
// (o ^ swz)]; the value row (v = 0) is scaled by wp.  The first image
// assigns, later images add (several images of one atom reach a point only
// in cells smaller than the cutoff sphere).
__device__ __forceinline__ void eval_phi_grad(const Geo &g, const DevRadial *__restrict__ rads, int k0, int k1,
                                              double rc, const double *__restrict__ coef, const double *X, int icnt,
                                              int pk0, int ioff, const int *__restrict__ img, const double *r,
                                              double wp, double *out, int vstride, int swz)
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
        const double u[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
        const bool add = i > 0;
        auto put = [&](int o, double ph, double gx, double gy, double gz) {
            double *q = out + (o ^ swz);
            if (add) {
                q[0] += wp * ph;
                q[vstride] += gx;
                q[2 * vstride] += gy;
                q[3 * vstride] += gz;
            } else {
                q[0] = wp * ph;
                q[vstride] = gx;
                q[2 * vstride] = gy;
                q[3 * vstride] = gz;
            }
        };
        // the spline coefficients of U radials are loaded together, then
        // the radials are evaluated one by one
        constexpr int U = 3;
        for (int kb = k0; kb < k1; kb += U) {
        double2 c01[U], c23[U];
        double tt[U];
#pragma unroll
        for (int iu = 0; iu < U; ++iu) {
            const int k = kb + iu;
            c01[iu] = double2{0.0, 0.0};
            c23[iu] = double2{0.0, 0.0};
            tt[iu] = 0.0;
            if (k < k1) {
                const DevRadial R = rads[k];
                if (inside && rr < R.rc) {
                    const int iv = spline_interval(R, rr, &tt[iu]);
                    c01[iu] = *reinterpret_cast<const double2 *>(coef + R.coef_off + 4 * iv);
                    c23[iu] = *reinterpret_cast<const double2 *>(coef + R.coef_off + 4 * iv + 2);
                }
            }
        }
#pragma unroll
        for (int iu = 0; iu < U; ++iu) {
            const int k = kb + iu;
            if (k >= k1)
                break;
            const DevRadial R = rads[k];
            const double t = tt[iu];
            const double f = c01[iu].x + t * (c01[iu].y + t * (c23[iu].x + t * c23[iu].y));
            const double fp = c01[iu].y + t * (2.0 * c23[iu].x + t * 3.0 * c23[iu].y);
            const int o = R.orb0;
            const double fr = f * ir;
            if (R.l == 0) {
                // grad (f Y00) = f' Y00 u (zero at the centre, where u = 0)
                const double a = fp * Y_C00;
                put(o, f * Y_C00, a * u[0], a * u[1], a * u[2]);
            } else if (R.l == 1) {
                // m = -1, 0, 1 -> y, z, x; Y = C1 u_a, dY/du = C1 e_a;
                // grad (f Y) = f' Y u + (f / r)(C1 e_a - Y u); f'(0) C1 e_a at the centre
                const int ax[3] = {1, 2, 0};
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const int a = ax[m];
                    const double Y = Y_C1 * u[a];
                    double gv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double e = (c == a) ? Y_C1 : 0.0;
                        gv[c] = tiny ? fp * e : fp * Y * u[c] + fr * (e - Y * u[c]);
                    }
                    put(o + m, f * Y, gv[0], gv[1], gv[2]);
                }
            } else {
                // m = -2 .. 2 -> xy, yz, 2z^2 - x^2 - y^2, xz, x^2 - y^2 (zero
                // value and gradient at the centre); G = dY/du,
                // grad (f Y) = f' Y u + (f / r)(G - 2 Y u)
                const double x = u[0], y = u[1], z = u[2];
                const double Y[5] = {Y_C2 * x * y, Y_C2 * y * z, Y_C20 * (2.0 * z * z - x * x - y * y), Y_C2 * x * z,
                                     Y_C22 * (x * x - y * y)};
                const double G[5][3] = {{Y_C2 * y, Y_C2 * x, 0.0},
                                        {0.0, Y_C2 * z, Y_C2 * y},
                                        {-2.0 * Y_C20 * x, -2.0 * Y_C20 * y, 4.0 * Y_C20 * z},
                                        {Y_C2 * z, 0.0, Y_C2 * x},
                                        {2.0 * Y_C22 * x, -2.0 * Y_C22 * y, 0.0}};
#pragma unroll
                for (int m = 0; m < 5; ++m) {
                    double gv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        gv[c] = tiny ? 0.0 : fp * Y[m] * u[c] + fr * (G[m][c] - 2.0 * Y[m] * u[c]);
                    put(o + m, f * Y[m], gv[0], gv[1], gv[2]);
                }
            }
        }
        }
    }
}

}  // namespace

// Entry descriptors of the pairs' block lists, once per geometry: list
// entry k holds, in batch order for its pair, the index q of the pair's
// block among the H block partials (boff[b] <= q < boff[b+1], block
// (lo, hi) of batch b's slot triangle), negated as -(q + 1) when the owner
// sits in the higher slot; desc[k] = (b, entry of the owner, entry of the
// partner, 0).
__global__ __launch_bounds__(256) void k_DK_desc(long long n, int nbatch, const int *__restrict__ list,
                                                 const int *__restrict__ boff, const int *__restrict__ bptr,
                                                 int4 *__restrict__ desc)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const int code = list[k];
    const int q = code >= 0 ? code : -code - 1;
    int lo = 0, hi = nbatch;  // last b with boff[b] <= q
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (boff[mid] <= q)
            lo = mid;
        else
            hi = mid;
    }
    const int b = lo;
    const int e0 = bptr[b], nb = bptr[b + 1] - e0;
    int t = q - boff[b], slo = 0;
    while (t >= nb - slo) {  // row slo of the triangle holds nb - slo blocks
        t -= nb - slo;
        ++slo;
    }
    const int shi = slo + t;
    desc[k] = int4{b, e0 + (code >= 0 ? slo : shi), e0 + (code >= 0 ? shi : slo), 0};
}

hipError_t launch_DK_desc(hipStream_t s, long long n, int nbatch, const int *list, const int *boff, const int *bptr,
                          int4 *desc)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_DK_desc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nbatch, list, boff, bptr,
                       desc);
    return hipGetLastError();
}

// One workgroup (kDKWaves waves) per owned pair p = (pown[p], plist[p])
// (internal atoms) over its list entries desc[lptr[p] .. lptr[p+1]).  DK
// (3 x norb x norb, input orbital order) must be zero outside the blocks of
// the owned pairs; each owned pair's blocks are written once (rows of I,
// columns of J, and rows of J, columns of I).
template <int P>
__global__ __launch_bounds__(64 * kDKWaves) void k_DK_pairs(Geo g, Bins bn, Basis bs, const double *__restrict__ W,
                                                           double wscale, int npair, const int *__restrict__ order,
                                                           const int *__restrict__ pown,
                                                           const int *__restrict__ plist,
                                                           const int *__restrict__ lptr,
                                                           const int4 *__restrict__ desc, int norb,
                                                           double *__restrict__ DK)
{
    constexpr int NV = kDKVals;
    // the batch's points in passes of HP (16 KB of LDS per wave, so that two
    // workgroups share a compute unit)
    constexpr int HP = P < 16 ? P : 16;
    constexpr int REG = NV * 2 * HP * kMaxOrb;  // doubles of one wave's LDS region
    extern __shared__ __align__(16) double s_dyn[];
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    // with a heaviest-first order, consecutive workgroups take consecutive
    // pairs (the hardware deals them round-robin over the XCDs, so every XCD
    // gets heavy and light pairs); without one, each XCD takes a contiguous
    // range of pairs (their batches overlap in its L2)
    const int w = order ? ((int)blockIdx.x < npair ? (int)blockIdx.x : -1) : xcd_batch(blockIdx.x, 0, npair);
    for (int k = tid; k < g.nrad; k += 64 * kDKWaves)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += 64 * kDKWaves)
        s_sp[k] = bs.sp[k];
    __syncthreads();
    if (w < 0)
        return;
    const int p = order ? order[w] : w;
    const int I = pown[p], J = plist[p];
    const bool self = I == J;
    double *reg = s_dyn + (size_t)wave * REG;
    // element (value v, slot s, point q, orbital o) of this wave's region
    auto at = [&](int v, int s, int q) { return reg + ((size_t)(v * 2 + s) * HP + q) * kMaxOrb; };

    typedef MM<double>::acc acc_t;
    acc_t cIJ[3], cJI[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        cIJ[c] = cJI[c] = MM<double>::zero();

    const int l0 = lptr[p], l1 = lptr[p + 1];
    // the wave's next descriptor is loaded one entry ahead
    int4 dn = l0 + wave < l1 ? desc[l0 + wave] : int4{0, 0, 0, 0};
    for (int k = l0 + wave; k < l1; k += kDKWaves) {
        const int4 dc = dn;
        if (k + kDKWaves < l1)
            dn = desc[k + kDKWaves];
        const int b = dc.x;  // the batch and the two atoms' entries in it (wave-uniform)
        int ib[3];
        batch_coords(g, b, ib);

#pragma unroll 1
        for (int h = 0; h < P / HP; ++h) {
        // ---- phit, grad phit of (atom slot s, point qp): two lanes each,
        // the first half of the atom's radials on one, the rest on the other ----
        wave_lds_sync();  // the previous pass's operand reads are done
        {
            const int it = lane % (2 * HP), part = lane / (2 * HP);
            const int s = it / HP, ql = it % HP, qp = h * HP + ql;
            if (s < 2 && !(self && s == 1)) {
                const int e = s == 0 ? dc.y : dc.z;
                const int atom = s == 0 ? I : J;
                const DevSpecies &S = s_sp[bs.spc[atom]];
                int n[3];
                const bool valid = batch_point(g, ib, qp, n);
                const int swz = ql & 15;
                double *row = at(0, s, ql);
                const int vs = 2 * HP * kMaxOrb;  // stride between values
                if (part == 0)
                    for (int o = valid ? S.norb : 0; o < kMaxOrb; ++o)
#pragma unroll
                        for (int v = 0; v < NV; ++v)
                            row[v * vs + (o ^ swz)] = 0.0;
                const int kmid = S.rad0 + (S.nrad + 1) / 2;
                const int k0 = part == 0 ? S.rad0 : kmid, k1 = part == 0 ? kmid : S.rad0 + S.nrad;
                if (valid && k0 < k1) {
                    const double wp = wscale * (W ? W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 1.0);
                    const int io = bn.ent_img[e];
                    const int cnt = bn.ent_img[e + 1] - io;
                    const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
                    double r[3];
                    mesh_cart(g, n, r);
                    eval_phi_grad(g, s_rad, k0, k1, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img, r, wp, row, vs,
                                  swz);
                }
            }
        }
        wave_lds_sync();

        // ---- the six (three for I == J) blocks on the matrix cores ----
        const int sj = self ? 0 : 1;
#pragma unroll
        for (int kk = 0; kk < HP / 4; ++kk) {
            const int ql = 4 * kk + lk;
            const int o = li ^ (ql & 15);
            const double aI = at(0, 0, ql)[o];
            const double aJ = at(0, sj, ql)[o];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cIJ[c] = MM<double>::mma(aI, at(1 + c, sj, ql)[o], cIJ[c]);
                if (!self)
                    cJI[c] = MM<double>::mma(aJ, at(1 + c, 0, ql)[o], cJI[c]);
            }
        }
        }
    }

    // ---- the waves' sums in a fixed order, then one write per element ----
    __syncthreads();
    double *red = s_dyn;  // [wave][block 0..5][16 x 16]
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = MM<double>::row(lk, v) * 16 + li;
            red[((size_t)wave * 6 + c) * 256 + e] = cIJ[c][v];
            red[((size_t)wave * 6 + 3 + c) * 256 + e] = cJI[c][v];
        }
    __syncthreads();
    const int Iin = bs.perm[I], Jin = bs.perm[J];
    const int mu0 = bs.orb0[Iin], nI = bs.orb0[Iin + 1] - mu0;
    const int nu0 = bs.orb0[Jin], nJ = bs.orb0[Jin + 1] - nu0;
    const size_t nn = (size_t)norb * norb;
    for (int e = tid; e < 6 * 256; e += 64 * kDKWaves) {
        const int blk = e >> 8, rc = e & 255, row = rc >> 4, col = rc & 15;
        if (self && blk >= 3)
            continue;
        const bool ij = blk < 3;
        const int c = ij ? blk : blk - 3;
        if (row >= (ij ? nI : nJ) || col >= (ij ? nJ : nI))
            continue;
        double sum = red[(size_t)(0 * 6 + blk) * 256 + rc];
#pragma unroll
        for (int w = 1; w < kDKWaves; ++w)
            sum += red[(size_t)(w * 6 + blk) * 256 + rc];
        const size_t off = ij ? (size_t)(mu0 + row) * norb + nu0 + col : (size_t)(nu0 + row) * norb + mu0 + col;
        DK[c * nn + off] = -sum;
    }
}

size_t DK_pairs_lds(int P)
{
    const int HP = P < 16 ? P : 16;
    // the phi / grad phi rows, and after the list the waves' six blocks
    return std::max(sizeof(double) * (size_t)kDKWaves * kDKVals * 2 * HP * kMaxOrb,
                    sizeof(double) * (size_t)kDKWaves * 6 * 256);
}

hipError_t launch_DK_pairs(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, const double *W, double wscale,
                           int npair, const int *order, const int *pown, const int *plist, const int *lptr,
                           const int4 *desc, int norb, double *DK)
{
    if (npair <= 0)
        return hipSuccess;
    const size_t lds = DK_pairs_lds(g.P);
    const unsigned nblk = (unsigned)(kXcd * ((npair + kXcd - 1) / kXcd));
    hipError_t e;
    if (g.P == 32) {
        e = hipFuncSetAttribute((const void *)k_DK_pairs<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_DK_pairs<32>, dim3(nblk), dim3(64 * kDKWaves), lds, s, g, bn, b, W, wscale, npair, order,
                           pown, plist, lptr, desc, norb, DK);
    } else if (g.P == 16) {
        e = hipFuncSetAttribute((const void *)k_DK_pairs<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_DK_pairs<16>, dim3(nblk), dim3(64 * kDKWaves), lds, s, g, bn, b, W, wscale, npair, order,
                           pown, plist, lptr, desc, norb, DK);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gint
