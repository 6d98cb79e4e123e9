// gint_sphere.hip -- spherical-grid integration of the projector overlaps of
// the velocity-gauge nonlocal pseudopotential (Sec. 3.3.2, "Spherical Grid
// Integration for Nonlocal Potentials"):
//
//     Q[p][mu] = < phit_mu | e^{-i A.r} | beta_p >
//              = sum_{i,j} W_ij phit_mu(tau_I + x_ij) e^{-i A.(tau_I + x_ij)} beta_p(x_ij)
//
// on the product grid around the projector's atom I: x_ij = r_i u_j,
// r_i = rb x_i, W_ij = rb q_i r_i^2 w_j (the caller's angular rule (u_j, w_j)
// and radial rule (x_i, q_i) on [0, 1]; rb the largest projector cutoff of
// I's species), beta_p(x) = b(|x|) Y_lm(x/|x|), phit the orbital folded over
// lattice images.
//
// One workgroup per projector atom, as in the paper's atom-level batching,
// but the sum over quadrature points is a dense contraction and runs on the
// FP64 matrix cores: points are taken 64 at a time (one per lane); the workgroup first
// tabulates W e^{-iA.r} beta_p at the chunk's points in LDS (the A operands,
// real and imaginary parts), then each wave evaluates phit of its
// neighbouring atoms at the same points (one lane per point, one spline
// evaluation per radial) and accumulates Q_re, Q_im of every (projector,
// orbital) block in registers across all chunks.  Each (I, J) block is
// written once: no atomics, repeatable bits.
#include <hip/hip_runtime.h>

#include "gint_device.h"

namespace gint {

namespace {

constexpr int kPBWaves = 8;
constexpr int kPBChunk = 64;                    // quadrature points per chunk (one per lane)
constexpr int kPBPerWave = 2;                   // neighbour entries per wave
constexpr int kPBGroup = kPBWaves * kPBPerWave;  // entries per workgroup

}  // namespace

// ---------------------------------------------------------------------------
// Neighbour lists: for projector atom a (internal index ia = pint[a]) and
// orbital atom J (internal), the lattice multiples n with
// |xw_ia - xw_J - n.A| < rb(ia) + rc(J) (wrapped positions).  Pass 0 counts
// into cnt[a * natom + J]; pass 1 writes the images at off[a * natom + J].
template <bool FILL>
__global__ __launch_bounds__(256) void k_pb_images(Geo g, Basis bs, int npa, const int *__restrict__ pint,
                                                   const double *__restrict__ prb, int m0, int m1, int m2,
                                                   int *__restrict__ cnt, const int *__restrict__ off,
                                                   int *__restrict__ img)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)npa * g.natom)
        return;
    const int a = (int)(t / g.natom), J = (int)(t % g.natom);
    const int I = pint[a];
    const double reach = prb[a] + bs.sp[bs.spc[J]].rc;
    double d0[3];
    for (int k = 0; k < 3; ++k)
        d0[k] = bs.xw[3 * I + k] - bs.xw[3 * J + k];
    int n = 0;
    const int o = FILL ? off[t] : 0;
    for (int n0 = -m0; n0 <= m0; ++n0)
        for (int n1 = -m1; n1 <= m1; ++n1)
            for (int n2 = -m2; n2 <= m2; ++n2) {
                double r2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double dk = d0[k] - (n0 * g.lat[k] + n1 * g.lat[3 + k] + n2 * g.lat[6 + k]);
                    r2 += dk * dk;
                }
                if (sqrt(r2) < reach) {
                    if (FILL)
                        img[o + n] = (n0 & 0xff) | ((n1 & 0xff) << 8) | ((n2 & 0xff) << 16);
                    ++n;
                }
            }
    if (!FILL)
        cnt[t] = n;
}

// entries with at least one image: atom, first image, image count; per
// projector atom its entry range (ecnt[a] counts)
__global__ __launch_bounds__(256) void k_pb_entries(int npa, int natom, const int *__restrict__ cnt,
                                                    const int *__restrict__ ioff, const int *__restrict__ eoff,
                                                    int *__restrict__ ent)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)npa * natom || cnt[t] == 0)
        return;
    const int e = eoff[t];
    ent[3 * e] = (int)(t % natom);
    ent[3 * e + 1] = ioff[t];
    ent[3 * e + 2] = cnt[t];
}

hipError_t launch_pb_images(hipStream_t s, const Geo &g, const Basis &b, int npa, const int *pint, const double *prb,
                            const int *m, int *cnt, const int *off, int *img)
{
    const long long n = (long long)npa * g.natom;
    if (n <= 0)
        return hipSuccess;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    if (img)
        hipLaunchKernelGGL(k_pb_images<true>, dim3(nblk), dim3(256), 0, s, g, b, npa, pint, prb, m[0], m[1], m[2],
                           cnt, off, img);
    else
        hipLaunchKernelGGL(k_pb_images<false>, dim3(nblk), dim3(256), 0, s, g, b, npa, pint, prb, m[0], m[1], m[2],
                           cnt, off, img);
    return hipGetLastError();
}

hipError_t launch_pb_entries(hipStream_t s, int npa, int natom, const int *cnt, const int *ioff, const int *eoff,
                             int *ent)
{
    const long long n = (long long)npa * natom;
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pb_entries, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, npa, natom, cnt, ioff, eoff,
                       ent);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The overlaps.  Workgroup (a, gi) takes the gi-th group of kPBGroup
// neighbour entries of projector atom a (ngrp groups per atom, the last
// ones possibly empty), so that each atom's work spreads over several
// compute units.  Projector atom a: internal index pint[a], input index
// pin[a], first row prow[a] of Q, entries eptr[a] .. eptr[a+1] of ent
// (orbital atom J internal, first image, image count).  prad / psp: the
// projector radials and per-species projector tables (DevSpecies of the
// projectors: rad0, nrad, norb = projectors, rc = rb); pcoef their spline
// coefficients.  pos: positions as given (input order) for the phase.
// Q: nproj x norb complex (re, im), zero outside the written blocks.
__global__ __launch_bounds__(64 * kPBWaves) void k_psibeta(
    Geo g, Basis bs, const DevRadial *__restrict__ prad, const DevSpecies *__restrict__ psp,
    const double *__restrict__ pcoef, int nprad, int npa, const int *__restrict__ pint, const int *__restrict__ pin,
    const int *__restrict__ prow, const int *__restrict__ eptr, const int *__restrict__ ent,
    const int *__restrict__ img, const double *__restrict__ pos, int nang, const double *__restrict__ ang, int nrq,
    const double *__restrict__ rq, double A0, double A1, double A2, int norb, int ngrp, double *__restrict__ Q)
{
    constexpr int CH = kPBChunk;
    __shared__ DevRadial s_rad[kMaxRadTotal], s_prad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    // dynamic LDS: [re, im][CH][16] W e^{-iA.r} beta at the chunk's points,
    // then [wave][CH][16] phit of one neighbour per wave
    extern __shared__ __align__(16) double s_dyn[];
    double(*s_B)[CH][kMaxOrb] = reinterpret_cast<double(*)[CH][kMaxOrb]>(s_dyn);
    double(*s_phi)[CH][kMaxOrb] = reinterpret_cast<double(*)[CH][kMaxOrb]>(s_dyn + 2 * CH * kMaxOrb);
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int t = xcd_batch(blockIdx.x, 0, npa * ngrp);  // consecutive groups of one atom share an XCD
    const int a = t < 0 ? -1 : t / ngrp, gi = t < 0 ? 0 : t - a * ngrp;
    for (int k = tid; k < g.nrad; k += 64 * kPBWaves)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < nprad; k += 64 * kPBWaves)
        s_prad[k] = prad[k];
    for (int k = tid; k < g.nspecies; k += 64 * kPBWaves)
        s_sp[k] = bs.sp[k];
    __syncthreads();
    if (a < 0)
        return;
    const int I = pint[a];
    const DevSpecies P = psp[bs.spc[I]];
    const double rb = P.rc;
    const double X[3] = {bs.xw[3 * I], bs.xw[3 * I + 1], bs.xw[3 * I + 2]};
    const int Iin = pin[a];
    const double T[3] = {pos[3 * Iin], pos[3 * Iin + 1], pos[3 * Iin + 2]};
    const int npts = nang * nrq;
    const int nchunk = (npts + CH - 1) / CH;
    const int e0 = eptr[a] + gi * kPBGroup, e1 = min(eptr[a + 1], e0 + kPBGroup);
    if (e0 >= e1)
        return;
    double(*phw)[kMaxOrb] = s_phi[wave];

    {
        const int g0 = e0;
        typedef MM<double>::acc acc_t;
        acc_t cre[kPBPerWave], cim[kPBPerWave];
#pragma unroll
        for (int u = 0; u < kPBPerWave; ++u)
            cre[u] = cim[u] = MM<double>::zero();
        for (int c = 0; c < nchunk; ++c) {
            __syncthreads();  // every wave is done with the previous chunk's table
            if (wave == 0) {
                const int qg = c * CH + lane;
                double *row = s_B[0][lane];
                const int swz = lane & 15;
                for (int o = 0; o < kMaxOrb; ++o)
                    row[o] = 0.0;
                if (qg < npts) {
                    const int i = qg / nang, j = qg - i * nang;
                    const double r = rb * rq[2 * i];
                    const double W = rb * rq[2 * i + 1] * r * r * ang[4 * j + 3];
                    const double x[3] = {r * ang[4 * j], r * ang[4 * j + 1], r * ang[4 * j + 2]};
                    const double zero[3] = {0.0, 0.0, 0.0};
                    // beta at x: one image at the centre
                    eval_orbitals<double, 1>(g, s_prad, P.rad0, P.rad0 + P.nrad, rb, pcoef, zero, 1, 0, 0, img, x,
                                             row, swz);
                    const double th = -(A0 * (T[0] + x[0]) + A1 * (T[1] + x[1]) + A2 * (T[2] + x[2]));
                    double sn, cs;
                    sincos(th, &sn, &cs);
                    for (int o = 0; o < kMaxOrb; ++o) {
                        const double b = row[o];
                        row[o] = W * cs * b;
                        s_B[1][lane][o] = W * sn * b;
                    }
                } else {
                    for (int o = 0; o < kMaxOrb; ++o)
                        s_B[1][lane][o] = 0.0;
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kPBPerWave; ++u) {
                const int e = g0 + wave + kPBWaves * u;
                if (e < e1) {  // (no early exit: keeps the accumulators in registers)
                const int J = ent[3 * e], io = ent[3 * e + 1], cnt = ent[3 * e + 2];
                const DevSpecies &S = s_sp[bs.spc[J]];
                // phit_J at this lane's point (the point relative to the
                // wrapped position of I; phit is periodic)
                wave_lds_sync();  // the previous neighbour's operand reads are done
                {
                    const int qg = c * CH + lane;
                    double *row = phw[lane];
                    const int swz = lane & 15;
                    for (int o = qg < npts ? S.norb : 0; o < kMaxOrb; ++o)
                        row[o ^ swz] = 0.0;
                    if (qg < npts) {
                        const int i = qg / nang, j = qg - i * nang;
                        const double r = rb * rq[2 * i];
                        const double pt[3] = {X[0] + r * ang[4 * j], X[1] + r * ang[4 * j + 1],
                                              X[2] + r * ang[4 * j + 2]};
                        const double XJ[3] = {bs.xw[3 * J], bs.xw[3 * J + 1], bs.xw[3 * J + 2]};
                        eval_orbitals<double, 1>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, XJ, cnt, img[io],
                                                 io, img, pt, row, swz);
                    }
                }
                wave_lds_sync();
#pragma unroll
                for (int kk = 0; kk < CH / 4; ++kk) {
                    const int q = 4 * kk + lk;
                    const int o = li ^ (q & 15);
                    const double bv = phw[q][o];
                    cre[u] = MM<double>::mma(s_B[0][q][o], bv, cre[u]);
                    cim[u] = MM<double>::mma(s_B[1][q][o], bv, cim[u]);
                }
                }
            }
        }
        // this pass's blocks: rows of the projectors of I, columns of J
#pragma unroll
        for (int u = 0; u < kPBPerWave; ++u) {
            const int e = g0 + wave + kPBWaves * u;
            if (e >= e1)
                continue;
            const int J = ent[3 * e];
            const int Jin = bs.perm[J];
            const int nu0 = bs.orb0[Jin], nJ = bs.orb0[Jin + 1] - nu0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int p = MM<double>::row(lk, v);
                if (p < P.norb && li < nJ) {
                    double2 *o = reinterpret_cast<double2 *>(Q) + (size_t)(prow[a] + p) * norb + nu0 + li;
                    *o = double2{cre[u][v], cim[u][v]};
                }
            }
        }
    }
}

hipError_t launch_psibeta(hipStream_t s, const Geo &g, const Basis &b, const DevRadial *prad, const DevSpecies *psp,
                          const double *pcoef, int nprad, int npa, const int *pint, const int *pin, const int *prow,
                          const int *eptr, const int *ent, const int *img, const double *pos, int nang,
                          const double *ang, int nrq, const double *rq, const double *A, int norb, int max_entries,
                          double *Q)
{
    if (npa <= 0 || max_entries <= 0)
        return hipSuccess;
    const int ngrp = (max_entries + kPBGroup - 1) / kPBGroup;
    const long long nw = (long long)npa * ngrp;
    const unsigned nblk = (unsigned)(kXcd * ((nw + kXcd - 1) / kXcd));
    const size_t lds = sizeof(double) * (2 + kPBWaves) * kPBChunk * kMaxOrb;
    const hipError_t e =
        hipFuncSetAttribute((const void *)k_psibeta, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_psibeta, dim3(nblk), dim3(64 * kPBWaves), lds, s, g, b, prad, psp, pcoef, nprad, npa, pint,
                       pin, prow, eptr, ent, img, pos, nang, ang, nrq, rq, A[0], A[1], A[2], norb, ngrp, Q);
    return hipGetLastError();
}

}  // namespace gint
