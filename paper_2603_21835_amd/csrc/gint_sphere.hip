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
// The paper batches per projector atom and reduces over quadrature points
// with wave and shared-memory reductions.  Here the sum over quadrature
// points is a dense contraction and runs on the FP64 matrix cores: a table
// pass writes W e^{-iA.r} beta_p at every grid point of every projector atom,
// then one wave per (projector atom, neighbouring atom) pair streams the
// table and the neighbour's orbitals at the same points, 64 at a time, into
// two 16 x 16 accumulators (real and imaginary parts).
#include <hip/hip_runtime.h>

#include "gint_device.h"

namespace gint {

namespace {

constexpr int kPBWaves = 4;   // one neighbour entry per wave
constexpr int kPBChunk = 64;  // quadrature points per chunk (one per lane)

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

// ---------------------------------------------------------------------------
// The overlaps, in two kernels.
//
// k_pb_table: one thread per (projector atom a, quadrature point q) writes
// W_q e^{-i A.(tau_I + x_q)} beta_p(x_q) for the atom's projectors p as
// (re, im) pairs: tab[(a npts + q) nps + p].  prad / psp: the projector
// radials and per-species tables (DevSpecies of the projectors: rad0, nrad,
// norb = projectors, rc = rb); pcoef their spline coefficients; pos the
// positions as given (input order, for the phase).
//
// k_psibeta: one wave per neighbour entry e = (projector atom a, orbital
// atom J with its images), four waves per workgroup, consecutive entries
// (the same projector atom) on one XCD.  Per chunk of 64 points the wave
// evaluates phit_J at the points (one lane per point, one spline
// evaluation per radial) into its own LDS rows and contracts them with the
// table's rows on the FP64 matrix cores (A: the table, real and imaginary
// parts; B: phit), keeping the two 16 x 16 accumulators for the whole
// quadrature grid; waves never wait for each other.  Each (a, J) block is
// written once: no atomics, repeatable bits.
__global__ __launch_bounds__(256) void k_pb_table(Geo g, Basis bs, const DevRadial *__restrict__ prad,
                                                  const DevSpecies *__restrict__ psp,
                                                  const double *__restrict__ pcoef, int nprad, int npa,
                                                  const int *__restrict__ pint, const int *__restrict__ pin,
                                                  const double *__restrict__ pos, int nang,
                                                  const double *__restrict__ ang, int nrq,
                                                  const double *__restrict__ rq, double A0, double A1, double A2,
                                                  int nps, double2 *__restrict__ tab)
{
    __shared__ DevRadial s_prad[kMaxRadTotal];
    __shared__ double s_row[256][kMaxOrb];
    for (int k = threadIdx.x; k < nprad; k += 256)
        s_prad[k] = prad[k];
    __syncthreads();
    const int npts = nang * nrq;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)npa * npts)
        return;
    const int a = (int)(t / npts), q = (int)(t - (long long)a * npts);
    const DevSpecies P = psp[bs.spc[pint[a]]];
    const double rb = P.rc;
    const int i = q / nang, j = q - i * nang;
    const double r = rb * rq[2 * i];
    const double W = rb * rq[2 * i + 1] * r * r * ang[4 * j + 3];
    const double x[3] = {r * ang[4 * j], r * ang[4 * j + 1], r * ang[4 * j + 2]};
    const double zero[3] = {0.0, 0.0, 0.0};
    double *row = s_row[threadIdx.x];
    for (int o = 0; o < kMaxOrb; ++o)
        row[o] = 0.0;
    // beta at x: one image at the centre
    eval_orbitals<double, 1>(g, s_prad, P.rad0, P.rad0 + P.nrad, rb, pcoef, zero, 1, 0, 0, nullptr, x, row, 0);
    const int Iin = pin[a];
    const double th = -(A0 * (pos[3 * Iin] + x[0]) + A1 * (pos[3 * Iin + 1] + x[1]) + A2 * (pos[3 * Iin + 2] + x[2]));
    double sn, cs;
    sincos(th, &sn, &cs);
    double2 *o = tab + (size_t)t * nps;
    for (int p = 0; p < nps; ++p)
        o[p] = p < P.norb ? double2{W * cs * row[p], W * sn * row[p]} : double2{0.0, 0.0};
}

__global__ __launch_bounds__(64 * kPBWaves) void k_psibeta(Geo g, Basis bs, const DevSpecies *__restrict__ psp,
                                                          int nent, const int *__restrict__ pint,
                                                          const int *__restrict__ prow, const int4 *__restrict__ ent,
                                                          const int *__restrict__ img, int nang,
                                                          const double *__restrict__ ang, int nrq,
                                                          const double *__restrict__ rq, int nps,
                                                          const double2 *__restrict__ tab, int norb,
                                                          double *__restrict__ Q)
{
    constexpr int CH = kPBChunk;
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ double s_phi[kPBWaves][CH][kMaxOrb];  // phit of the wave's neighbour at the chunk's points
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    for (int k = tid; k < g.nrad; k += 64 * kPBWaves)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += 64 * kPBWaves)
        s_sp[k] = bs.sp[k];
    __syncthreads();
    const int nwg = (nent + kPBWaves - 1) / kPBWaves;
    const int wg = xcd_batch(blockIdx.x, 0, nwg);
    const int e = wg * kPBWaves + wave;
    if (wg < 0 || e >= nent)
        return;
    const int4 en = ent[e];  // (orbital atom J, first image, image count, projector atom a)
    const int J = en.x, io = en.y, cnt = en.z, a = en.w;
    const int I = pint[a];
    const DevSpecies P = psp[bs.spc[I]];
    const double rb = P.rc;
    const double X[3] = {bs.xw[3 * I], bs.xw[3 * I + 1], bs.xw[3 * I + 2]};
    const double XJ[3] = {bs.xw[3 * J], bs.xw[3 * J + 1], bs.xw[3 * J + 2]};
    const DevSpecies &S = s_sp[bs.spc[J]];
    const int npts = nang * nrq;
    const int nchunk = (npts + CH - 1) / CH;
    const int pk0 = img[io];
    const double2 *ta = tab + (size_t)a * npts * nps;
    double(*phw)[kMaxOrb] = s_phi[wave];
    const bool prow_ok = li < P.norb;  // this lane's table row (projector li) exists
    typedef MM<double>::acc acc_t;
    acc_t cre = MM<double>::zero(), cim = MM<double>::zero();
    for (int c = 0; c < nchunk; ++c) {
        // phit_J at this lane's point (relative to the wrapped position of
        // the projector atom; phit is periodic)
        wave_lds_sync();  // the previous chunk's operand reads are done
        {
            const int qg = c * CH + lane;
            double *row = phw[lane];
            const int swz = lane & 15;
            for (int o = qg < npts ? S.norb : 0; o < kMaxOrb; ++o)
                row[o ^ swz] = 0.0;
            if (qg < npts) {
                const int i = qg / nang, j = qg - i * nang;
                const double r = rb * rq[2 * i];
                const double pt[3] = {X[0] + r * ang[4 * j], X[1] + r * ang[4 * j + 1], X[2] + r * ang[4 * j + 2]};
                eval_orbitals<double, 1, 4>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, XJ, cnt, pk0, io,
                                            img, pt, row, swz);
            }
        }
        // the chunk's table values of this lane (loaded after the evaluation:
        // fewer live registers, three waves per SIMD)
        double2 av[CH / 4];
#pragma unroll
        for (int kk = 0; kk < CH / 4; ++kk) {
            const int q = c * CH + 4 * kk + lk;
            av[kk] = (prow_ok && q < npts) ? ta[(size_t)q * nps + li] : double2{0.0, 0.0};
        }
        wave_lds_sync();
#pragma unroll
        for (int kk = 0; kk < CH / 4; ++kk) {
            const int q = 4 * kk + lk;
            const double bv = phw[q][li ^ (q & 15)];
            cre = MM<double>::mma(av[kk].x, bv, cre);
            cim = MM<double>::mma(av[kk].y, bv, cim);
        }
    }
    // rows of the projectors of I, columns of the orbitals of J
    const int Jin = bs.perm[J];
    const int nu0 = bs.orb0[Jin], nJ = bs.orb0[Jin + 1] - nu0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int p = MM<double>::row(lk, v);
        if (p < P.norb && li < nJ) {
            double2 *o = reinterpret_cast<double2 *>(Q) + (size_t)(prow[a] + p) * norb + nu0 + li;
            *o = double2{cre[v], cim[v]};
        }
    }
}

hipError_t launch_psibeta(hipStream_t s, const Geo &g, const Basis &b, const DevRadial *prad, const DevSpecies *psp,
                          const double *pcoef, int nprad, int npa, const int *pint, const int *pin, const int *prow,
                          const int4 *ent, int nent, const int *img, const double *pos, int nang, const double *ang,
                          int nrq, const double *rq, const double *A, int nps, void *tab, int norb, double *Q)
{
    if (npa <= 0 || nent <= 0)
        return hipSuccess;
    const long long nt = (long long)npa * nang * nrq;
    hipLaunchKernelGGL(k_pb_table, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, g, b, prad, psp, pcoef, nprad,
                       npa, pint, pin, pos, nang, ang, nrq, rq, A[0], A[1], A[2], nps,
                       static_cast<double2 *>(tab));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int nwg = (nent + kPBWaves - 1) / kPBWaves;
    const unsigned nblk = (unsigned)(kXcd * ((nwg + kXcd - 1) / kXcd));
    hipLaunchKernelGGL(k_psibeta, dim3(nblk), dim3(64 * kPBWaves), 0, s, g, b, psp, nent, pint, prow, ent, img, nang,
                       ang, nrq, rq, nps, static_cast<const double2 *>(tab), norb, Q);
    return hipGetLastError();
}

}  // namespace gint
