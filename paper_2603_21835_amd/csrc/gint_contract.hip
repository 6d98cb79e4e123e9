// gint_contract.hip -- the grid contractions of Sec. 3.3.1 of arXiv:2603.21835
// on gfx950 matrix cores (v_mfma_f64_16x16x4), and their reductions.
//
//   H^loc   output-stationary over atom-pair blocks: a workgroup owns a pair
//           of 4-atom groups and streams the mesh batches both reach, so H
//           leaves the chip once (k_pairs_H, k_H_convert).
//   rho     point-stationary: a workgroup owns a mesh batch, evaluates every
//           atom's folded orbitals there once into LDS and contracts all
//           atom-pair blocks against packed D + D^T fragments (k_rho_batch).
//   force   point-stationary likewise: T_I = sum_J (D + D^T)_IJ phi_J per
//           batch, dotted with grad phi_I; per-(batch, atom) partials are
//           summed per atom in a fixed order (k_force_batch, k_force_reduce).
//
// MFMA lane layouts (lane l, checked on gfx950 with a lane-layout probe):
//   operands   A[i][k], B[k][j] with i, j = l & 15, k = l >> 4
//   result     C[i][j] with i = (l >> 4) + 4 v, j = l & 15, v < 4
// Orbital tiles in LDS: [atom slot][point][orbital], row pitch kRow doubles.
#include <hip/hip_runtime.h>

#include "gint_device.h"

namespace gint {

// ---------------------------------------------------------------------------
// H: group-pair workgroups.
//
// Workgroup = (group pair (A, B), chunk of A's batch list); 4 waves.  Wave w
// owns the row atom I = 4A + w and the blocks (I, J = 4B + j), j = 0..3 (for
// A == B only j >= w).  The workgroup first filters its chunk of A's batch
// list for batches that B also reaches and records, for each kept batch, the
// batch coordinates and the image lists of its <= 8 atoms (slots 0-3: group
// A, 4-7: group B).  Per kept batch it stages the folded orbitals of the 8
// slots at the batch's points into LDS and each wave accumulates
// C_IJ += (w phi_I)^T phi_J over the points on the matrix cores.

constexpr int kNL = 128;  // candidate batches per filter round

__global__ __launch_bounds__(256) void k_pairs_H(Geo g, Bins bn, Basis bs, int nchunk, const double *__restrict__ W,
                                                 double wscale, double *__restrict__ out)
{
    constexpr int PT = 32;  // points staged per step (a whole batch)
    __shared__ double s_phi[8][PT][kRow];
    __shared__ double s_w[PT];
    __shared__ double s_X[8][3];
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ int s_k0[8], s_k1[8], s_norb[8];
    __shared__ double s_rc[8];
    __shared__ int s_bi[3][kNL];
    __shared__ int s_icnt[8][kNL], s_ipk[8][kNL], s_ioff[8][kNL];
    __shared__ int s_wcnt[4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int pair = blockIdx.x / nchunk, chunk = blockIdx.x % nchunk;
    const int A = bn.pairA[pair], B = bn.pairB[pair];
    const bool diag = (A == B);
    const int natom = g.natom;
    const bool Iex = A * kGroup + wave < natom;

    for (int k = tid; k < g.nrad; k += 256)
        s_rad[k] = bs.rad[k];
    if (tid < 8) {
        const int atom = (tid < 4) ? A * kGroup + tid : B * kGroup + (tid - 4);
        const bool ok = atom < natom && !(diag && tid >= 4);
        if (ok) {
            const DevSpecies S = bs.sp[bs.spc[atom]];
            s_X[tid][0] = bs.xw[3 * atom];
            s_X[tid][1] = bs.xw[3 * atom + 1];
            s_X[tid][2] = bs.xw[3 * atom + 2];
            s_k0[tid] = S.rad0;
            s_k1[tid] = S.rad0 + S.nrad;
            s_norb[tid] = S.norb;
            s_rc[tid] = S.rc;
        } else {
            s_X[tid][0] = s_X[tid][1] = s_X[tid][2] = 0.0;
            s_k0[tid] = s_k1[tid] = 0;
            s_norb[tid] = 0;
            s_rc[tid] = 0.0;
        }
    }

    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        acc[j] = d4{0.0, 0.0, 0.0, 0.0};

    const int st_s = tid / PT, st_p = tid % PT;
    const int gb0 = bn.gptr[A], gb1 = bn.gptr[A + 1];
    const long long len = gb1 - gb0;
    const int c0 = gb0 + (int)(len * chunk / nchunk);
    const int c1 = gb0 + (int)(len * (chunk + 1) / nchunk);
    __syncthreads();

    for (int base = c0; base < c1; base += kNL) {
        // ---- filter: batches of this chunk that group B also reaches ----
        bool keep = false;
        int b = -1, e_a = 0, e_b = 0, e_end = 0;
        if (tid < kNL && base + tid < c1) {
            b = bn.gbatch[base + tid];
            const int e0 = bn.bptr[b];
            e_end = bn.bptr[b + 1];
            e_a = lower_bound_i(bn.ent_atom, e0, e_end, A * kGroup);
            if (diag) {
                keep = true;
            } else {
                e_b = lower_bound_i(bn.ent_atom, e_a, e_end, B * kGroup);
                keep = e_b < e_end && bn.ent_atom[e_b] < (B + 1) * kGroup;
            }
        }
        const unsigned long long m = __ballot(keep);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0)
            s_wcnt[wave] = __popcll(m);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; ++w)
            off += s_wcnt[w];
        const int nlist = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
        if (keep) {
            const int q = off + pre;
            int ib[3];
            batch_coords(g, b, ib);
            s_bi[0][q] = ib[0];
            s_bi[1][q] = ib[1];
            s_bi[2][q] = ib[2];
            int ea = e_a, eb = e_b;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int grp = (s < 4) ? A : B;
                int &e = (s < 4) ? ea : eb;
                int cnt = 0, pk = 0, io = 0;
                if (!(diag && s >= 4) && e < e_end && bn.ent_atom[e] == grp * kGroup + (s & 3)) {
                    io = bn.ent_img[e];
                    cnt = bn.ent_img[e + 1] - io;
                    pk = bn.img[io];
                    ++e;
                }
                s_icnt[s][q] = cnt;
                s_ipk[s][q] = pk;
                s_ioff[s][q] = io;
            }
        }
        __syncthreads();

        // weight of this thread's point in the first kept batch
        double wnext = 0.0;
        if (tid < PT && nlist > 0) {
            const int ib[3] = {s_bi[0][0], s_bi[1][0], s_bi[2][0]};
            int n[3];
            if (batch_point(g, ib, tid, n))
                wnext = wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]];
        }

        for (int it = 0; it < nlist; ++it) {
            // ---- stage the folded orbitals (PhiOperator) ----
            {
                double *row = &s_phi[st_s][st_p][0];
                const int ib[3] = {s_bi[0][it], s_bi[1][it], s_bi[2][it]};
                int n[3];
                const bool valid = batch_point(g, ib, st_p, n);
                const int icnt = valid ? s_icnt[st_s][it] : 0;
                const int zlo = (icnt > 0) ? s_norb[st_s] : 0;
                for (int o = zlo; o < kMaxOrb; ++o)
                    row[o] = 0.0;
                if (icnt > 0) {
                    double r[3];
                    mesh_cart(g, n, r);
                    eval_orbitals<false>(g, s_rad, s_k0[st_s], s_k1[st_s], s_rc[st_s], bs.coef, s_X[st_s], icnt,
                                         s_ipk[st_s][it], s_ioff[st_s][it], bn.img, r, row, nullptr, nullptr,
                                         nullptr);
                }
                if (tid < PT)
                    s_w[tid] = wnext;
            }
            __syncthreads();
            // prefetch the next batch's weight while the matrix cores run
            if (tid < PT && it + 1 < nlist) {
                const int ib[3] = {s_bi[0][it + 1], s_bi[1][it + 1], s_bi[2][it + 1]};
                int n[3];
                wnext = batch_point(g, ib, tid, n) ? wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 0.0;
            }

            // ---- contraction on the matrix cores ----
            if (Iex && s_icnt[wave][it] > 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int sj = diag ? j : 4 + j;
                    if ((!diag || j >= wave) && s_icnt[sj][it] > 0) {
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
            __syncthreads();
        }
    }

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
}

hipError_t launch_pairs_H(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int npair, int nchunk,
                          const double *W, double wscale, double *Hblk)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pairs_H, dim3(npair * nchunk), dim3(256), 0, s, g, bn, b, nchunk, W, wscale, Hblk);
    return hipGetLastError();
}

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

// ---------------------------------------------------------------------------
// D + D^T packed as MFMA A-operand fragments, for every canonical atom-pair
// block (X, Y) of every active group pair (X = 4A + sX, Y = 4B + sY, with
// sX <= sY when A == B), in two orientations:
//   orient 0: lane l, chunk c holds S2_XY[l & 15][4c + (l >> 4)]   (S2_XY as A)
//   orient 1: lane l, chunk c holds S2_XY[4c + (l >> 4)][l & 15]   (S2_YX as A)
// so each lane reads its four values of a block with two 16-byte loads.

__global__ __launch_bounds__(256) void k_pack_S2(Geo g, Bins bn, Basis bs, const double *__restrict__ D, int norb,
                                                 double *__restrict__ pk)
{
    const int pair = blockIdx.x >> 4, blk = blockIdx.x & 15;
    const int A = bn.pairA[pair], B = bn.pairB[pair];
    const int sX = blk >> 2, sY = blk & 3;
    const int X = A * kGroup + sX, Y = B * kGroup + sY;
    const int t = threadIdx.x, c = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
    const bool ok = X < g.natom && Y < g.natom && !(A == B && sX > sY);
    double v0 = 0.0, v1 = 0.0;
    if (ok) {
        const int Xin = bs.perm[X], Yin = bs.perm[Y];
        const int mx = bs.orb0[Xin], nx = bs.orb0[Xin + 1] - mx;
        const int my = bs.orb0[Yin], ny = bs.orb0[Yin + 1] - my;
        const int kb = 4 * c + lk;
        if (li < nx && kb < ny)
            v0 = D[(size_t)(mx + li) * norb + my + kb] + D[(size_t)(my + kb) * norb + mx + li];
        if (kb < nx && li < ny)
            v1 = D[(size_t)(mx + kb) * norb + my + li] + D[(size_t)(my + li) * norb + mx + kb];
    }
    const size_t base = (size_t)blockIdx.x * 512;
    pk[base + t] = v0;
    pk[base + 256 + t] = v1;
}

hipError_t launch_pack_S2(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int npair, const double *D,
                          int norb, double *pk)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pack_S2, dim3(npair * 16), dim3(256), 0, s, g, bn, b, D, norb, pk);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Point-stationary kernels: one workgroup per mesh batch, 16-point tiles.

// Per-batch setup shared by rho and force: radial and species tables, the
// batch's atoms and their group ranks, and the pair ids of the batch's group
// pairs (canonical order).
template <bool FORCE>
__global__ __launch_bounds__(256) void k_batch(Geo g, Bins bn, Basis bs, const double *__restrict__ pk,
                                               const double *__restrict__ W, double wscale, double *__restrict__ out)
{
    extern __shared__ double s_phi[];  // [nbmax][16][kRow]
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_grank[kMaxBatchAtoms];
    __shared__ int s_ptab[kMaxBatchGroups * kMaxBatchGroups];
    __shared__ double s_red[4][16];
    __shared__ double s_w[16];
    __shared__ double s_F[FORCE ? kMaxBatchAtoms : 1][3];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int b = blockIdx.x;
    const int e0 = bn.bptr[b], nb = bn.bptr[b + 1] - e0;
    const int g0 = bn.bgptr[b], ngb = bn.bgptr[b + 1] - g0;
    int ib[3];
    batch_coords(g, b, ib);

    for (int k = tid; k < g.nrad; k += 256)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += 256)
        s_sp[k] = bs.sp[k];
    for (int a = tid; a < nb; a += 256) {
        const int atom = bn.ent_atom[e0 + a];
        s_atom[a] = atom;
        s_grank[a] = lower_bound_i(bn.bgrp, g0, g0 + ngb, atom / kGroup) - g0;
        if (FORCE)
            s_F[a][0] = s_F[a][1] = s_F[a][2] = 0.0;
    }
    for (int k = tid; k < ngb * ngb; k += 256) {
        const int ra = k / ngb, rb = k % ngb;
        const int ga = bn.bgrp[g0 + ra], gb = bn.bgrp[g0 + rb];
        s_ptab[k] = (ra <= rb) ? bn.pair_index[(size_t)ga * g.ngroup + gb] : -1;
    }
    __syncthreads();

    for (int sub = 0; sub < g.P; sub += 16) {
        // ---- stage the folded orbitals of every atom of the batch ----
        for (int idx = tid; idx < nb * 16; idx += 256) {
            const int a = idx >> 4, p = idx & 15;
            const int e = e0 + a;
            const int atom = s_atom[a];
            double *row = s_phi + (size_t)(a * 16 + p) * kRow;
            int n[3];
            const bool valid = batch_point(g, ib, sub + p, n);
            const DevSpecies &S = s_sp[bs.spc[atom]];
            const int zlo = valid ? S.norb : 0;
            for (int o = zlo; o < kMaxOrb; ++o)
                row[o] = 0.0;
            if (valid) {
                const int io = bn.ent_img[e];
                const int cnt = bn.ent_img[e + 1] - io;
                const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
                double r[3];
                mesh_cart(g, n, r);
                eval_orbitals<false>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, cnt, bn.img[io], io,
                                     bn.img, r, row, nullptr, nullptr, nullptr);
            }
        }
        if (FORCE && tid < 16) {
            int n[3];
            s_w[tid] = batch_point(g, ib, sub + tid, n) ? wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 0.0;
        }
        __syncthreads();

        if (!FORCE) {
            // rho_p = sum_{I<J} phi_I . (S2_IJ phi_J) + 1/2 sum_I phi_I . (S2_II phi_I)
            double rp = 0.0;
            const int nblk = nb * (nb + 1) / 2;
            int ia = 0, ja = 0;
            for (int k = 0; k < wave; ++k)
                if (++ja == nb) {
                    ++ia;
                    ja = ia;
                }
            for (int k = wave; k < nblk; k += 4) {
                const int I = s_atom[ia], J = s_atom[ja];
                const int pr = s_ptab[s_grank[ia] * ngb + s_grank[ja]];  // active: both groups are here
                const int blk = (I % kGroup) * 4 + (J % kGroup);
                const double *f = pk + ((size_t)(pr * 16 + blk) * 2) * 256 + lane;
                const double fa0 = f[0], fa1 = f[64], fa2 = f[128], fa3 = f[192];
                const double *pJ = s_phi + (size_t)(ja * 16 + li) * kRow + lk;
                d4 u = d4{0.0, 0.0, 0.0, 0.0};
                u = __builtin_amdgcn_mfma_f64_16x16x4f64(fa0, pJ[0], u, 0, 0, 0);
                u = __builtin_amdgcn_mfma_f64_16x16x4f64(fa1, pJ[4], u, 0, 0, 0);
                u = __builtin_amdgcn_mfma_f64_16x16x4f64(fa2, pJ[8], u, 0, 0, 0);
                u = __builtin_amdgcn_mfma_f64_16x16x4f64(fa3, pJ[12], u, 0, 0, 0);
                const double *pI = s_phi + (size_t)(ia * 16 + li) * kRow + lk;
                const double dot = u[0] * pI[0] + u[1] * pI[4] + u[2] * pI[8] + u[3] * pI[12];
                rp += (ia == ja) ? 0.5 * dot : dot;
                for (int s = 0; s < 4; ++s)
                    if (++ja == nb) {
                        ++ia;
                        ja = ia;
                    }
            }
            rp += __shfl_xor(rp, 16);
            rp += __shfl_xor(rp, 32);
            if (lane < 16)
                s_red[wave][lane] = rp;
            __syncthreads();
            if (tid < 16) {
                int n[3];
                if (batch_point(g, ib, sub + tid, n))
                    out[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] =
                        ((s_red[0][tid] + s_red[1][tid]) + s_red[2][tid]) + s_red[3][tid];
            }
        } else {
            // dE/dR_I partial = -sum_p w_p grad phi_I(p) . T_I(p),  T_I = sum_J S2_IJ phi_J
            int n[3];
            const bool pvalid = batch_point(g, ib, sub + li, n);
            double r[3];
            mesh_cart(g, n, r);
            const double wp = s_w[li];
            for (int ia = wave; ia < nb; ia += 4) {
                const int I = s_atom[ia];
                d4 T = d4{0.0, 0.0, 0.0, 0.0};
                for (int ja = 0; ja < nb; ++ja) {
                    const int J = s_atom[ja];
                    const bool fwd = ia <= ja;
                    const int ra = fwd ? s_grank[ia] : s_grank[ja], rb = fwd ? s_grank[ja] : s_grank[ia];
                    const int pr = s_ptab[ra * ngb + rb];
                    const int blk = fwd ? (I % kGroup) * 4 + (J % kGroup) : (J % kGroup) * 4 + (I % kGroup);
                    const double *f = pk + ((size_t)(pr * 16 + blk) * 2 + (fwd ? 0 : 1)) * 256 + lane;
                    const double *pJ = s_phi + (size_t)(ja * 16 + li) * kRow + lk;
                    T = __builtin_amdgcn_mfma_f64_16x16x4f64(f[0], pJ[0], T, 0, 0, 0);
                    T = __builtin_amdgcn_mfma_f64_16x16x4f64(f[64], pJ[4], T, 0, 0, 0);
                    T = __builtin_amdgcn_mfma_f64_16x16x4f64(f[128], pJ[8], T, 0, 0, 0);
                    T = __builtin_amdgcn_mfma_f64_16x16x4f64(f[192], pJ[12], T, 0, 0, 0);
                }
                // gradients of orbitals lk + 4v of atom I at point li
                double gr[3][4];
                const int e = e0 + ia;
                const DevSpecies &S = s_sp[bs.spc[I]];
                const double X[3] = {bs.xw[3 * I], bs.xw[3 * I + 1], bs.xw[3 * I + 2]};
                const int io = bn.ent_img[e];
                const int cnt = pvalid ? bn.ent_img[e + 1] - io : 0;
                grad4(g, s_rad, S.orb_rad, S.orb_m, S.norb, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img, r, lk, gr);
                double fx[3];
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    double v = wp * (T[0] * gr[x][0] + T[1] * gr[x][1] + T[2] * gr[x][2] + T[3] * gr[x][3]);
                    for (int o = 32; o > 0; o >>= 1)
                        v += __shfl_xor(v, o);
                    fx[x] = v;
                }
                if (lane == 0) {
                    s_F[ia][0] -= fx[0];
                    s_F[ia][1] -= fx[1];
                    s_F[ia][2] -= fx[2];
                }
            }
        }
        __syncthreads();
    }
    if (FORCE)
        for (int k = tid; k < nb * 3; k += 256)
            out[(size_t)(e0 + k / 3) * 3 + k % 3] = s_F[k / 3][k % 3];
}

size_t batch_lds_bytes(int nbmax) { return sizeof(double) * (size_t)nbmax * 16 * kRow; }

hipError_t launch_rho_batch(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, const double *pk,
                            double *rho)
{
    const size_t lds = batch_lds_bytes(nbmax);
    hipError_t e = hipFuncSetAttribute((const void *)k_batch<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_batch<false>, dim3(g.nbatch), dim3(256), lds, s, g, bn, b, pk, (const double *)nullptr,
                       0.0, rho);
    return hipGetLastError();
}

hipError_t launch_force_batch(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                              const double *pk, const double *W, double wscale, double *Fent)
{
    const size_t lds = batch_lds_bytes(nbmax);
    hipError_t e = hipFuncSetAttribute((const void *)k_batch<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_batch<true>, dim3(g.nbatch), dim3(256), lds, s, g, bn, b, pk, W, wscale, Fent);
    return hipGetLastError();
}

// dE/dR per atom: fixed-order sum of its per-(batch, atom) partials over the
// batches of its group's list.
__global__ __launch_bounds__(256) void k_force_reduce(Geo g, Bins bn, Basis bs, const double *__restrict__ Fent,
                                                      double *__restrict__ dEdR)
{
    __shared__ double red[3][256];
    const int ii = blockIdx.x;
    const int grp = ii / kGroup;
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = bn.gptr[grp] + threadIdx.x; k < bn.gptr[grp + 1]; k += 256) {
        const int b = bn.gbatch[k];
        const int lo = bn.bptr[b], hi = bn.bptr[b + 1];
        const int e = lower_bound_i(bn.ent_atom, lo, hi, ii);
        if (e < hi && bn.ent_atom[e] == ii)
            for (int x = 0; x < 3; ++x)
                v[x] += Fent[(size_t)e * 3 + x];
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

hipError_t launch_force_reduce(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, const double *Fent,
                               double *dEdR)
{
    hipLaunchKernelGGL(k_force_reduce, dim3(g.natom), dim3(256), 0, s, g, bn, b, Fent, dEdR);
    return hipGetLastError();
}

}  // namespace gint
