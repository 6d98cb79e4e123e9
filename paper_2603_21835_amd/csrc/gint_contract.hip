// gint_contract.hip -- the grid contractions of Sec. 3.3.1 of arXiv:2603.21835
// on gfx950 matrix cores, and their reductions.  Orbital tiles, packed D and
// H block partials are FP64 (v_mfma_f64_16x16x4) or FP32
// (v_mfma_f32_16x16x4); sums across batches and all dot products are FP64.
//
//   H^loc   point-stationary: a workgroup owns a mesh batch and forms every
//           atom-pair block of it from orbitals evaluated once into LDS
//           (k_H_batch); a per-atom workgroup then sums each block over the
//           atom's batches in a fixed order into dense symmetric H
//           (k_H_rowreduce).
//   rho     point-stationary: a workgroup owns a mesh batch, evaluates every
//           atom's folded orbitals there once into LDS and contracts all
//           atom-pair blocks against packed D + D^T fragments (k_rho_batch).
//   force   point-stationary likewise: T_I = sum_J (D + D^T)_IJ phi_J per
//           batch, dotted with grad phi_I; per-(batch, atom) partials are
//           summed per atom in a fixed order (k_force_batch, k_force_reduce).
//
// MFMA lane layouts: see MM<T> in gint_device.h.
// Orbital tiles in LDS: [atom slot][point][orbital], row pitch kRow elements.
#include <hip/hip_runtime.h>

#include "gint_device.h"

namespace gint {

// ---------------------------------------------------------------------------
// H^loc, point-stationary.
//
// k_H_batch: one workgroup per mesh batch evaluates the folded orbitals of
// every atom reaching the batch once (all P points in LDS) and forms every
// atom-pair block (ia <= ja in the batch's atom order)
//     C_IJ = sum_{p in batch} (w_p phi_I(p)) phi_J(p)^T
// on the matrix cores, writing it to a partial buffer (n_I x n_J of a
// mno x mno tile; block k of batch b at boff[b] + k).
//
// k_H_rowreduce: one workgroup per atom I owns the blocks (I, J) of the
// partners J it owns (each unordered pair has one owner) and sums their
// partials over I's batches in increasing batch order (fixed order, no
// atomics), then writes H_IJ and its mirror H_JI into the dense matrix, so
// H is exactly symmetric.

template <typename T>
__global__ __launch_bounds__(512) void k_H_batch(Geo g, Bins bn, Basis bs, const double *__restrict__ W,
                                                 double wscale, int b0, const int *__restrict__ boff, int mno,
                                                 T *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    T *s_phi = reinterpret_cast<T *>(s_dyn);  // [nbmax][P][kRow]
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_nor[kMaxBatchAtoms];
    __shared__ double s_w[kMaxP];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int b = b0 + blockIdx.x;
    const int e0 = bn.bptr[b], nb = bn.bptr[b + 1] - e0;
    const int P = g.P;
    int ib[3];
    batch_coords(g, b, ib);

    for (int k = tid; k < g.nrad; k += blockDim.x)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += blockDim.x)
        s_sp[k] = bs.sp[k];
    for (int a = tid; a < nb; a += blockDim.x) {
        const int atom = bn.ent_atom[e0 + a];
        s_atom[a] = atom;
        s_nor[a] = bs.sp[bs.spc[atom]].norb;
    }
    for (int p = tid; p < P; p += blockDim.x) {
        int n[3];
        s_w[p] = batch_point(g, ib, p, n) ? wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 0.0;
    }
    __syncthreads();

    // ---- stage the folded orbitals of every atom at every batch point ----
    for (int idx = tid; idx < nb * P; idx += blockDim.x) {
        const int a = idx / P, p = idx % P;
        const int e = e0 + a;
        const int atom = s_atom[a];
        T *row = s_phi + (size_t)(a * P + p) * kRow;
        int n[3];
        const bool valid = batch_point(g, ib, p, n);
        const DevSpecies &S = s_sp[bs.spc[atom]];
        const int zlo = valid ? S.norb : 0;
        for (int o = zlo; o < kMaxOrb; ++o)
            row[o] = (T)0;
        if (valid) {
            const int io = bn.ent_img[e];
            const int cnt = bn.ent_img[e + 1] - io;
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            double r[3];
            mesh_cart(g, n, r);
            eval_orbitals<T>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img, r,
                             row);
        }
    }
    __syncthreads();

    // ---- every block (ia <= ja), round-robin over the waves ----
    const int nblk = nb * (nb + 1) / 2;
    int ia = 0, ja = 0;
    for (int k = 0; k < wave; ++k)
        if (++ja == nb) {
            ++ia;
            ja = ia;
        }
    const size_t mm = (size_t)mno * mno;
    for (int k = wave; k < nblk; k += nw) {
        const T *pI = s_phi + (size_t)(ia * P) * kRow;
        const T *pJ = s_phi + (size_t)(ja * P) * kRow;
        typename MM<T>::acc acc = MM<T>::zero();
#pragma unroll
        for (int kk = 0; kk < kMaxP / 4; ++kk) {
            if (4 * kk < P) {
                const int p = 4 * kk + lk;
                const T av = (T)s_w[p] * pI[p * kRow + li];
                const T bv = pJ[p * kRow + li];
                acc = MM<T>::mma(av, bv, acc);
            }
        }
        const int nI = s_nor[ia], nJ = s_nor[ja];
        T *o = part + (size_t)(boff[b] - boff[b0] + k) * mm;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = MM<T>::row(lk, v);
            if (row < nI && li < nJ)
                o[row * mno + li] = acc[v];
        }
        for (int s = 0; s < nw; ++s)
            if (++ja == nb) {
                ++ia;
                ja = ia;
            }
    }
}

template <typename T>
static hipError_t launch_H_batch_t(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int b0,
                                   int b1, const double *W, double wscale, const int *boff, int mno, void *part)
{
    if (b1 <= b0)
        return hipSuccess;
    const size_t lds = sizeof(T) * (size_t)nbmax * g.P * kRow;
    hipError_t e =
        hipFuncSetAttribute((const void *)k_H_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_H_batch<T>, dim3(b1 - b0), dim3(512), lds, s, g, bn, b, W, wscale, b0, boff, mno,
                       static_cast<T *>(part));
    return hipGetLastError();
}

hipError_t launch_H_batch(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int b0,
                          int b1, const double *W, double wscale, const int *boff, int mno, void *part)
{
    return f32 ? launch_H_batch_t<float>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part)
               : launch_H_batch_t<double>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
}

constexpr int kRowChunk = 16;         // batches staged per round
constexpr int kMaxPartnerPass = 128;  // partners per pass
constexpr int kRowThreads = 1024;

__device__ __forceinline__ int tri_index(int lo, int hi, int n) { return lo * n - lo * (lo - 1) / 2 + (hi - lo); }

// Thread (partner slot sl, orbital row a of I) accumulates the row a of block
// (I, J_sl) over I's batches in increasing batch order.
template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_H_rowreduce(Geo g, Bins bn, Basis bs, AtomLists al, int mno,
                                                             int norb, const T *__restrict__ part,
                                                             const int *__restrict__ boff, int b0, int b1,
                                                             int accumulate, double *__restrict__ H)
{
    __shared__ int s_pos[kRowChunk][kMaxPartnerPass];
    __shared__ int s_part[kMaxPartnerPass];
    __shared__ int s_ia[kRowChunk], s_nb[kRowChunk], s_e0[kRowChunk], s_pb[kRowChunk];

    const int tid = threadIdx.x;
    const int I = blockIdx.x;
    const int Iin = bs.perm[I];
    const int mu0 = bs.orb0[Iin], nI = bs.orb0[Iin + 1] - mu0;
    const int np = al.pptr[I + 1] - al.pptr[I];
    const size_t mm = (size_t)mno * mno;
    // this atom's entries inside the batch range [b0, b1)
    const int ent_lo = lower_bound_i(al.aent, al.aptr[I], al.aptr[I + 1], bn.bptr[b0]);
    const int ent_hi = lower_bound_i(al.aent, al.aptr[I], al.aptr[I + 1], bn.bptr[b1]);
    int npc_max = kRowThreads / nI;
    if (npc_max > kMaxPartnerPass)
        npc_max = kMaxPartnerPass;
    const int sl = tid / nI, a = tid % nI;

    for (int s0 = 0; s0 < np; s0 += npc_max) {
        const int npc = (np - s0 < npc_max) ? np - s0 : npc_max;
        __syncthreads();
        for (int j = tid; j < npc; j += kRowThreads)
            s_part[j] = al.plist[al.pptr[I] + s0 + j];
        const bool mine = sl < npc;
        double acc[kMaxOrb];
#pragma unroll
        for (int c = 0; c < kMaxOrb; ++c)
            acc[c] = 0.0;

        for (int c0 = ent_lo; c0 < ent_hi; c0 += kRowChunk) {
            const int nk = (ent_hi - c0 < kRowChunk) ? ent_hi - c0 : kRowChunk;
            __syncthreads();
            for (int idx = tid; idx < kRowChunk * npc; idx += kRowThreads)
                s_pos[idx / npc][idx % npc] = -1;
            if (tid < nk) {
                const int e = al.aent[c0 + tid];
                const int b = al.abat[c0 + tid];
                s_e0[tid] = bn.bptr[b];
                s_ia[tid] = e - bn.bptr[b];
                s_nb[tid] = bn.bptr[b + 1] - bn.bptr[b];
                s_pb[tid] = boff[b] - boff[b0];
            }
            __syncthreads();
            // positions of this pass's partners in each staged batch
            for (int idx = tid; idx < nk * kMaxBatchAtoms; idx += kRowThreads) {
                const int k = idx / kMaxBatchAtoms, j = idx % kMaxBatchAtoms;
                if (j < s_nb[k]) {
                    const int J = bn.ent_atom[s_e0[k] + j];
                    const int f = lower_bound_i(s_part, 0, npc, J);
                    if (f < npc && s_part[f] == J)
                        s_pos[k][f] = j;
                }
            }
            __syncthreads();
            if (mine) {
                for (int k = 0; k < nk; ++k) {
                    const int ja = s_pos[k][sl];
                    if (ja < 0)
                        continue;
                    const int ia = s_ia[k];
                    if (ia <= ja) {
                        const T *src = part + (size_t)(s_pb[k] + tri_index(ia, ja, s_nb[k])) * mm + a * mno;
#pragma unroll
                        for (int c = 0; c < kMaxOrb; ++c)
                            if (c < mno)
                                acc[c] += (double)src[c];
                    } else {
                        const T *src = part + (size_t)(s_pb[k] + tri_index(ja, ia, s_nb[k])) * mm + a;
#pragma unroll
                        for (int c = 0; c < kMaxOrb; ++c)
                            if (c < mno)
                                acc[c] += (double)src[c * mno];
                    }
                }
            }
        }
        // H_IJ row a and its mirror column (diagonal blocks: c >= a, mirrored)
        if (mine) {
            const int J = s_part[sl];
            const int Jin = bs.perm[J];
            const int nu0 = bs.orb0[Jin], nJ = bs.orb0[Jin + 1] - nu0;
#pragma unroll
            for (int c = 0; c < kMaxOrb; ++c) {
                if (c < nJ && !(J == I && c < a)) {
                    const size_t i1 = (size_t)(mu0 + a) * norb + nu0 + c;
                    const size_t i2 = (size_t)(nu0 + c) * norb + mu0 + a;
                    const double v = accumulate ? H[i1] + acc[c] : acc[c];
                    H[i1] = v;
                    H[i2] = v;
                }
            }
        }
    }
}

hipError_t launch_H_rowreduce(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b,
                              const AtomLists &al, int mno, int norb, const void *part, const int *boff, int b0,
                              int b1, int accumulate, double *H)
{
    if (f32)
        hipLaunchKernelGGL(k_H_rowreduce<float>, dim3(g.natom), dim3(kRowThreads), 0, s, g, bn, b, al, mno, norb,
                           static_cast<const float *>(part), boff, b0, b1, accumulate, H);
    else
        hipLaunchKernelGGL(k_H_rowreduce<double>, dim3(g.natom), dim3(kRowThreads), 0, s, g, bn, b, al, mno, norb,
                           static_cast<const double *>(part), boff, b0, b1, accumulate, H);
    return hipGetLastError();
}

__global__ void k_fill_f64(double *p, long long n, double v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

hipError_t launch_fill_f64(hipStream_t s, double *p, long long n, double v)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// D + D^T packed as MFMA A-operand fragments, for every canonical atom-pair
// block (X, Y) of every active group pair (X = 4A + sX, Y = 4B + sY, with
// sX <= sY when A == B), in two orientations:
//   orient 0: lane l, chunk c holds S2_XY[l & 15][4c + (l >> 4)]   (S2_XY as A)
//   orient 1: lane l, chunk c holds S2_XY[4c + (l >> 4)][l & 15]   (S2_YX as A)
// so each lane reads its four values of a block with two 16-byte loads.

template <typename T>
__global__ __launch_bounds__(256) void k_pack_S2(Geo g, Bins bn, Basis bs, const double *__restrict__ D, int norb,
                                                 T *__restrict__ pk)
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
    pk[base + t] = (T)v0;
    pk[base + 256 + t] = (T)v1;
}

hipError_t launch_pack_S2(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int npair,
                          const double *D, int norb, void *pk)
{
    if (npair <= 0)
        return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_pack_S2<float>, dim3(npair * 16), dim3(256), 0, s, g, bn, b, D, norb,
                           static_cast<float *>(pk));
    else
        hipLaunchKernelGGL(k_pack_S2<double>, dim3(npair * 16), dim3(256), 0, s, g, bn, b, D, norb,
                           static_cast<double *>(pk));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Point-stationary kernels: one workgroup per mesh batch, 16-point tiles.

// Per-batch setup shared by rho and force: radial and species tables, the
// batch's atoms and their group ranks, and the pair ids of the batch's group
// pairs (canonical order).
template <bool FORCE, typename T>
__global__ __launch_bounds__(256) void k_batch(Geo g, Bins bn, Basis bs, const T *__restrict__ pk,
                                               const double *__restrict__ W, double wscale, double *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    T *s_phi = reinterpret_cast<T *>(s_dyn);  // [nbmax][16][kRow]
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
            T *row = s_phi + (size_t)(a * 16 + p) * kRow;
            int n[3];
            const bool valid = batch_point(g, ib, sub + p, n);
            const DevSpecies &S = s_sp[bs.spc[atom]];
            const int zlo = valid ? S.norb : 0;
            for (int o = zlo; o < kMaxOrb; ++o)
                row[o] = (T)0;
            if (valid) {
                const int io = bn.ent_img[e];
                const int cnt = bn.ent_img[e + 1] - io;
                const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
                double r[3];
                mesh_cart(g, n, r);
                eval_orbitals<T>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img,
                                 r, row);
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
                const T *f = pk + ((size_t)(pr * 16 + blk) * 2) * 256 + lane;
                const T fa0 = f[0], fa1 = f[64], fa2 = f[128], fa3 = f[192];
                const T *pJ = s_phi + (size_t)(ja * 16 + li) * kRow + lk;
                typename MM<T>::acc u = MM<T>::zero();
                u = MM<T>::mma(fa0, pJ[0], u);
                u = MM<T>::mma(fa1, pJ[4], u);
                u = MM<T>::mma(fa2, pJ[8], u);
                u = MM<T>::mma(fa3, pJ[12], u);
                const T *pI = s_phi + (size_t)(ia * 16 + li) * kRow;
                double dot = 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    dot += (double)u[v] * (double)pI[MM<T>::row(lk, v)];
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
                typename MM<T>::acc Tt = MM<T>::zero();
                for (int ja = 0; ja < nb; ++ja) {
                    const int J = s_atom[ja];
                    const bool fwd = ia <= ja;
                    const int ra = fwd ? s_grank[ia] : s_grank[ja], rb = fwd ? s_grank[ja] : s_grank[ia];
                    const int pr = s_ptab[ra * ngb + rb];
                    const int blk = fwd ? (I % kGroup) * 4 + (J % kGroup) : (J % kGroup) * 4 + (I % kGroup);
                    const T *f = pk + ((size_t)(pr * 16 + blk) * 2 + (fwd ? 0 : 1)) * 256 + lane;
                    const T *pJ = s_phi + (size_t)(ja * 16 + li) * kRow + lk;
                    Tt = MM<T>::mma(f[0], pJ[0], Tt);
                    Tt = MM<T>::mma(f[64], pJ[4], Tt);
                    Tt = MM<T>::mma(f[128], pJ[8], Tt);
                    Tt = MM<T>::mma(f[192], pJ[12], Tt);
                }
                // gradients of orbitals row(lk, v) of atom I at point li
                double gr[3][4];
                const int e = e0 + ia;
                const DevSpecies &S = s_sp[bs.spc[I]];
                const double X[3] = {bs.xw[3 * I], bs.xw[3 * I + 1], bs.xw[3 * I + 2]};
                const int io = bn.ent_img[e];
                const int cnt = pvalid ? bn.ent_img[e + 1] - io : 0;
                grad4(g, s_rad, S.orb_rad, S.orb_m, S.norb, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img, r,
                      MM<T>::row(lk, 0), MM<T>::row(lk, 1) - MM<T>::row(lk, 0), gr);
                double fx[3];
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    double v = wp * ((double)Tt[0] * gr[x][0] + (double)Tt[1] * gr[x][1] + (double)Tt[2] * gr[x][2] +
                                     (double)Tt[3] * gr[x][3]);
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

size_t batch_lds_bytes(int nbmax, bool f32) { return (f32 ? 4 : 8) * (size_t)nbmax * 16 * kRow; }

template <bool FORCE, typename T>
static hipError_t launch_batch_t(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                                 const void *pk, const double *W, double wscale, double *out)
{
    const size_t lds = sizeof(T) * (size_t)nbmax * 16 * kRow;
    hipError_t e =
        hipFuncSetAttribute((const void *)k_batch<FORCE, T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_batch<FORCE, T>), dim3(g.nbatch), dim3(256), lds, s, g, bn, b, static_cast<const T *>(pk),
                       W, wscale, out);
    return hipGetLastError();
}

hipError_t launch_rho_batch(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                            const void *pk, double *rho)
{
    return f32 ? launch_batch_t<false, float>(s, g, bn, b, nbmax, pk, nullptr, 0.0, rho)
               : launch_batch_t<false, double>(s, g, bn, b, nbmax, pk, nullptr, 0.0, rho);
}

hipError_t launch_force_batch(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                              const void *pk, const double *W, double wscale, double *Fent)
{
    return f32 ? launch_batch_t<true, float>(s, g, bn, b, nbmax, pk, W, wscale, Fent)
               : launch_batch_t<true, double>(s, g, bn, b, nbmax, pk, W, wscale, Fent);
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
