// gint_hr.hip -- lattice-vector blocks of the local Hamiltonian,
//     H_mu,nu(R) = dV sum_g phi_mu(r_g - tau_I) V(r_g) phi_nu(r_g - tau_J - R)
// (Sec. 3.3.1, H^loc(R) equation; the sum runs over the mesh points of the
// whole crystal), the per-R storage from which H(k) = sum_R e^{ik.R} H(R)
// of Sec. 2.1 is assembled.  tau are the positions as the caller gave them.
//
// Point-stationary like the Gamma-point H kernels, with the images of each
// atom kept apart instead of folded: a workgroup owns a mesh batch,
// evaluates every (atom, image) that reaches it into LDS once, and forms
// every block of two of them (ia <= ja) on the matrix cores.  With image T_a
// of atom I and T_b of atom J, a block is the contribution of the crystal
// points r_g - T_a to H_IJ(T_b - T_a); its transpose goes to
// H_JI(T_a - T_b).
//
// Default (fixed order): the per-batch kernels of the Gamma-point H write
// the blocks of the unfolded images as partials; every block gets the key
// of its canonical triple (I, J, R) (I < J, or I = J and R >= 0 in
// lexicographic order; the block or its transpose), the keys are sorted
// once per geometry (stable: batch order inside a triple), and one wave per
// triple sums its blocks in that order and writes H_IJ(R) and H_JI(-R)
// (k_HR_reduce).  When the partials exceed the partial-buffer budget, the
// blocks are added into the output with FP64 atomics instead (k_HR_batch;
// the order of the additions is then not fixed).
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>
#include <mutex>

#include "gint_device.h"

namespace gint {

// internal atom of every image (image i belongs to the entry e with
// ent_img[e] <= i < ent_img[e + 1])
__global__ void k_image_atoms(long long nent, const int *__restrict__ ent_atom, const int *__restrict__ ent_img,
                              int *__restrict__ img_atom)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nent)
        return;
    const int a = ent_atom[e];
    for (int i = ent_img[e]; i < ent_img[e + 1]; ++i)
        img_atom[i] = a;
}

// lattice multiples W of each internal atom: the position as given is the
// wrapped one plus W . (a1, a2, a3)
__global__ void k_wrap_shift(Geo g, const int *__restrict__ perm, const double *__restrict__ pos_in,
                             const double *__restrict__ xw, int *__restrict__ wsh)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= g.natom)
        return;
    const int q = perm[a];
    const double x[3] = {pos_in[3 * q], pos_in[3 * q + 1], pos_in[3 * q + 2]};
    const double y[3] = {xw[3 * a], xw[3 * a + 1], xw[3 * a + 2]};
    double s[3], t[3];
    frac_of(g, x, s);
    frac_of(g, y, t);
    for (int k = 0; k < 3; ++k)
        wsh[3 * a + k] = (int)rint(s[k] - t[k]);
}

hipError_t launch_HR_prep(hipStream_t s, const Geo &g, long long nent, const int *ent_atom, const int *ent_img,
                          int *img_atom, const int *perm, const double *pos_in, const double *xw, int *wsh)
{
    if (nent > 0)
        hipLaunchKernelGGL(k_image_atoms, dim3((unsigned)((nent + 255) / 256)), dim3(256), 0, s, nent, ent_atom,
                           ent_img, img_atom);
    hipLaunchKernelGGL(k_wrap_shift, dim3((g.natom + 255) / 256), dim3(256), 0, s, g, perm, pos_in, xw, wsh);
    return hipGetLastError();
}

// Lattice vectors R = T_c - T_a over every ordered pair of atom images (a, c)
// reaching one batch: a superset of the R with a non-zero block.  mark is
// the box |n_k| <= M (row-major, n3 fastest); entries are set to 1.
__global__ __launch_bounds__(256) void k_HR_mark(Geo g, const int *__restrict__ iptr, const int *__restrict__ img_atom,
                                                 const int *__restrict__ img, const int *__restrict__ wsh, int M,
                                                 int *__restrict__ mark)
{
    const int b = blockIdx.x;
    const int i0 = iptr[b], nb = iptr[b + 1] - i0;
    const int w = 2 * M + 1;
    for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) {
        const int a = q / nb, c = q - a * nb;
        int na[3], nc[3];
        unpack_image(img[i0 + a], na);
        unpack_image(img[i0 + c], nc);
        const int A = img_atom[i0 + a], C = img_atom[i0 + c];
        int R[3];
        bool in = true;
        for (int k = 0; k < 3; ++k) {
            R[k] = (nc[k] - wsh[3 * C + k]) - (na[k] - wsh[3 * A + k]);
            in = in && R[k] >= -M && R[k] <= M;
        }
        if (in)
            mark[((R[0] + M) * w + R[1] + M) * w + R[2] + M] = 1;
    }
}

hipError_t launch_HR_mark(hipStream_t s, const Geo &g, const int *iptr, const int *img_atom, const int *img,
                          const int *wsh, int M, int *mark)
{
    hipLaunchKernelGGL(k_HR_mark, dim3((unsigned)g.nbatch), dim3(256), 0, s, g, iptr, img_atom, img, wsh, M, mark);
    return hipGetLastError();
}

// 0, 1, ..., n - 1
__global__ void k_iota(long long n, int *__restrict__ a)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        a[i] = (int)i;
}

// Canonical triple of every unfolded block: key = (I n_atom + J) 2^18 +
// index of R in the box |n_k| <= kHRBox, I, J input atom ids; code = the
// block's partial index q (stored as H_IJ) or -q - 1 (stored as H_JI).
// *bad is set when some R falls outside the box (the key then sorts last).
__global__ __launch_bounds__(256) void k_HR_keys(const int *__restrict__ iptr, const int *__restrict__ boff,
                                                 const int *__restrict__ img_atom, const int *__restrict__ img,
                                                 const int *__restrict__ perm, const int *__restrict__ wsh, int natom,
                                                 unsigned long long *__restrict__ key, int *__restrict__ code,
                                                 int *__restrict__ bad)
{
    const int b = blockIdx.x;
    const int i0 = iptr[b], nb = iptr[b + 1] - i0, q0 = boff[b];
    const int nblk = nb * (nb + 1) / 2;
    constexpr int M = kHRBox, w = 2 * kHRBox + 1;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
        int ia = 0, r = k;
        while (r >= nb - ia) {
            r -= nb - ia;
            ++ia;
        }
        const int ja = ia + r;
        const int A = img_atom[i0 + ia], C = img_atom[i0 + ja];
        int na[3], nc[3], R[3];
        unpack_image(img[i0 + ia], na);
        unpack_image(img[i0 + ja], nc);
        for (int d = 0; d < 3; ++d)
            R[d] = (nc[d] - wsh[3 * C + d]) - (na[d] - wsh[3 * A + d]);
        const int Ii = perm[A], Ji = perm[C];
        const bool Rnonneg = R[0] > 0 || (R[0] == 0 && (R[1] > 0 || (R[1] == 0 && R[2] >= 0)));
        const bool up = Ii < Ji || (Ii == Ji && Rnonneg);
        const int I = up ? Ii : Ji, J = up ? Ji : Ii, s = up ? 1 : -1;
        bool in = true;
        for (int d = 0; d < 3; ++d)
            in = in && s * R[d] >= -M && s * R[d] <= M;
        const int q = q0 + k;
        if (in) {
            const int ridx = ((s * R[0] + M) * w + s * R[1] + M) * w + s * R[2] + M;
            key[q] = (((unsigned long long)I * natom + J) << 18) | (unsigned long long)ridx;
        } else {
            key[q] = ~0ULL;
            *bad = 1;
        }
        code[q] = up ? q : -q - 1;
    }
}

// first position of every run of equal sorted keys: flag, then (after an
// exclusive scan of the flags) start and key of each run
__global__ void k_seg_flag(long long n, const unsigned long long *__restrict__ key, int *__restrict__ flag)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        flag[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_seg_fill(long long n, const unsigned long long *__restrict__ key, const int *__restrict__ fscan,
                           int *__restrict__ tstart, unsigned long long *__restrict__ tkey)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    if (i == 0 || key[i] != key[i - 1]) {
        tstart[fscan[i]] = (int)i;
        tkey[fscan[i]] = key[i];
    }
    if (i == n - 1)
        tstart[fscan[n]] = (int)n;
}

hipError_t launch_iota(hipStream_t s, long long n, int *a)
{
    if (n > 0)
        hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a);
    return hipGetLastError();
}

hipError_t launch_HR_keys(hipStream_t s, int nbatch, const int *iptr, const int *boff, const int *img_atom,
                          const int *img, const int *perm, const int *wsh, int natom, unsigned long long *key,
                          int *code, int *bad)
{
    hipLaunchKernelGGL(k_HR_keys, dim3((unsigned)nbatch), dim3(256), 0, s, iptr, boff, img_atom, img, perm, wsh, natom,
                       key, code, bad);
    return hipGetLastError();
}

hipError_t launch_seg(hipStream_t s, long long n, const unsigned long long *key, int *flag, int *fscan, int *tstart,
                      unsigned long long *tkey, bool fill)
{
    if (n <= 0)
        return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (fill)
        hipLaunchKernelGGL(k_seg_fill, dim3(nb), dim3(256), 0, s, n, key, fscan, tstart, tkey);
    else
        hipLaunchKernelGGL(k_seg_flag, dim3(nb), dim3(256), 0, s, n, key, flag);
    return hipGetLastError();
}

hipError_t sort_HR_keys(hipStream_t s, void *tmp, size_t &tmp_bytes, const unsigned long long *key_in,
                        unsigned long long *key_out, const int *code_in, int *code_out, int n, int end_bit)
{
    return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key_in, key_out, code_in, code_out, n, 0, end_bit, s);
}

// Per unfolded block entry (batch block of image pair a <= c, in the order
// of k_HR_keys): 2 t + o, t = its canonical (I, J, R) triple (the run of equal
// sorted keys it falls in), o = 1 where the canonical orientation swaps the
// pair, so that the entry's block is the transpose of the triple's.
__global__ void k_entry_tri(long long n, const int *__restrict__ code, const int *__restrict__ fscan,
                            int *__restrict__ etri)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int c = code[s];
    const int e = c >= 0 ? c : -c - 1;
    etri[e] = 2 * (fscan[s + 1] - 1) + (c < 0 ? 1 : 0);
}

hipError_t launch_entry_tri(hipStream_t s, long long n, const int *code, const int *fscan, int *etri)
{
    if (n > 0)
        hipLaunchKernelGGL(k_entry_tri, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, code, fscan, etri);
    return hipGetLastError();
}

// The density-matrix block of a canonical triple (I, J, R) as the rho and
// force contractions use it (Sec. 3.3.1, rho(r_g) equation with its sums
// over R and R'):
//     S_IJ(R) = D_IJ(R) + D_JI(-R)^T,
// each term zero where its lattice vector is not in the caller's list,
// zero-padded to 16 x 16, in both orientations (o = 0: S, o = 1: S^T), laid
// out in the lane order of the FP64 MFMA A operand: lane (i, k0) of 64
// holds elements (i, k0 + 4 s), s = 0..3, as 4 consecutive doubles, so that
// a wave reads one block with two 16-byte loads per lane.  One wave per
// triple; nz[t] = 0 when neither R nor -R is listed.
constexpr int kPackWaves = 4;
__global__ __launch_bounds__(64 * kPackWaves) void k_S_pack(int ntri, const unsigned long long *__restrict__ tkey,
                                                            int natom, const int *__restrict__ orb0, HRMap m,
                                                            int norb, const double *__restrict__ DR,
                                                            double *__restrict__ spk, int *__restrict__ nz)
{
    const int t = blockIdx.x * kPackWaves + (threadIdx.x >> 6);
    if (t >= ntri)
        return;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const unsigned long long key = tkey[t];
    const unsigned long long ij = key >> 18;
    const int ridx = (int)(key & ((1ULL << 18) - 1));
    const int I = (int)(ij / (unsigned long long)natom), J = (int)(ij % (unsigned long long)natom);
    constexpr int M = kHRBox, w = 2 * kHRBox + 1;
    const int R0 = ridx / (w * w) - M, R1 = (ridx / w) % w - M, R2 = ridx % w - M;
    const int qR = hr_lookup(m, R0, R1, R2), qN = hr_lookup(m, -R0, -R1, -R2);
    if (lane == 0)
        nz[t] = (qR >= 0 || qN >= 0) ? 1 : 0;
    const int mI = orb0[I], nI = orb0[I + 1] - mI, mJ = orb0[J], nJ = orb0[J + 1] - mJ;
    const size_t nn = (size_t)norb * norb;
    double v0[4], v1[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int kc = lk + 4 * st;
        // o = 0: S[li][kc]; o = 1: S^T[li][kc] = S[kc][li]
        const bool in0 = li < nI && kc < nJ, in1 = kc < nI && li < nJ;
        const double a0 = (in0 && qR >= 0) ? DR[qR * nn + (size_t)(mI + li) * norb + mJ + kc] : 0.0;
        const double b0 = (in0 && qN >= 0) ? DR[qN * nn + (size_t)(mJ + kc) * norb + mI + li] : 0.0;
        const double a1 = (in1 && qR >= 0) ? DR[qR * nn + (size_t)(mI + kc) * norb + mJ + li] : 0.0;
        const double b1 = (in1 && qN >= 0) ? DR[qN * nn + (size_t)(mJ + li) * norb + mI + kc] : 0.0;
        v0[st] = a0 + b0;
        v1[st] = a1 + b1;
    }
    double4 *o = reinterpret_cast<double4 *>(spk) + (size_t)2 * t * 64;
    o[lane] = double4{v0[0], v0[1], v0[2], v0[3]};
    o[64 + lane] = double4{v1[0], v1[1], v1[2], v1[3]};
}

hipError_t launch_S_pack(hipStream_t s, int ntri, const unsigned long long *tkey, int natom, const int *orb0,
                         const HRMap &m, int norb, const double *DR, double *spk, int *nz)
{
    if (ntri > 0)
        hipLaunchKernelGGL(k_S_pack, dim3((unsigned)((ntri + kPackWaves - 1) / kPackWaves)), dim3(64 * kPackWaves),
                           0, s, ntri, tkey, natom, orb0, m, norb, DR, spk, nz);
    return hipGetLastError();
}

// Packed index (2 t + o) of image pair (a, c) of batch b, or -1 when its
// triple has no listed lattice vector; c < a takes the transpose of (c, a).
__device__ __forceinline__ int packed_block(const PackedS &ps, int b, int nb, int a, int c)
{
    const int lo = a < c ? a : c, hi = a < c ? c : a;
    const int v = ps.etri[ps.boff[b] + lo * nb - lo * (lo - 1) / 2 + (hi - lo)];
    if (!ps.nz[v >> 1])
        return -1;
    return a <= c ? v : v ^ 1;
}

// this lane's four elements of a packed block (zeros for v < 0), times f
__device__ __forceinline__ void load_packed(const PackedS &ps, int v, int lane, double f, double (&x)[4])
{
    if (v < 0) {
        x[0] = x[1] = x[2] = x[3] = 0.0;
        return;
    }
    const double4 d = reinterpret_cast<const double4 *>(ps.spk)[(size_t)v * 64 + lane];
    x[0] = f * d.x;
    x[1] = f * d.y;
    x[2] = f * d.z;
    x[3] = f * d.w;
}

constexpr int kHRWaves = 16;

template <typename T, int P>
__global__ __launch_bounds__(64 * kHRWaves) void k_HR_batch(Geo g, const int *__restrict__ iptr,
                                                   const int *__restrict__ img_atom, const int *__restrict__ img,
                                                   Basis bs, const int *__restrict__ wsh,
                                                   const double *__restrict__ W, double wscale, HRMap m, int norb,
                                                   double *__restrict__ HR)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    T *s_phi = reinterpret_cast<T *>(s_dyn);  // [nbmax][P][kRow]
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_nor[kMaxBatchAtoms], s_mu0[kMaxBatchAtoms];
    __shared__ int s_T[kMaxBatchAtoms][3];
    __shared__ double s_w[kMaxP];

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6),
              nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int b = xcd_batch(blockIdx.x, 0, g.nbatch);
    if (b < 0)
        return;
    const int i0 = iptr[b], nb = iptr[b + 1] - i0;
    int ib[3];
    batch_coords(g, b, ib);

    for (int k = tid; k < g.nrad; k += blockDim.x)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += blockDim.x)
        s_sp[k] = bs.sp[k];
    for (int a = tid; a < nb; a += blockDim.x) {
        const int atom = img_atom[i0 + a];
        s_atom[a] = atom;
        s_nor[a] = bs.sp[bs.spc[atom]].norb;
        s_mu0[a] = bs.orb0[bs.perm[atom]];
        // image of the wrapped atom, as a lattice vector from the position
        // the caller gave
        int n[3];
        unpack_image(img[i0 + a], n);
        for (int k = 0; k < 3; ++k)
            s_T[a][k] = n[k] - wsh[3 * atom + k];
    }
    for (int p = tid; p < P; p += blockDim.x) {
        int n[3];
        s_w[p] = batch_point(g, ib, p, n) ? wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 0.0;
    }
    __syncthreads();

    // ---- one image of one atom per LDS slot, every batch point ----
    for (int idx = tid; idx < nb * P; idx += blockDim.x) {
        const int a = idx / P, p = idx % P;
        const int atom = s_atom[a];
        T *row = s_phi + (size_t)(a * P + p) * kRow;
        const int swz = p & 15;
        int n[3];
        const bool valid = batch_point(g, ib, p, n);
        const DevSpecies &S = s_sp[bs.spc[atom]];
        const int zlo = valid ? S.norb : 0;
        for (int o = zlo; o < kMaxOrb; ++o)
            row[o ^ swz] = (T)0;
        if (valid) {
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            double r[3];
            mesh_cart(g, n, r);
            eval_orbitals<T>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, 1, img[i0 + a], i0 + a, img, r,
                             row, swz);
        }
    }
    __syncthreads();

    const int nblk = nb * (nb + 1) / 2;
    const int k0 = wave * nblk / nw, k1 = (wave + 1) * nblk / nw;
    int ia = 0, ja = 0;
    {
        // (ia, ja) of block k0 in the row-major order of ia <= ja < nb
        int k = k0;
        while (ia < nb && k >= nb - ia) {
            k -= nb - ia;
            ++ia;
        }
        ja = ia + k;
    }
    T wl[P / 4];
    int off[P / 4];
#pragma unroll
    for (int kk = 0; kk < P / 4; ++kk) {
        const int p = 4 * kk + lk;
        wl[kk] = (T)s_w[p];
        off[kk] = p * kRow + (li ^ (p & 15));
    }
    const size_t nn = (size_t)norb * norb;
    for (int k = k0; k < k1; ++k) {
        const int Rx = s_T[ja][0] - s_T[ia][0], Ry = s_T[ja][1] - s_T[ia][1], Rz = s_T[ja][2] - s_T[ia][2];
        const int rp = hr_lookup(m, Rx, Ry, Rz);
        const int rn = ia != ja ? hr_lookup(m, -Rx, -Ry, -Rz) : -1;
        if (rp >= 0 || rn >= 0) {
            const T *pI = s_phi + (size_t)(ia * P) * kRow;
            const T *pJ = s_phi + (size_t)(ja * P) * kRow;
            typename MM<T>::acc acc = MM<T>::zero();
#pragma unroll
            for (int kk = 0; kk < P / 4; ++kk)
                acc = MM<T>::mma(wl[kk] * pI[off[kk]], pJ[off[kk]], acc);
            const int nI = s_nor[ia], nJ = s_nor[ja], mI = s_mu0[ia], mJ = s_mu0[ja];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = MM<T>::row(lk, v);
                if (row < nI && li < nJ) {
                    const double x = (double)acc[v];
                    if (rp >= 0)
                        unsafeAtomicAdd(HR + rp * nn + (size_t)(mI + row) * norb + mJ + li, x);
                    if (rn >= 0)
                        unsafeAtomicAdd(HR + rn * nn + (size_t)(mJ + li) * norb + mI + row, x);
                }
            }
        }
        if (++ja == nb) {
            ++ia;
            ja = ia;
        }
    }
}

// rho from lattice-vector density-matrix blocks (Sec. 3.3.1, rho(r_g)
// equation with its sums over R and R'): with the images of the batch
// unfolded as above,
//     rho_p = sum_{a <= c} phi_a(p)^T S_ac phi_c(p),
//     S_ac = D_{I_a I_c}(T_c - T_a) + D_{I_c I_a}(T_a - T_c)^T  (a < c),
//     S_aa = D_{I_a I_a}(0),
// D blocks of unlisted R being zero.  Per block, S_ac phi_c on the matrix
// cores (16 points per product) is added to T_a in the result registers,
// which is dotted with phi_a once per row of blocks; lanes and waves are
// summed in a fixed order.  Each point is written once.  The list indices
// of both lattice vectors of every image pair are looked up once per batch
// into LDS, and each lane's D(R) elements are loaded two blocks ahead.
template <typename T, int P, bool PK>
__global__ __launch_bounds__(64 * kHRWaves) void k_rhoR_batch(Geo g, const int *__restrict__ iptr,
                                                     const int *__restrict__ img_atom, const int *__restrict__ img,
                                                     Basis bs, const int *__restrict__ wsh, HRMap m, int norb,
                                                     const double *__restrict__ DR, PackedS ps, int nbmax,
                                                     double *__restrict__ rho)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    T *s_phi = reinterpret_cast<T *>(s_dyn);  // [nbmax][P][kRow]
    // then per image pair (a, c), a * nb + c: list indices of R = T_c - T_a and of -R
    int2 *s_q = reinterpret_cast<int2 *>(s_dyn + sizeof(T) * (size_t)nbmax * P * kRow);
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_nor[kMaxBatchAtoms], s_mu0[kMaxBatchAtoms];
    __shared__ int s_T[kMaxBatchAtoms][3];
    __shared__ double s_part[kHRWaves][kMaxP];

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6),
              nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int b = xcd_batch(blockIdx.x, 0, g.nbatch);
    if (b < 0)
        return;
    const int i0 = iptr[b], nb = iptr[b + 1] - i0;
    int ib[3];
    batch_coords(g, b, ib);

    for (int k = tid; k < g.nrad; k += blockDim.x)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += blockDim.x)
        s_sp[k] = bs.sp[k];
    for (int a = tid; a < nb; a += blockDim.x) {
        const int atom = img_atom[i0 + a];
        s_atom[a] = atom;
        s_nor[a] = bs.sp[bs.spc[atom]].norb;
        s_mu0[a] = bs.orb0[bs.perm[atom]];
        int n[3];
        unpack_image(img[i0 + a], n);
        for (int k = 0; k < 3; ++k)
            s_T[a][k] = n[k] - wsh[3 * atom + k];
    }
    __syncthreads();

    for (int idx = tid; idx < nb * P; idx += blockDim.x) {
        const int a = idx / P, p = idx % P;
        const int atom = s_atom[a];
        T *row = s_phi + (size_t)(a * P + p) * kRow;
        const int swz = p & 15;
        int n[3];
        const bool valid = batch_point(g, ib, p, n);
        const DevSpecies &S = s_sp[bs.spc[atom]];
        const int zlo = valid ? S.norb : 0;
        for (int o = zlo; o < kMaxOrb; ++o)
            row[o ^ swz] = (T)0;
        if (valid) {
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            double r[3];
            mesh_cart(g, n, r);
            eval_orbitals<T>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, 1, img[i0 + a], i0 + a, img, r,
                             row, swz);
        }
    }
    for (int k = tid; k < nb * nb; k += blockDim.x) {
        const int a = k / nb, c = k - a * nb;
        if (PK) {
            if (a <= c)
                s_q[k] = int2{packed_block(ps, b, nb, a, c), -1};
        } else {
            const int Rx = s_T[c][0] - s_T[a][0], Ry = s_T[c][1] - s_T[a][1], Rz = s_T[c][2] - s_T[a][2];
            s_q[k] = int2{hr_lookup(m, Rx, Ry, Rz), a != c ? hr_lookup(m, -Rx, -Ry, -Rz) : -1};
        }
    }
    __syncthreads();

    constexpr int NT = P / 16;  // 16-point tiles
    double racc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        racc[t] = 0.0;
    const int nblk = nb * (nb + 1) / 2;
    const int k0 = wave * nblk / nw, k1 = (wave + 1) * nblk / nw;
    int ia = 0, ja = 0;
    {
        int k = k0;
        while (ia < nb && k >= nb - ia) {
            k -= nb - ia;
            ++ia;
        }
        ja = ia + k;
    }
    const size_t nn = (size_t)norb * norb;
    // a wave's blocks are consecutive in row-major order: T_a = sum_c S_ac
    // phi_c accumulates in the result registers over the blocks of one row
    // a, and is dotted with phi_a once per row (at a row change and at the
    // end)
    typename MM<T>::acc acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        acc[t] = MM<T>::zero();
    int cur = ia;
    auto flush = [&](int a) {
        const T *pA = s_phi + (size_t)(a * P) * kRow;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int p = 16 * t + li;
            double d = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = MM<T>::row(lk, v);
                d += (double)pA[p * kRow + (i ^ (p & 15))] * (double)acc[t][v];
            }
            racc[t] += d;
            acc[t] = MM<T>::zero();
        }
    };
    // this lane's D(R) elements of image pair (a, c): both terms loaded
    // (zero outside the blocks, for unlisted R or past the wave's range),
    // summed at use
    auto load = [&](double (&xp)[4], double (&xn)[4], int a, int c, bool ok) {
        const int2 q = ok ? s_q[a * nb + c] : int2{-1, -1};
        if (PK) {
            // the packed S_ac (S_aa = D_II(0) + D_II(0)^T: half of it on the diagonal)
            load_packed(ps, q.x, lane, a == c ? 0.5 : 1.0, xp);
            return;
        }
        const int nI = ok ? s_nor[a] : 0, nJ = ok ? s_nor[c] : 0;
        const int mI = ok ? s_mu0[a] : 0, mJ = ok ? s_mu0[c] : 0;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int kc = lk + 4 * st;
            const bool in = li < nI && kc < nJ;
            xp[st] = (in && q.x >= 0) ? DR[q.x * nn + (size_t)(mI + li) * norb + mJ + kc] : 0.0;
            xn[st] = (in && q.y >= 0) ? DR[q.y * nn + (size_t)(mJ + kc) * norb + mI + li] : 0.0;
        }
    };
    auto block = [&](const double (&xp)[4], const double (&xn)[4], int a, int c) {
        if (a != cur) {
            flush(cur);
            cur = a;
        }
        const int2 q = s_q[a * nb + c];
        if (q.x < 0 && q.y < 0)
            return;
        const T *pC = s_phi + (size_t)(c * P) * kRow;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int p = 16 * t + li;  // this lane's point (B and result column)
#pragma unroll
            for (int st = 0; st < 4; ++st)
                acc[t] = MM<T>::mma((T)(PK ? xp[st] : xp[st] + xn[st]), pC[p * kRow + ((lk + 4 * st) ^ (p & 15))],
                                    acc[t]);
        }
    };
    auto next = [&](int &x, int &y) {
        if (++y == nb) {
            ++x;
            y = x;
        }
    };
    // blocks k, k + 1 and k + 2 of the wave's range in three register sets:
    // the D(R) elements of block k + 2 are in flight while block k runs
    double p0[4], n0[4], p1[4], n1[4], p2[4], n2[4];
    int a0 = ia, c0 = ja, a1 = ia, c1 = ja, a2, c2;
    next(a1, c1);
    load(p0, n0, a0, c0, k0 < k1);
    load(p1, n1, a1, c1, k0 + 1 < k1);
    int k = k0;
    for (; k + 2 < k1; k += 3) {
        a2 = a1;
        c2 = c1;
        next(a2, c2);
        load(p2, n2, a2, c2, true);
        block(p0, n0, a0, c0);
        a0 = a2;
        c0 = c2;
        next(a0, c0);
        load(p0, n0, a0, c0, k + 3 < k1);
        block(p1, n1, a1, c1);
        a1 = a0;
        c1 = c0;
        next(a1, c1);
        load(p1, n1, a1, c1, k + 4 < k1);
        block(p2, n2, a2, c2);
    }
    if (k < k1)
        block(p0, n0, a0, c0);
    if (k + 1 < k1)
        block(p1, n1, a1, c1);
    if (k0 < k1)
        flush(cur);
    // lanes li, li + 16, li + 32, li + 48 hold the same point
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        double x = racc[t];
        x += __shfl_xor(x, 16);
        x += __shfl_xor(x, 32);
        if (lk == 0)
            s_part[wave][16 * t + li] = x;
    }
    __syncthreads();
    for (int p = tid; p < P; p += blockDim.x) {
        int n[3];
        if (!batch_point(g, ib, p, n))
            continue;
        double x = 0.0;
        for (int w = 0; w < nw; ++w)
            x += s_part[w][p];
        rho[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] = x;
    }
}

// dE/dR for E = dV sum_g V_g rho_g with rho from D(R) (Sec. 3.3.1,
// F^{loc,Pulay} equation with its sum over R): per unfolded image a of the
// batch, T_a = sum_c S'_ac phi_c on the matrix cores with
// S'_ac = D_{I_a I_c}(T_c - T_a) + D_{I_c I_a}(T_a - T_c)^T over every image
// c (c = a included), held in the MFMA result registers; then each lane
// dots the gradients of its four orbitals at its point with w T_a
// (grad4_dot) and the wave sums the lanes.  One partial per (batch, image),
// summed per atom in batch order by k_forceR_reduce.  The list indices of
// both lattice vectors of every image pair (a, c) are looked up once per
// batch into LDS, and each lane's D(R) elements of image c + 2 are loaded
// while the products of image c run (three register sets in rotation).
constexpr int kFRWaves = 12;  // three waves per SIMD (147 VGPRs in FP64)

template <typename T, int P, bool PK>
__global__ __launch_bounds__(64 * kFRWaves) void k_forceR_batch(Geo g, const int *__restrict__ iptr,
                                                       const int *__restrict__ img_atom,
                                                       const int *__restrict__ img, Basis bs,
                                                       const int *__restrict__ wsh, HRMap m, int norb,
                                                       const double *__restrict__ DR, const double *__restrict__ W,
                                                       double wscale, PackedS ps, int nbmax,
                                                       double *__restrict__ Fimg)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    T *s_phi = reinterpret_cast<T *>(s_dyn);  // [nbmax][P][kRow]
    // then per image pair (a, c), a * nb + c: list indices of R = T_c - T_a and of -R
    int2 *s_q = reinterpret_cast<int2 *>(s_dyn + sizeof(T) * (size_t)nbmax * P * kRow);
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_nor[kMaxBatchAtoms], s_mu0[kMaxBatchAtoms];
    __shared__ int s_T[kMaxBatchAtoms][3];
    __shared__ double s_w[kMaxP];

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6),
              nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int b = xcd_batch(blockIdx.x, 0, g.nbatch);
    if (b < 0)
        return;
    const int i0 = iptr[b], nb = iptr[b + 1] - i0;
    int ib[3];
    batch_coords(g, b, ib);

    for (int k = tid; k < g.nrad; k += blockDim.x)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += blockDim.x)
        s_sp[k] = bs.sp[k];
    for (int a = tid; a < nb; a += blockDim.x) {
        const int atom = img_atom[i0 + a];
        s_atom[a] = atom;
        s_nor[a] = bs.sp[bs.spc[atom]].norb;
        s_mu0[a] = bs.orb0[bs.perm[atom]];
        int n[3];
        unpack_image(img[i0 + a], n);
        for (int k = 0; k < 3; ++k)
            s_T[a][k] = n[k] - wsh[3 * atom + k];
    }
    for (int p = tid; p < P; p += blockDim.x) {
        int n[3];
        s_w[p] = batch_point(g, ib, p, n) ? wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 0.0;
    }
    __syncthreads();

    for (int idx = tid; idx < nb * P; idx += blockDim.x) {
        const int a = idx / P, p = idx % P;
        const int atom = s_atom[a];
        T *row = s_phi + (size_t)(a * P + p) * kRow;
        const int swz = p & 15;
        int n[3];
        const bool valid = batch_point(g, ib, p, n);
        const DevSpecies &S = s_sp[bs.spc[atom]];
        const int zlo = valid ? S.norb : 0;
        for (int o = zlo; o < kMaxOrb; ++o)
            row[o ^ swz] = (T)0;
        if (valid) {
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            double r[3];
            mesh_cart(g, n, r);
            eval_orbitals<T>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, 1, img[i0 + a], i0 + a, img, r,
                             row, swz);
        }
    }
    for (int k = tid; k < nb * nb; k += blockDim.x) {
        const int a = k / nb, c = k - a * nb;
        if (PK) {
            s_q[k] = int2{packed_block(ps, b, nb, a, c), -1};
        } else {
            const int Rx = s_T[c][0] - s_T[a][0], Ry = s_T[c][1] - s_T[a][1], Rz = s_T[c][2] - s_T[a][2];
            s_q[k] = int2{hr_lookup(m, Rx, Ry, Rz), hr_lookup(m, -Rx, -Ry, -Rz)};
        }
    }
    __syncthreads();

    constexpr int NT = P / 16;
    const size_t nn = (size_t)norb * norb;
    for (int a = wave; a < nb; a += nw) {
        const int nI = s_nor[a], mI = s_mu0[a];
        typename MM<T>::acc acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
            acc[t] = MM<T>::zero();
        // this lane's D(R) elements of image pair (a, c): both terms loaded
        // (zero outside the blocks or for unlisted R), summed at use
        auto load = [&](double (&xp)[4], double (&xn)[4], int c) {
            const int2 q = s_q[a * nb + c];
            if (PK) {
                load_packed(ps, q.x, lane, 1.0, xp);
                return;
            }
            const int nJ = s_nor[c], mJ = s_mu0[c];
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int kc = lk + 4 * st;
                const bool in = li < nI && kc < nJ;
                xp[st] = (in && q.x >= 0) ? DR[q.x * nn + (size_t)(mI + li) * norb + mJ + kc] : 0.0;
                xn[st] = (in && q.y >= 0) ? DR[q.y * nn + (size_t)(mJ + kc) * norb + mI + li] : 0.0;
            }
        };
        auto block = [&](const double (&xp)[4], const double (&xn)[4], int c) {
            const int2 q = s_q[a * nb + c];
            if (q.x < 0 && q.y < 0)
                return;
            const T *pC = s_phi + (size_t)(c * P) * kRow;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int p = 16 * t + li;
#pragma unroll
                for (int st = 0; st < 4; ++st)
                    acc[t] = MM<T>::mma((T)(PK ? xp[st] : xp[st] + xn[st]),
                                        pC[p * kRow + ((lk + 4 * st) ^ (p & 15))], acc[t]);
            }
        };
        auto cl = [&](int c) { return c < nb ? c : nb - 1; };
        double p0[4], n0[4], p1[4], n1[4], p2[4], n2[4];
        load(p0, n0, 0);
        load(p1, n1, cl(1));
        int c = 0;
        for (; c + 2 < nb; c += 3) {
            load(p2, n2, c + 2);
            block(p0, n0, c);
            load(p0, n0, cl(c + 3));
            block(p1, n1, c + 1);
            load(p1, n1, cl(c + 4));
            block(p2, n2, c + 2);
        }
        if (c < nb)
            block(p0, n0, c);
        if (c + 1 < nb)
            block(p1, n1, c + 1);
        // gradients of this lane's four orbitals of image a at its point
        const int atom = s_atom[a];
        const DevSpecies &S = s_sp[bs.spc[atom]];
        const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
        double fx[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int p = 16 * t + li;
            int n[3];
            const bool valid = batch_point(g, ib, p, n);
            double r[3];
            mesh_cart(g, n, r);
            const double wp = s_w[p];
            const double wv[4] = {wp * (double)acc[t][0], wp * (double)acc[t][1], wp * (double)acc[t][2],
                                  wp * (double)acc[t][3]};
            grad4_dot(g, s_rad, S.orb_rad, S.orb_m, S.norb, S.rc, bs.coef, X, valid ? 1 : 0, img[i0 + a], i0 + a,
                      img, r, MM<T>::row(lk, 0), MM<T>::row(lk, 1) - MM<T>::row(lk, 0), wv, fx);
        }
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            double v = fx[x];
            for (int o = 32; o > 0; o >>= 1)
                v += __shfl_xor(v, o);
            fx[x] = v;
        }
        if (lane == 0)
            for (int x = 0; x < 3; ++x)
                Fimg[3 * (size_t)(i0 + a) + x] = -fx[x];
    }
}

// per internal atom: its image partials in batch order (entries of the atom
// in batch order, images of each entry in order), tree-summed in a fixed
// order; written at the atom's input index
__global__ __launch_bounds__(256) void k_forceR_reduce(const int *__restrict__ aptr, const int *__restrict__ aent,
                                                       const int *__restrict__ ent_img, const int *__restrict__ perm,
                                                       const double *__restrict__ Fimg, double *__restrict__ dEdR)
{
    __shared__ double red[3][256];
    const int a = blockIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = aptr[a] + threadIdx.x; k < aptr[a + 1]; k += 256) {
        const int e = aent[k];
        for (int i = ent_img[e]; i < ent_img[e + 1]; ++i)
            for (int x = 0; x < 3; ++x)
                v[x] += Fimg[3 * (size_t)i + x];
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
        dEdR[3 * perm[a] + threadIdx.x] = red[threadIdx.x][0];
}

template <typename T, int P, bool PK>
static hipError_t launch_forceR_p(hipStream_t s, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                                  const int *img, const Basis &b, const int *wsh, const HRMap &m, int norb,
                                  const double *DR, const PackedS &ps, const double *W, double wscale, double *Fimg)
{
    const size_t lds = sizeof(T) * (size_t)nbmax * P * kRow + sizeof(int2) * (size_t)nbmax * nbmax;
    hipError_t e = hipFuncSetAttribute((const void *)k_forceR_batch<T, P, PK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_forceR_batch<T, P, PK>), dim3((unsigned)(kXcd * ((g.nbatch + kXcd - 1) / kXcd))),
                       dim3(64 * kFRWaves), lds, s, g, iptr, img_atom, img, b, wsh, m, norb, DR, W, wscale, ps, nbmax,
                       Fimg);
    return hipGetLastError();
}

template <typename T, int P>
static hipError_t launch_forceR_pk(hipStream_t s, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                                   const int *img, const Basis &b, const int *wsh, const HRMap &m, int norb,
                                   const double *DR, const PackedS *ps, const double *W, double wscale, double *Fimg)
{
    if (ps)
        return launch_forceR_p<T, P, true>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, *ps, W, wscale,
                                           Fimg);
    return launch_forceR_p<T, P, false>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, PackedS{}, W, wscale,
                                        Fimg);
}

hipError_t launch_forceR_batch(hipStream_t s, bool f32, const Geo &g, int nbmax, const int *iptr,
                               const int *img_atom, const int *img, const Basis &b, const int *wsh, const HRMap &m,
                               int norb, const double *DR, const PackedS *ps, const double *W, double wscale,
                               double *Fimg)
{
    if (g.P == 32)
        return f32 ? launch_forceR_pk<float, 32>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, ps, W, wscale,
                                                 Fimg)
                   : launch_forceR_pk<double, 32>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, ps, W,
                                                  wscale, Fimg);
    if (g.P == 16)
        return f32 ? launch_forceR_pk<float, 16>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, ps, W, wscale,
                                                 Fimg)
                   : launch_forceR_pk<double, 16>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, ps, W,
                                                  wscale, Fimg);
    return hipErrorInvalidValue;
}

hipError_t launch_forceR_reduce(hipStream_t s, int natom, const int *aptr, const int *aent, const int *ent_img,
                                const int *perm, const double *Fimg, double *dEdR)
{
    hipLaunchKernelGGL(k_forceR_reduce, dim3((unsigned)natom), dim3(256), 0, s, aptr, aent, ent_img, perm, Fimg, dEdR);
    return hipGetLastError();
}

template <typename T, int P, bool PK>
static hipError_t launch_rhoR_p(hipStream_t s, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                                const int *img, const Basis &b, const int *wsh, const HRMap &m, int norb,
                                const double *DR, const PackedS &ps, double *rho)
{
    const size_t lds = sizeof(T) * (size_t)nbmax * P * kRow + sizeof(int2) * (size_t)nbmax * nbmax;
    hipError_t e = hipFuncSetAttribute((const void *)k_rhoR_batch<T, P, PK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_rhoR_batch<T, P, PK>), dim3((unsigned)(kXcd * ((g.nbatch + kXcd - 1) / kXcd))),
                       dim3(64 * kHRWaves), lds, s, g, iptr, img_atom, img, b, wsh, m, norb, DR, ps, nbmax, rho);
    return hipGetLastError();
}

template <typename T, int P>
static hipError_t launch_rhoR_pk(hipStream_t s, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                                 const int *img, const Basis &b, const int *wsh, const HRMap &m, int norb,
                                 const double *DR, const PackedS *ps, double *rho)
{
    if (ps)
        return launch_rhoR_p<T, P, true>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, *ps, rho);
    return launch_rhoR_p<T, P, false>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, PackedS{}, rho);
}

hipError_t launch_rhoR_batch(hipStream_t s, bool f32, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                             const int *img, const Basis &b, const int *wsh, const HRMap &m, int norb,
                             const double *DR, const PackedS *ps, double *rho)
{
    if (g.P == 32)
        return f32 ? launch_rhoR_pk<float, 32>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, ps, rho)
                   : launch_rhoR_pk<double, 32>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, ps, rho);
    if (g.P == 16)
        return f32 ? launch_rhoR_pk<float, 16>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, ps, rho)
                   : launch_rhoR_pk<double, 16>(s, g, nbmax, iptr, img_atom, img, b, wsh, m, norb, DR, ps, rho);
    return hipErrorInvalidValue;
}

// H(k) = sum_q e^{i 2 pi kappa . n_q} H(R_q) (Sec. 2.1, H(k) equation), with
// kappa the fractional reciprocal coordinates of k and n_q the lattice
// multiples of R_q; ph holds (cos, sin) of the phase for every (k, q).  One
// thread per matrix element reads each H(R) value once per chunk of kHkChunk
// k-points; Hk is [nk][norb*norb] of (re, im) pairs.
constexpr int kHkChunk = 8;

__global__ __launch_bounds__(256) void k_Hk(long long nel, int nR, int nk, const double *__restrict__ ph,
                                            const double *__restrict__ HR, double *__restrict__ Hk)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nel)
        return;
    for (int k0 = 0; k0 < nk; k0 += kHkChunk) {
        double re[kHkChunk], im[kHkChunk];
#pragma unroll
        for (int j = 0; j < kHkChunk; ++j)
            re[j] = im[j] = 0.0;
        for (int q = 0; q < nR; ++q) {
            const double h = HR[(size_t)q * nel + e];
#pragma unroll
            for (int j = 0; j < kHkChunk; ++j) {
                if (k0 + j < nk) {
                    const double *c = ph + 2 * ((size_t)(k0 + j) * nR + q);
                    re[j] = fma(c[0], h, re[j]);
                    im[j] = fma(c[1], h, im[j]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kHkChunk; ++j)
            if (k0 + j < nk) {
                double2 *o = reinterpret_cast<double2 *>(Hk) + (size_t)(k0 + j) * nel + e;
                *o = double2{re[j], im[j]};
            }
    }
}

hipError_t launch_Hk(hipStream_t s, long long nel, int nR, int nk, const double *ph, const double *HR, double *Hk)
{
    if (nel <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_Hk, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, s, nel, nR, nk, ph, HR, Hk);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// H(k) without device allocations (gint_HR_to_Hk_noalloc).  The phase table
// and the staged inputs (kappa, n) live in one file-scope device array, one
// copy per GPU.  Host code never uses the array's name as an address: the
// address of each device's copy comes from hipGetSymbolAddress, looked up
// once per device (with that device current) and kept in g_scratch_ptr.
// Layout: [phases: 2 kHkNaMaxPhase doubles][kappa: 3 kHkNaMaxK doubles]
//         [n: 3 kHkNaMaxR ints].  Every call overwrites what it reads, so
// nothing needs clearing; calls that overlap on one GPU race on the array.
constexpr size_t kScrPh = 0, kScrKf = kScrPh + sizeof(double) * 2 * kHkNaMaxPhase,
                 kScrR = kScrKf + sizeof(double) * 3 * kHkNaMaxK, kScrBytes = kScrR + sizeof(int) * 3 * kHkNaMaxR;
static __device__ __align__(256) unsigned char scratch[kScrBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxScratchDevices] = {};

// (cos, sin) of 2 pi (kappa_k . n_q) reduced to [0, 1) turns, for every (k, q)
__global__ __launch_bounds__(256) void k_Hk_phases(int nk, int nR, const double *__restrict__ kf,
                                                   const int *__restrict__ n, double *__restrict__ ph)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nk * nR)
        return;
    const int k = i / nR, q = i - k * nR;
    double t = 0.0;
    for (int d = 0; d < 3; ++d)
        t += kf[3 * k + d] * (double)n[3 * q + d];
    t -= floor(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    ph[2 * (size_t)i] = cs;
    ph[2 * (size_t)i + 1] = sn;
}

hipError_t Hk_noalloc(hipStream_t s, int device, long long nel, int nR, const int *R, int nk, const double *kfrac,
                      const double *HR, double *Hk)
{
    if (device < 0 || device >= kMaxScratchDevices || nR > kHkNaMaxR || nk > kHkNaMaxK ||
        (long long)nR * nk > kHkNaMaxPhase)
        return hipErrorInvalidValue;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            // the caller made `device` current
            const hipError_t e = hipGetSymbolAddress((void **)&g_scratch_ptr[device], HIP_SYMBOL(scratch));
            if (e != hipSuccess) {
                g_scratch_ptr[device] = nullptr;
                return e;
            }
        }
        base = g_scratch_ptr[device];
    }
    double *ph = reinterpret_cast<double *>(base + kScrPh);
    double *kf = reinterpret_cast<double *>(base + kScrKf);
    int *n = reinterpret_cast<int *>(base + kScrR);
    hipError_t e = hipMemcpyAsync(kf, kfrac, sizeof(double) * 3 * nk, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(n, R, sizeof(int) * 3 * nR, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // the caller's host arrays outlive the copies
    if (e != hipSuccess)
        return e;
    const int np = nk * nR;
    hipLaunchKernelGGL(k_Hk_phases, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, nk, nR, kf, n, ph);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_Hk(s, nel, nR, nk, ph, HR, Hk);
}

template <typename T, int P>
static hipError_t launch_HR_p(hipStream_t s, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                              const int *img, const Basis &b, const int *wsh, const double *W, double wscale,
                              const HRMap &m, int norb, double *HR)
{
    const size_t lds = sizeof(T) * (size_t)nbmax * P * kRow;
    hipError_t e =
        hipFuncSetAttribute((const void *)k_HR_batch<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_HR_batch<T, P>), dim3((unsigned)(kXcd * ((g.nbatch + kXcd - 1) / kXcd))),
                       dim3(64 * kHRWaves), lds, s, g, iptr, img_atom, img, b, wsh, W, wscale, m, norb, HR);
    return hipGetLastError();
}

hipError_t launch_HR_batch(hipStream_t s, bool f32, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                           const int *img, const Basis &b, const int *wsh, const double *W, double wscale,
                           const HRMap &m, int norb, double *HR)
{
    if (g.P == 32)
        return f32 ? launch_HR_p<float, 32>(s, g, nbmax, iptr, img_atom, img, b, wsh, W, wscale, m, norb, HR)
                   : launch_HR_p<double, 32>(s, g, nbmax, iptr, img_atom, img, b, wsh, W, wscale, m, norb, HR);
    if (g.P == 16)
        return f32 ? launch_HR_p<float, 16>(s, g, nbmax, iptr, img_atom, img, b, wsh, W, wscale, m, norb, HR)
                   : launch_HR_p<double, 16>(s, g, nbmax, iptr, img_atom, img, b, wsh, W, wscale, m, norb, HR);
    return hipErrorInvalidValue;
}

}  // namespace gint
