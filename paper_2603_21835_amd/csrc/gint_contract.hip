// gint_contract.hip -- the grid contractions of Sec. 3.3.1 of arXiv:2603.21835
// on gfx950 matrix cores, and their reductions.  Orbital tiles, packed D and
// H block partials are FP64 (v_mfma_f64_16x16x4) or FP32
// (v_mfma_f32_16x16x4); sums across batches and all dot products are FP64.
//
//   H^loc   point-stationary: a workgroup owns a mesh batch and forms every
//           atom-pair block of it from orbitals evaluated once into LDS
//           (k_H_batch, k_H_batch16); one wave per owned atom pair then sums
//           the pair's blocks over its batches in a fixed order into dense
//           symmetric H (k_H_pairreduce).
//   rho     point-stationary: a workgroup owns a mesh batch, evaluates every
//           atom's folded orbitals there once into LDS and contracts all
//           atom-pair blocks against packed D + D^T fragments (k_batch).
//   force   point-stationary likewise: T_I = sum_J (D + D^T)_IJ phi_J per
//           batch, dotted with grad phi_I; per-(batch, atom) partials are
//           summed per atom in a fixed order (k_batch, k_force_reduce).
//
// MFMA lane layouts: see MM<T> in gint_device.h.
// Orbital tiles in LDS: H kernels [atom slot][point][orbital] (row pitch
// kRow = 16 elements, orbital o of point p in slot o ^ (p & 15)); rho /
// force [atom slot][16-point tile][orbital][point].  Either way the 64 lanes
// of one operand read touch 64 consecutive elements.
#include <hip/hip_runtime.h>

#include "gint_device.h"

namespace gint {

// workgroups for n batches dispatched XCD-contiguously (xcd_batch)
static unsigned xcd_grid(int n) { return (unsigned)(kXcd * ((n + kXcd - 1) / kXcd)); }

// One element of an H block partial.  FP64 partials are streamed out with
// non-temporal stores (each is read once, by the reduction, which measured
// faster that way); FP32 partials use ordinary stores.
template <typename T>
__device__ __forceinline__ void store_partial(T *p, T x)
{
    if constexpr (sizeof(T) == 8)
        __builtin_nontemporal_store(x, p);
    else
        *p = x;
}

// Advance (ia, ja) by st places in the row-major order of the pairs
// ia <= ja < nb (row ia holds ja = ia .. nb-1).
__device__ __forceinline__ void tri_advance(int &ia, int &ja, int st, int nb)
{
    ja += st;
    while (ja >= nb && ia < nb) {
        ++ia;
        ja += ia - nb;
    }
}

constexpr int kHWaves = 16;  // waves of the H block kernels

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
// k_H_pairreduce: each unordered atom pair has one owner; one wave per
// owned pair sums the pair's block partials over its batches in increasing
// batch order (fixed order, no atomics), then writes H_IJ and its mirror
// H_JI into the dense matrix, so H is exactly symmetric.

template <typename T, int P>
__global__ __launch_bounds__(64 * kHWaves) void k_H_batch(Geo g, Bins bn, Basis bs, const double *__restrict__ W,
                                                 double wscale, int b0, int b1, const int *__restrict__ boff, int mno,
                                                 T *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    T *s_phi = reinterpret_cast<T *>(s_dyn);  // [nbmax][P][kRow]
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_nor[kMaxBatchAtoms];
    __shared__ double s_w[kMaxP];

    // (the wave index through readfirstlane: known uniform, so that the
    // block bookkeeping that depends on it stays in scalar registers)
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6),
              nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int b = xcd_batch(blockIdx.x, b0, b1 - b0);
    if (b < 0)
        return;
    const int e0 = bn.bptr[b], nb = bn.bptr[b + 1] - e0;
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
        // orbital o of point p at row[o ^ (p & 15)] (swizzled: the stores of
        // consecutive points spread over the LDS banks)
        T *row = s_phi + (size_t)(a * P + p) * kRow;
        const int swz = p & 15;
        int n[3];
        const bool valid = batch_point(g, ib, p, n);
        const DevSpecies &S = s_sp[bs.spc[atom]];
        const int zlo = valid ? S.norb : 0;
        for (int o = zlo; o < kMaxOrb; ++o)
            row[o ^ swz] = (T)0;
        if (valid) {
            const int io = bn.ent_img[e];
            const int cnt = bn.ent_img[e + 1] - io;
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            double r[3];
            mesh_cart(g, n, r);
            eval_orbitals<T>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img, r,
                             row, swz);
        }
    }
    __syncthreads();

    // ---- every block (ia <= ja), in contiguous ranges over the waves ----
    const int nblk = nb * (nb + 1) / 2;
    int ia = 0, ja = 0;
    // a contiguous range of blocks per wave (triangle order): the left
    // operand changes only at the end of a row
    const int k0 = wave * nblk / nw, k1 = (wave + 1) * nblk / nw;
    tri_advance(ia, ja, k0, nb);
    const size_t mm = (size_t)block_pitch(mno, sizeof(T));
    // this lane's points are 4 kk + lk: their weights stay in registers
    // and the (swizzled) offsets of (point 4 kk + lk, orbital li)
    T wl[P / 4];
    int off[P / 4];
#pragma unroll
    for (int kk = 0; kk < P / 4; ++kk) {
        const int p = 4 * kk + lk;
        wl[kk] = (T)s_w[p];
        off[kk] = p * kRow + (li ^ (p & 15));
    }
    // a wave's consecutive blocks mostly share ia: its weighted operand
    // w phi_I stays in registers until ia changes
    int cur = -1;
    T aw[P / 4];
    for (int k = k0; k < k1; ++k) {
        if (ia != cur) {
            const T *pI = s_phi + (size_t)(ia * P) * kRow;
#pragma unroll
            for (int kk = 0; kk < P / 4; ++kk)
                aw[kk] = wl[kk] * pI[off[kk]];
            cur = ia;
        }
        const T *pJ = s_phi + (size_t)(ja * P) * kRow;
        T bv[P / 4];
#pragma unroll
        for (int kk = 0; kk < P / 4; ++kk)
            bv[kk] = pJ[off[kk]];
        typename MM<T>::acc acc = MM<T>::zero();
#pragma unroll
        for (int kk = 0; kk < P / 4; ++kk)
            acc = MM<T>::mma(aw[kk], bv[kk], acc);
        const int nI = s_nor[ia], nJ = s_nor[ja];
        T *o = part + (size_t)(boff[b] - boff[b0] + k) * mm;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = MM<T>::row(lk, v);
            if (row < nI && li < nJ)
                store_partial(o + row * mno + li, acc[v]);
        }
        if (++ja == nb) {
            ++ia;
            ja = ia;
        }
    }
}

// ---------------------------------------------------------------------------
// H^loc with 16-bit matrix-core operands (v_mfma_f32_16x16x32_{bf16,f16}),
// FP32 accumulation within a batch and FP64 across batches (k_H_pairreduce).
//
// With psi_p = sqrt|w_p| phi(p) and s_p = sign(w_p),
//     C_IJ = sum_p (s_p psi_I(p)) psi_J(p)^T,
// so one 16-bit tile per atom serves as both operands (the sign is a bit
// flip, exact).  In the split modes psi = hi + lo with hi = round16(psi) and
// lo = round16(psi - hi), and C = hi.hi + hi.lo + lo.hi (the lo.lo term is
// below the FP32 accumulation's rounding).  FP16 operands carry a 2^8 scale
// (removed exactly at the end) that keeps lo clear of the subnormal range.
//
// After the FP32 orbitals are staged, each atom's region is rewritten in
// place as planes [hi | lo][chunk 0..3][orbital 0..15][8 points]: lane
// l = 16 chunk + orbital then reads its whole operand (8 points of one
// orbital, k = 8 chunk + j) with one 16-byte load at plane + 16 l.  A batch
// holds exactly 32 points (the K of one instruction).

namespace {
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

// round-to-nearest-even FP32 -> BF16 bits (finite inputs)
__device__ __forceinline__ unsigned bf16_bits(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_value(unsigned h) { return __uint_as_float(h << 16); }

template <bool F16>
__device__ __forceinline__ void split16(float x, unsigned &hi, unsigned &lo)
{
    if (F16) {
        const _Float16 h = (_Float16)x;
        const _Float16 l = (_Float16)(x - (float)h);
        hi = __builtin_bit_cast(unsigned short, h);
        lo = __builtin_bit_cast(unsigned short, l);
    } else {
        hi = bf16_bits(x);
        lo = bf16_bits(x - bf16_value(hi));
    }
}

// v_mfma_f32_16x16x16_f16 on two 4-half operands held as 2 x 32 bits each
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f4 mma16k16(u2v a, u2v b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4v, a), __builtin_bit_cast(h4v, b), c, 0, 0,
                                                 0);
}

// FP16 hi/lo planes of four values (scaled by 2^8): {hi 0|1, hi 2|3, lo 0|1,
// lo 2|3}
__device__ __forceinline__ u4v split4_f16(float x0, float x1, float x2, float x3)
{
    unsigned h[4], l[4];
    const float x[4] = {x0, x1, x2, x3};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const _Float16 hv = (_Float16)(x[m] * 256.0f);
        const _Float16 lv = (_Float16)(x[m] * 256.0f - (float)hv);
        h[m] = __builtin_bit_cast(unsigned short, hv);
        l[m] = __builtin_bit_cast(unsigned short, lv);
    }
    return u4v{h[0] | (h[1] << 16), h[2] | (h[3] << 16), l[0] | (l[1] << 16), l[2] | (l[3] << 16)};
}

template <bool F16>
__device__ __forceinline__ f4 mma16(u4v a, u4v b, f4 c)
{
    if (F16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0,
                                                      0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c,
                                                       0, 0, 0);
}
}  // namespace

template <bool F16, bool SPLIT>
__global__ __launch_bounds__(64 * kHWaves) void k_H_batch16(Geo g, Bins bn, Basis bs, const double *__restrict__ W,
                                                   double wscale, int b0, int b1, const int *__restrict__ boff,
                                                   int mno, float *__restrict__ part)
{
    constexpr int P = 32;
    constexpr float kScale = F16 ? 256.0f : 1.0f;
    constexpr float kUnscale = 1.0f / (kScale * kScale);
    extern __shared__ __align__(16) unsigned char s_dyn[];
    float *s_phi = reinterpret_cast<float *>(s_dyn);  // [nbmax][P][kRow], then the 16-bit planes
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_nor[kMaxBatchAtoms];
    __shared__ float s_sw[P];
    __shared__ unsigned s_neg[P];

    // (the wave index through readfirstlane: known uniform, so that the
    // block bookkeeping that depends on it stays in scalar registers)
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6),
              nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int b = xcd_batch(blockIdx.x, b0, b1 - b0);
    if (b < 0)
        return;
    const int e0 = bn.bptr[b], nb = bn.bptr[b + 1] - e0;
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
        const double w = batch_point(g, ib, p, n) ? wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 0.0;
        s_sw[p] = (float)(sqrt(fabs(w)) * (double)kScale);
        s_neg[p] = w < 0.0 ? 1u : 0u;
    }
    __syncthreads();

    for (int idx = tid; idx < nb * P; idx += blockDim.x) {
        const int a = idx / P, p = idx % P;
        const int e = e0 + a;
        const int atom = s_atom[a];
        float *row = s_phi + (size_t)(a * P + p) * kRow;  // swizzled as in k_H_batch
        const int swz = p & 15;
        int n[3];
        const bool valid = batch_point(g, ib, p, n);
        const DevSpecies &S = s_sp[bs.spc[atom]];
        const int zlo = valid ? S.norb : 0;
        for (int o = zlo; o < kMaxOrb; ++o)
            row[o ^ swz] = 0.0f;
        if (valid) {
            const int io = bn.ent_img[e];
            const int cnt = bn.ent_img[e + 1] - io;
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            double r[3];
            mesh_cart(g, n, r);
            eval_orbitals<float>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img,
                                 r, row, swz);
        }
    }
    __syncthreads();

    // ---- in place: FP32 [p][orbital] -> 16-bit planes, one wave per atom ----
    // (a wave reads its atom's region completely before it writes it)
    for (int a = wave; a < nb; a += nw) {
        float *reg = s_phi + (size_t)a * P * kRow;
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            v[j] = reg[(8 * lk + j) * kRow + (li ^ ((8 * lk + j) & 15))] * s_sw[8 * lk + j];
        unsigned hi[8], lo[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            split16<F16>(v[j], hi[j], lo[j]);
        u4v H, L;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            H[d] = hi[2 * d] | (hi[2 * d + 1] << 16);
            L[d] = lo[2 * d] | (lo[2 * d + 1] << 16);
        }
        u4v *pl = reinterpret_cast<u4v *>(reg);
        pl[lane] = H;
        pl[64 + lane] = L;
    }
    // the sign of w at this lane's eight points, as a mask on packed pairs
    u4v neg;
#pragma unroll
    for (int d = 0; d < 4; ++d)
        neg[d] = (s_neg[8 * lk + 2 * d] << 15) | (s_neg[8 * lk + 2 * d + 1] << 31);
    __syncthreads();

    const int nblk = nb * (nb + 1) / 2;
    int ia = 0, ja = 0;
    tri_advance(ia, ja, wave, nb);
    const int mm = block_pitch(mno, sizeof(float));
    const u4v *pl = reinterpret_cast<const u4v *>(s_phi);
    const int apitch = P * kRow / 4;  // u4v per atom region
    // this wave's block in LDS (row-major, pitch mno) past the batch's
    // planes, streamed out as one contiguous run of 16-byte stores
    float *s_hb = s_phi + (size_t)nb * P * kRow + kMaxOrb * kMaxOrb * wave;
    for (int k = wave; k < nblk; k += nw) {
        const u4v aH = pl[ia * apitch + lane] ^ neg;
        const u4v bH = pl[ja * apitch + lane];
        f4 acc = f4{0.0f, 0.0f, 0.0f, 0.0f};
        acc = mma16<F16>(aH, bH, acc);
        if (SPLIT) {
            const u4v aL = pl[ia * apitch + 64 + lane] ^ neg;
            const u4v bL = pl[ja * apitch + 64 + lane];
            acc = mma16<F16>(aH, bL, acc);
            acc = mma16<F16>(aL, bH, acc);
        }
        const int nI = s_nor[ia], nJ = s_nor[ja];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * lk + v;
            if (row < nI && li < nJ)
                s_hb[row * mno + li] = acc[v] * kUnscale;
        }
        // (wave-level fences: the reads below see the writes above, and the
        // next block's writes follow them)
        wave_lds_sync();
        if (4 * lane < mm) {
            f4 *o = reinterpret_cast<f4 *>(part) + ((size_t)(boff[b] - boff[b0] + k) * mm >> 2);
            __builtin_nontemporal_store(*reinterpret_cast<const f4 *>(s_hb + 4 * lane), o + lane);
        }
        wave_lds_sync();
        tri_advance(ia, ja, nw, nb);
    }
}

template <bool F16, bool SPLIT>
static hipError_t launch_H16_t(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int b0, int b1,
                               const double *W, double wscale, const int *boff, int mno, void *part)
{
    // the batch's tiles (then its planes), then one block per wave
    const size_t lds = sizeof(float) * ((size_t)nbmax * g.P * kRow + kMaxOrb * kMaxOrb * kHWaves);
    hipError_t e = hipFuncSetAttribute((const void *)k_H_batch16<F16, SPLIT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_H_batch16<F16, SPLIT>), dim3(xcd_grid(b1 - b0)), dim3(64 * kHWaves), lds, s, g, bn, b, W, wscale,
                       b0, b1, boff, mno, static_cast<float *>(part));
    return hipGetLastError();
}

template <typename T, int P>
static hipError_t launch_H_batch_p(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int b0,
                                   int b1, const double *W, double wscale, const int *boff, int mno, void *part)
{
    const size_t lds = sizeof(T) * (size_t)nbmax * P * kRow;
    hipError_t e =
        hipFuncSetAttribute((const void *)k_H_batch<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_H_batch<T, P>), dim3(xcd_grid(b1 - b0)), dim3(64 * kHWaves), lds, s, g, bn, b, W, wscale, b0, b1,
                       boff, mno, static_cast<T *>(part));
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_H_batch_t(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int b0,
                                   int b1, const double *W, double wscale, const int *boff, int mno, void *part)
{
    if (g.P == 32)
        return launch_H_batch_p<T, 32>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
    if (g.P == 16)
        return launch_H_batch_p<T, 16>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
    return hipErrorInvalidValue;
}

static hipError_t launch_H_packed(hipStream_t s, int mode, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                                  int b0, int b1, const double *W, double wscale, const int *boff, int mno,
                                  void *part);

hipError_t launch_H_batch(hipStream_t s, int mode, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int b0,
                          int b1, const double *W, double wscale, const int *boff, int mno, void *part)
{
    if (b1 <= b0)
        return hipSuccess;
    if (mode != kModeF64 && mode != kModeF32 && g.P != 32)
        return hipErrorInvalidValue;
    if (mode == kModeF32) {
        // FP32: the packed-row form where the batch's tiles fit it (the same
        // bits; 16.0 -> 14.8 ms at Si-512).  In FP64 the per-block form is
        // faster (19.6 against 32.0 ms), so it stays.
        const hipError_t e = launch_H_packed(s, mode, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
        if (e != hipErrorNotSupported)
            return e;
    }
    switch (mode) {
    case kModeF64: return launch_H_batch_t<double>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
    case kModeF32: return launch_H_batch_t<float>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
    case kModeBF16: return launch_H16_t<false, false>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
    case kModeF16: return launch_H16_t<true, false>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
    case kModeBF16x3: return launch_H16_t<false, true>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
    case kModeF16x3: return launch_H16_t<true, true>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff, mno, part);
    default: return hipErrorInvalidValue;
    }
}

// H^loc: fixed-order sums of the block partials.  One wave per owned atom
// pair (I, J) walks the pair's block list (batch order) restricted to the
// block range [q0, q1) and streams each stored block whole with 16-byte
// loads (lane l owns stored elements V l .. V l + V - 1, V = 16 / element
// size, and every 64 V further), summing the blocks stored as H_IJ and those
// stored as H_JI separately, each in list order; the two sums meet through
// LDS.  It writes H_IJ and its mirror H_JI (for J = I only the upper
// triangle, mirrored).
constexpr int kRedGroup = 16;  // list entries whose loads are in flight together

template <typename T>
struct Vec16;
// FP64 partials are read once: their loads are marked non-temporal (and
// their stores too, see store_partial).  FP32 partials keep ordinary loads
// and stores, which measured faster for them.
template <>
struct Vec16<double> {
    typedef double2 type;
    typedef double nt_type __attribute__((ext_vector_type(2)));
    static constexpr int V = 2;
    static __device__ __forceinline__ double at(const double2 &x, int i) { return i ? x.y : x.x; }
    static __device__ __forceinline__ double2 load(const double *p)
    {
        const nt_type x = __builtin_nontemporal_load(reinterpret_cast<const nt_type *>(p));
        return double2{x[0], x[1]};
    }
};
template <>
struct Vec16<float> {
    typedef float4 type;
    static constexpr int V = 4;
    static __device__ __forceinline__ double at(const float4 &x, int i)
    {
        return (double)(i == 0 ? x.x : (i == 1 ? x.y : (i == 2 ? x.z : x.w)));
    }
};

template <typename T>
__global__ __launch_bounds__(256) void k_H_pairreduce(int npair, const int *__restrict__ order,
                                                      const int *__restrict__ pown,
                                                      const int *__restrict__ plist, const int *__restrict__ lsl,
                                                      int nslab1, int si, const int *__restrict__ list, Basis bs,
                                                      int mno, int norb, const T *__restrict__ part, int q0,
                                                      int accumulate, double *__restrict__ H)
{
    typedef typename Vec16<T>::type VT;
    constexpr int V = Vec16<T>::V;
    constexpr int M = (kMaxOrb * kMaxOrb + 64 * V - 1) / (64 * V);  // vectors per lane
    __shared__ double s_sum[4][2][kMaxOrb * kMaxOrb];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int w = blockIdx.x * 4 + wv;
    if (w >= npair)
        return;
    const int p = order ? order[w] : w;
    auto qof = [](int c) { return c >= 0 ? c : -c - 1; };
    const int l0 = lsl[(size_t)p * nslab1 + si], l1 = lsl[(size_t)p * nslab1 + si + 1];
    if (accumulate && l0 == l1)
        return;
    const int pitch = block_pitch(mno, sizeof(T));
    double up[M][V], dn[M][V];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int i = 0; i < V; ++i)
            up[m][i] = dn[m][i] = 0.0;
    // list entries 64 at a time, one per lane, handed out with readlane:
    // the block loads of a group do not wait on list loads
    for (int kc = l0; kc < l1; kc += 64) {
        const int nc = min(64, l1 - kc);
        const int lcode = lane < nc ? list[kc + lane] : 0;
        for (int k0 = 0; k0 < nc; k0 += kRedGroup) {
        VT v[kRedGroup][M];
        bool isup[kRedGroup];
#pragma unroll
        for (int g = 0; g < kRedGroup; ++g) {
            const int k = k0 + g;
            const bool ok = k < nc;
            const int code = __builtin_amdgcn_readlane(lcode, ok ? k : 0);
            isup[g] = code >= 0;
            const T *blk = part + (size_t)(qof(code) - q0) * pitch;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int e = V * lane + 64 * V * m;
                if constexpr (sizeof(T) == 8)
                    v[g][m] = (ok && e < pitch) ? Vec16<T>::load(blk + e) : VT{};
                else
                    v[g][m] = (ok && e < pitch) ? *reinterpret_cast<const VT *>(blk + e) : VT{};
            }
        }
#pragma unroll
        for (int g = 0; g < kRedGroup; ++g)
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    const double x = Vec16<T>::at(v[g][m], i);
                    if (isup[g])
                        up[m][i] += x;
                    else
                        dn[m][i] += x;
                }
        }
    }
    // H_IJ(r, c) = up(r mno + c) + dn(c mno + r)
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int e = V * lane + 64 * V * m + i;
            if (e < kMaxOrb * kMaxOrb) {
                s_sum[wv][0][e] = up[m][i];
                s_sum[wv][1][e] = dn[m][i];
            }
        }
    // the sums of other lanes of this wave are read below: order the LDS
    // stores before those loads (a wave-level barrier; the per-wave early
    // exits rule out a workgroup barrier)
    wave_lds_sync();
    const int I = pown[p], J = plist[p];
    const int Iin = bs.perm[I], Jin = bs.perm[J];
    const int mu0 = bs.orb0[Iin], nI = bs.orb0[Iin + 1] - mu0;
    const int nu0 = bs.orb0[Jin], nJ = bs.orb0[Jin + 1] - nu0;
    const int mm = mno * mno;
    for (int e = lane; e < mm; e += 64) {
        const int r = e / mno, c = e - r * mno;
        if (r < nI && c < nJ && !(J == I && c < r)) {
            const double sum = s_sum[wv][0][e] + s_sum[wv][1][c * mno + r];
            const size_t i1 = (size_t)(mu0 + r) * norb + nu0 + c;
            const size_t i2 = (size_t)(nu0 + c) * norb + mu0 + r;
            const double val = accumulate ? H[i1] + sum : sum;
            H[i1] = val;
            H[i2] = val;
        }
    }
}

hipError_t launch_H_pairreduce(hipStream_t s, bool f32, int npair, const int *order, const int *pown,
                               const int *plist, const int *lsl, int nslab, int si, const int *list, const Basis &b,
                               int mno, int norb, const void *part, int q0, int accumulate, double *H)
{
    if (npair <= 0)
        return hipSuccess;
    const unsigned nblk = (unsigned)((npair + 3) / 4);
    if (f32)
        hipLaunchKernelGGL(k_H_pairreduce<float>, dim3(nblk), dim3(256), 0, s, npair, order, pown, plist, lsl,
                           nslab + 1, si, list, b, mno, norb, static_cast<const float *>(part), q0, accumulate, H);
    else
        hipLaunchKernelGGL(k_H_pairreduce<double>, dim3(nblk), dim3(256), 0, s, npair, order, pown, plist, lsl,
                           nslab + 1, si, list, b, mno, norb, static_cast<const double *>(part), q0, accumulate, H);
    return hipGetLastError();
}

// H(R): one wave per canonical triple (I, J, R) (key of k_HR_keys) sums the
// triple's block partials in their sorted (batch) order, streaming each
// block whole like k_H_pairreduce, and writes H_IJ(R) and its transpose
// H_JI(-R) for the listed R (for I = J and R = 0 the upper triangle,
// mirrored).
template <typename T>
__global__ __launch_bounds__(256) void k_HR_reduce(int ntri, const int *__restrict__ order,
                                                   const unsigned long long *__restrict__ tkey,
                                                   const int *__restrict__ tstart, const int *__restrict__ list,
                                                   int natom, HRMap hm, Basis bs, int mno, int norb,
                                                   const T *__restrict__ part, double *__restrict__ HR)
{
    typedef typename Vec16<T>::type VT;
    constexpr int V = Vec16<T>::V;
    constexpr int M = (kMaxOrb * kMaxOrb + 64 * V - 1) / (64 * V);  // vectors per lane
    constexpr int B = kHRBox, w = 2 * kHRBox + 1;
    __shared__ double s_sum[4][2][kMaxOrb * kMaxOrb];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int slot = blockIdx.x * 4 + wv;
    if (slot >= ntri)
        return;
    const int t = order ? order[slot] : slot;
    const unsigned long long key = tkey[t];
    const int ridx = (int)(key & 0x3ffffULL);
    const long long ij = (long long)(key >> 18);
    const int I = (int)(ij / natom), J = (int)(ij - (long long)I * natom);
    const int R0 = ridx / (w * w) - B, R1 = (ridx / w) % w - B, R2 = ridx % w - B;
    const bool self = I == J && R0 == 0 && R1 == 0 && R2 == 0;
    const int qo = hr_lookup(hm, R0, R1, R2);
    const int qm = self ? -1 : hr_lookup(hm, -R0, -R1, -R2);
    if (qo < 0 && qm < 0)
        return;
    auto qof = [](int c) { return c >= 0 ? c : -c - 1; };
    const int l0 = tstart[t], l1 = tstart[t + 1];
    const int pitch = block_pitch(mno, sizeof(T));
    double up[M][V], dn[M][V];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int i = 0; i < V; ++i)
            up[m][i] = dn[m][i] = 0.0;
    for (int kc = l0; kc < l1; kc += 64) {
        const int nc = min(64, l1 - kc);
        const int lcode = lane < nc ? list[kc + lane] : 0;
        for (int k0 = 0; k0 < nc; k0 += kRedGroup) {
            VT v[kRedGroup][M];
            bool isup[kRedGroup];
#pragma unroll
            for (int g = 0; g < kRedGroup; ++g) {
                const int k = k0 + g;
                const bool ok = k < nc;
                const int code = __builtin_amdgcn_readlane(lcode, ok ? k : 0);
                isup[g] = code >= 0;
                const T *blk = part + (size_t)qof(code) * pitch;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int e = V * lane + 64 * V * m;
                    if constexpr (sizeof(T) == 8)
                        v[g][m] = (ok && e < pitch) ? Vec16<T>::load(blk + e) : VT{};
                    else
                        v[g][m] = (ok && e < pitch) ? *reinterpret_cast<const VT *>(blk + e) : VT{};
                }
            }
#pragma unroll
            for (int g = 0; g < kRedGroup; ++g)
#pragma unroll
                for (int m = 0; m < M; ++m)
#pragma unroll
                    for (int i = 0; i < V; ++i) {
                        const double x = Vec16<T>::at(v[g][m], i);
                        if (isup[g])
                            up[m][i] += x;
                        else
                            dn[m][i] += x;
                    }
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int e = V * lane + 64 * V * m + i;
            if (e < kMaxOrb * kMaxOrb) {
                s_sum[wv][0][e] = up[m][i];
                s_sum[wv][1][e] = dn[m][i];
            }
        }
    wave_lds_sync();  // other lanes' sums are read below
    const int mu0 = bs.orb0[I], nI = bs.orb0[I + 1] - mu0;
    const int nu0 = bs.orb0[J], nJ = bs.orb0[J + 1] - nu0;
    const size_t nn = (size_t)norb * norb;
    const int mm = mno * mno;
    for (int e = lane; e < mm; e += 64) {
        const int r = e / mno, c = e - r * mno;
        if (r < nI && c < nJ && !(self && c < r)) {
            const double sum = s_sum[wv][0][e] + s_sum[wv][1][c * mno + r];
            if (qo >= 0) {
                HR[qo * nn + (size_t)(mu0 + r) * norb + nu0 + c] = sum;
                if (self)
                    HR[qo * nn + (size_t)(nu0 + c) * norb + mu0 + r] = sum;
            }
            if (qm >= 0)
                HR[qm * nn + (size_t)(nu0 + c) * norb + mu0 + r] = sum;
        }
    }
}

hipError_t launch_HR_reduce(hipStream_t s, bool f32, int ntri, const int *order, const unsigned long long *tkey,
                            const int *tstart, const int *list, int natom, const HRMap &m, const Basis &b, int mno,
                            int norb, const void *part, double *HR)
{
    if (ntri <= 0)
        return hipSuccess;
    const unsigned nblk = (unsigned)((ntri + 3) / 4);
    if (f32)
        hipLaunchKernelGGL(k_HR_reduce<float>, dim3(nblk), dim3(256), 0, s, ntri, order, tkey, tstart, list, natom, m,
                           b, mno, norb, static_cast<const float *>(part), HR);
    else
        hipLaunchKernelGGL(k_HR_reduce<double>, dim3(nblk), dim3(256), 0, s, ntri, order, tkey, tstart, list, natom,
                           m, b, mno, norb, static_cast<const double *>(part), HR);
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

// The same fragments as FP16 hi/lo planes for the 16-bit T of the FP16 hi/lo
// mode: per (block, orientation) 64 lanes of 16 bytes, lane (i, k0) holding
// the four values (i, k0 + 4 m), m = 0..3, of the FP32 form's lane (i, k0)
__global__ __launch_bounds__(128) void k_pack_S2_h16(Geo g, Bins bn, Basis bs, const double *__restrict__ D,
                                                     int norb, u4v *__restrict__ pk)
{
    const int pair = blockIdx.x >> 4, blk = blockIdx.x & 15;
    const int A = bn.pairA[pair], B = bn.pairB[pair];
    const int sX = blk >> 2, sY = blk & 3;
    const int X = A * kGroup + sX, Y = B * kGroup + sY;
    const int o = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const bool ok = X < g.natom && Y < g.natom && !(A == B && sX > sY);
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (ok) {
        const int Xin = bs.perm[X], Yin = bs.perm[Y];
        const int mx = bs.orb0[Xin], nx = bs.orb0[Xin + 1] - mx;
        const int my = bs.orb0[Yin], ny = bs.orb0[Yin + 1] - my;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int kb = lk + 4 * m;
            if (o == 0 && li < nx && kb < ny)
                v[m] = (float)(D[(size_t)(mx + li) * norb + my + kb] + D[(size_t)(my + kb) * norb + mx + li]);
            if (o == 1 && kb < nx && li < ny)
                v[m] = (float)(D[(size_t)(mx + kb) * norb + my + li] + D[(size_t)(my + li) * norb + mx + kb]);
        }
    }
    pk[((size_t)blockIdx.x * 2 + o) * 64 + lane] = split4_f16(v[0], v[1], v[2], v[3]);
}

hipError_t launch_pack_S2_h16(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int npair,
                              const double *D, int norb, void *pk)
{
    if (npair <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pack_S2_h16, dim3(npair * 16), dim3(128), 0, s, g, bn, b, D, norb, static_cast<u4v *>(pk));
    return hipGetLastError();
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
// Point-stationary rho and force: one workgroup (8 waves) per mesh batch.
// The folded orbitals of every atom reaching the batch are evaluated once
// into LDS at all P points; each D + D^T fragment a wave loads is applied to
// all P/16 sixteen-point tiles of the batch, and the next block's fragment is
// loaded while the current one is in use.

// waves of k_batch (one workgroup per CU): rho 16, the force (more registers) 12
template <int MODE>
constexpr int batch_waves() { return MODE == 0 ? 16 : 12; }
// what k_batch computes: rho; the force; both (the force's T_I also gives
// rho_p = 1/2 sum_I phi_I(p) . T_I(p), since sum_IJ phi_I S2_IJ phi_J = 2 rho_p)
constexpr int kRho = 0, kForce = 1, kRhoForce = 2;

template <int MODE, typename T, int P>
__global__ __launch_bounds__(64 * batch_waves<MODE>()) void k_batch(Geo g, Bins bn, Basis bs, const T *__restrict__ pk,
                                                            const double *__restrict__ W, double wscale,
                                                            double *__restrict__ out, double *__restrict__ rho2)
{
    constexpr bool FORCE = MODE != kRho, RHO = MODE != kForce;
    constexpr int kBatchWaves = batch_waves<MODE>();
    constexpr int NT = 64 * kBatchWaves;
    constexpr int NS = P / 16;  // sixteen-point tiles per batch
    extern __shared__ __align__(16) unsigned char s_dyn[];
    T *s_phi = reinterpret_cast<T *>(s_dyn);  // [nbmax][P / 16][16 orbitals][16 points]
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_grank[kMaxBatchAtoms];
    __shared__ int s_ptab[kMaxBatchGroups * kMaxBatchGroups];
    __shared__ double s_red[RHO ? kBatchWaves : 1][kMaxP];
    __shared__ double s_w[kMaxP];
    __shared__ double s_F[FORCE ? kMaxBatchAtoms : 1][3];

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int b = xcd_batch(blockIdx.x, 0, g.nbatch);
    if (b < 0)
        return;
    const int e0 = bn.bptr[b], nb = bn.bptr[b + 1] - e0;
    const int g0 = bn.bgptr[b], ngb = bn.bgptr[b + 1] - g0;
    int ib[3];
    batch_coords(g, b, ib);

    for (int k = tid; k < g.nrad; k += NT)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += NT)
        s_sp[k] = bs.sp[k];
    for (int a = tid; a < nb; a += NT) {
        const int atom = bn.ent_atom[e0 + a];
        s_atom[a] = atom;
        s_grank[a] = lower_bound_i(bn.bgrp, g0, g0 + ngb, atom / kGroup) - g0;
        if (FORCE)
            s_F[a][0] = s_F[a][1] = s_F[a][2] = 0.0;
    }
    for (int k = tid; k < ngb * ngb; k += NT) {
        const int ra = k / ngb, rb = k % ngb;
        const int ga = bn.bgrp[g0 + ra], gb = bn.bgrp[g0 + rb];
        s_ptab[k] = (ra <= rb) ? bn.pair_index[(size_t)ga * g.ngroup + gb] : -1;
    }
    if (FORCE)
        for (int p = tid; p < P; p += NT) {
            int n[3];
            s_w[p] = batch_point(g, ib, p, n) ? wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 0.0;
        }
    __syncthreads();

    // ---- stage the folded orbitals of every atom at every batch point ----
    for (int idx = tid; idx < nb * P; idx += NT) {
        const int a = idx / P, p = idx % P;
        const int e = e0 + a;
        const int atom = s_atom[a];
        // orbital o of this point at row[16 o]
        T *row = s_phi + (size_t)(a * NS + (p >> 4)) * 256 + (p & 15);
        int n[3];
        const bool valid = batch_point(g, ib, p, n);
        const DevSpecies &S = s_sp[bs.spc[atom]];
        const int zlo = valid ? S.norb : 0;
        for (int o = zlo; o < kMaxOrb; ++o)
            row[16 * o] = (T)0;
        if (valid) {
            const int io = bn.ent_img[e];
            const int cnt = bn.ent_img[e + 1] - io;
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            double r[3];
            mesh_cart(g, n, r);
            eval_orbitals<T, 16>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img,
                                 r, row);
        }
    }
    __syncthreads();
    // tile s2 of atom slot x: element (orbital o, point q) at [16 o + q]
    auto tile = [&](int x, int s2) -> const T * { return s_phi + (size_t)(x * NS + s2) * 256; };

    // fragment f of block (x, y) in orientation o (0: S2_XY, 1: S2_YX as A)
    auto frag = [&](int x, int y, int o) -> const T * {
        const int X = s_atom[x], Y = s_atom[y];
        const int pr = s_ptab[s_grank[x] * ngb + s_grank[y]];  // active: both groups reach the batch
        const int blk = (X % kGroup) * 4 + (Y % kGroup);
        return pk + ((size_t)(pr * 16 + blk) * 2 + o) * 256 + lane;
    };

    if (!FORCE) {
        // rho_p = sum_{I<J} phi_I . (S2_IJ phi_J) + 1/2 sum_I phi_I . (S2_II phi_I)
        double rp[NS];
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2)
            rp[s2] = 0.0;
        const int nblk = nb * (nb + 1) / 2;
        // this wave's blocks k = wave, wave + 8, ... as (ia <= ja); two
        // fragment register sets alternate so that the next block's loads
        // are in flight while the current block is on the matrix cores
        int ia = 0, ja = 0;
        auto advance = [&](int &x, int &y) { tri_advance(x, y, kBatchWaves, nb); };
        tri_advance(ia, ja, wave, nb);
        // (the scheduling barrier keeps the loads where they are issued: plain
        // scheduling would sink them to their first use, one block later)
        auto load = [&](T (&f4)[4], int x, int y) {
            const T *f = frag(x, y, 0);
#pragma unroll
            for (int c = 0; c < 4; ++c)
                f4[c] = f[64 * c];
            __builtin_amdgcn_sched_barrier(0);
        };
        auto block = [&](const T (&f4)[4], int x, int y) {
            const double half = (x == y) ? 0.5 : 1.0;
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                // B[k][j] = phi_y(orbital 4c + k, point j): k = lk, j = li
                const T *pJ = tile(y, s2) + 16 * lk + li;
                typename MM<T>::acc u = MM<T>::zero();
                u = MM<T>::mma(f4[0], pJ[0], u);
                u = MM<T>::mma(f4[1], pJ[64], u);
                u = MM<T>::mma(f4[2], pJ[128], u);
                u = MM<T>::mma(f4[3], pJ[192], u);
                const T *pI = tile(x, s2) + li;
                double dot = 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    dot += (double)u[v] * (double)pI[16 * MM<T>::row(lk, v)];
                rp[s2] += half * dot;
            }
        };
        // (one exit, no break between a load and its use; past the end a
        // valid fragment is reloaded)
        T fa[4], fb[4];
        if (wave < nblk) {
            load(fa, ia, ja);
            int k = wave;
            for (; k + kBatchWaves < nblk; k += 2 * kBatchWaves) {
                int ib2 = ia, jb2 = ja;
                advance(ib2, jb2);
                load(fb, ib2, jb2);
                block(fa, ia, ja);
                ia = ib2;
                ja = jb2;
                advance(ia, ja);
                const bool has_a = k + 2 * kBatchWaves < nblk;
                load(fa, has_a ? ia : ib2, has_a ? ja : jb2);
                block(fb, ib2, jb2);
            }
            if (k < nblk)
                block(fa, ia, ja);
        }
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) {
            double v = rp[s2];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lane < 16)
                s_red[wave][16 * s2 + lane] = v;
        }
        __syncthreads();
        for (int p = tid; p < P; p += NT) {
            int n[3];
            if (batch_point(g, ib, p, n)) {
                double v = s_red[0][p];
                for (int w = 1; w < kBatchWaves; ++w)
                    v += s_red[w][p];
                out[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] = v;
            }
        }
    } else {
        // dE/dR_I partial = -sum_p w_p grad phi_I(p) . T_I(p),  T_I = sum_J S2_IJ phi_J
        double rp[NS];
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2)
            rp[s2] = 0.0;
        for (int ia = wave; ia < nb; ia += kBatchWaves) {
            const int I = s_atom[ia];
            typename MM<T>::acc Tt[NS];
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2)
                Tt[s2] = MM<T>::zero();
            // T_I over every ja; fragment register sets alternate as in rho
            auto load = [&](T (&f4)[4], int y) {
                // (selects, not branches: the loads stay in one basic block
                // ahead of the scheduling barrier)
                const T *f = frag(min(ia, y), max(ia, y), ia <= y ? 0 : 1);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    f4[c] = f[64 * c];
                __builtin_amdgcn_sched_barrier(0);
            };
            auto block = [&](const T (&f4)[4], int y) {
#pragma unroll
                for (int s2 = 0; s2 < NS; ++s2) {
                    const T *pJ = tile(y, s2) + 16 * lk + li;
                    Tt[s2] = MM<T>::mma(f4[0], pJ[0], Tt[s2]);
                    Tt[s2] = MM<T>::mma(f4[1], pJ[64], Tt[s2]);
                    Tt[s2] = MM<T>::mma(f4[2], pJ[128], Tt[s2]);
                    Tt[s2] = MM<T>::mma(f4[3], pJ[192], Tt[s2]);
                }
            };
            // (one exit, no break between a load and its use: the
            // accumulators then stay in place instead of being copied)
            T fa[4], fb[4];
            load(fa, 0);
            int ja = 0;
            for (; ja + 1 < nb; ja += 2) {
                load(fb, ja + 1);
                block(fa, ja);
                load(fa, ja + 2 < nb ? ja + 2 : ja + 1);  // past the end: any valid fragment
                block(fb, ja + 1);
            }
            if (ja < nb)
                block(fa, ja);
            // gradients of orbitals row(lk, v) of atom I at point 16 s + li
            const int e = e0 + ia;
            const DevSpecies &S = s_sp[bs.spc[I]];
            const double X[3] = {bs.xw[3 * I], bs.xw[3 * I + 1], bs.xw[3 * I + 2]};
            const int io = bn.ent_img[e];
            double fx[3] = {0.0, 0.0, 0.0};
            // one tile at a time (the gradient code is large): select its T
#pragma unroll 1
            for (int s2 = 0; s2 < NS; ++s2) {
                typename MM<T>::acc Tc = Tt[0];
#pragma unroll
                for (int q = 1; q < NS; ++q)
                    if (q == s2)
                        Tc = Tt[q];
                if (RHO) {
                    const T *pI = tile(ia, s2) + li;
                    double dot = 0.0;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        dot += (double)Tc[v] * (double)pI[16 * MM<T>::row(lk, v)];
#pragma unroll
                    for (int q = 0; q < NS; ++q)
                        if (q == s2)
                            rp[q] += dot;
                }
                int n[3];
                const bool pvalid = batch_point(g, ib, 16 * s2 + li, n);
                double r[3];
                mesh_cart(g, n, r);
                const int cnt = pvalid ? bn.ent_img[e + 1] - io : 0;
                const double wp = s_w[16 * s2 + li];
                const double wv[4] = {wp * (double)Tc[0], wp * (double)Tc[1], wp * (double)Tc[2],
                                      wp * (double)Tc[3]};
                grad4_dot(g, s_rad, S.orb_rad, S.orb_m, S.norb, S.rc, bs.coef, X, cnt, bn.img[io], io, bn.img, r,
                          MM<T>::row(lk, 0), MM<T>::row(lk, 1) - MM<T>::row(lk, 0), wv, fx);
            }
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                double v = fx[x];
                for (int o = 32; o > 0; o >>= 1)
                    v += __shfl_xor(v, o);
                fx[x] = v;
            }
            if (lane == 0) {
                s_F[ia][0] = -fx[0];
                s_F[ia][1] = -fx[1];
                s_F[ia][2] = -fx[2];
            }
        }
        if (RHO) {
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                double v = rp[s2];
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                if (lane < 16)
                    s_red[wave][16 * s2 + lane] = v;
            }
        }
        __syncthreads();
        for (int k = tid; k < nb * 3; k += NT)
            out[(size_t)(e0 + k / 3) * 3 + k % 3] = s_F[k / 3][k % 3];
        if (RHO)
            for (int p = tid; p < P; p += NT) {
                int n[3];
                if (batch_point(g, ib, p, n)) {
                    double v = s_red[0][p];
                    for (int w = 1; w < kBatchWaves; ++w)
                        v += s_red[w][p];
                    rho2[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] = 0.5 * v;
                }
            }
    }
}

size_t batch_lds_bytes(int nbmax, int P, bool f32) { return (f32 ? 4 : 8) * (size_t)nbmax * P * kMaxOrb; }

template <int MODE, typename T, int P>
static hipError_t launch_batch_p(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                                 const void *pk, const double *W, double wscale, double *out, double *rho2)
{
    const size_t lds = sizeof(T) * (size_t)nbmax * P * kMaxOrb;
    hipError_t e = hipFuncSetAttribute((const void *)k_batch<MODE, T, P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_batch<MODE, T, P>), dim3(xcd_grid(g.nbatch)), dim3(64 * batch_waves<MODE>()), lds, s, g, bn,
                       b, static_cast<const T *>(pk), W, wscale, out, rho2);
    return hipGetLastError();
}

template <int MODE, typename T>
static hipError_t launch_batch_t(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                                 const void *pk, const double *W, double wscale, double *out, double *rho2)
{
    if (g.P == 32)
        return launch_batch_p<MODE, T, 32>(s, g, bn, b, nbmax, pk, W, wscale, out, rho2);
    if (g.P == 16)
        return launch_batch_p<MODE, T, 16>(s, g, bn, b, nbmax, pk, W, wscale, out, rho2);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Point-stationary force (and rho) with packed output rows.
//
// The orbitals of the atoms reaching a batch are numbered consecutively
// (atom slot a owns rows off[a] .. off[a] + norb_a - 1), and the output of
// T_I = sum_J S2_IJ phi_J is tiled over these packed rows, so that the
// 16-row matrix-core tiles carry no per-atom padding in the output; the
// contraction runs atom by atom (16 orbital slots, zero beyond norb).
//   phase A: for every 16-row tile, T over all atoms J; the left operand is
//            gathered per lane (a tile's rows may belong to several atoms)
//            from the packed D + D^T blocks, the next atom's values in
//            flight during the current one; the right operand is phi_J in
//            LDS.  Each wave keeps the T of its (at most KU) tiles in
//            registers; rho_p = 1/2 sum_r phi_r(p) T_r(p).
//   phase B: T replaces phi in LDS; one thread per (atom, point) evaluates
//            every orbital gradient of its atom there (one spline
//            evaluation per radial) against w_p T, and the P threads of an
//            atom sum their dot products.
// LDS: phi / T as [atom][P / 16 point tiles][16 orbitals][16 points].

constexpr int kForceWaves = 12;
// 16 x 16 (orbital x point) tiles with a row pitch of 17 elements: operand
// reads along points (the force's right operand, T) and along orbitals (the
// H operands) are both free of bank conflicts
constexpr int kPitch = 17, kTile = 16 * kPitch;

// bytes of the phi / T tiles and the slot-pair table of k_force_packed, i.e.
// where the 16-bit H planes start (16-byte aligned)
__host__ __device__ inline size_t h16_plane_offset(size_t esz, int nbmax, int P)
{
    const size_t b = esz * (size_t)nbmax * (P / 16) * kTile + sizeof(int) * (size_t)nbmax * nbmax;
    return (b + 15) & ~(size_t)15;
}

// HB (an arithmetic mode of the H kernels, kModeF64 + 1 .. kModeF16x3 + 1;
// 0: no H): the H blocks of the batch as well (batches b0 .. b1 - 1, one H
// slab), from the same orbital tiles, before phase A; the same operands and
// order as k_H_batch / k_H_batch16 (the same bits), written to part at block
// offset boff[b] - boff[b0] + k.
// T16 (the FP16 hi/lo mode; FP32 tiles, 32-point batches): T = S2 phi on
// FP16 matrix cores as well, from packed blocks in the 16-bit form
// (three products of FP16 hi/lo planes, FP32 accumulation).
// HONLY (FP32 H, HB = kModeF32 + 1): the H blocks alone (no packed D, no rho
// or force): the packed-row form of k_H_batch, with the same bits.
template <bool RHO, typename T, int P, int KU, int HB, bool T16 = HB == kModeF16x3 + 1, bool HONLY = false>
__global__ __launch_bounds__(64 * kForceWaves) void k_force_packed(Geo g, Bins bn, Basis bs, int nbmax,
                                                                  const T *__restrict__ pk,
                                                                  const double *__restrict__ W, double wscale,
                                                                  double *__restrict__ out, double *__restrict__ rho2,
                                                                  int b0, int b1, const int *__restrict__ boff,
                                                                  int mno, T *__restrict__ part)
{
    constexpr int NW = kForceWaves, NT = 64 * NW, NS = P / 16;
    extern __shared__ __align__(16) unsigned char s_dyn[];
    T *s_phi = reinterpret_cast<T *>(s_dyn);
    // after phi: the packed-fragment block of every slot pair (x, y), in
    // units of 256 elements: (pair * 16 + block) * 2 + orientation
    int *s_bb = reinterpret_cast<int *>(s_dyn + sizeof(T) * (size_t)nbmax * NS * kTile);
    __shared__ DevRadial s_rad[kMaxRadTotal];
    __shared__ DevSpecies s_sp[kMaxSpecies];
    __shared__ int s_atom[kMaxBatchAtoms], s_spc[kMaxBatchAtoms], s_off[kMaxBatchAtoms + 1];
    __shared__ int s_grank[kMaxBatchAtoms];
    __shared__ int s_ptab[kMaxBatchGroups * kMaxBatchGroups];
    // packed row -> (slot << 16) | (group rank << 8) | (atom % kGroup) << 4 | orbital, or -1
    __shared__ int s_row[kMaxBatchAtoms * kMaxOrb];
    __shared__ double s_red[RHO ? NW : 1][kMaxP];
    __shared__ double s_w[kMaxP];
    __shared__ double s_F[kMaxBatchAtoms][3];

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    constexpr int HMODE = HB - 1;  // arithmetic mode of the H blocks
    constexpr bool H16 = HB > kModeF32 + 1;
    static_assert(!T16 || (P == 32 && sizeof(T) == 4), "16-bit T: FP32 tiles of 32-point batches");
    static_assert(!HONLY || (HB && !H16 && !T16 && !RHO), "H alone: FP64 / FP32 H blocks");
    const int b = HB ? xcd_batch(blockIdx.x, b0, b1 - b0) : xcd_batch(blockIdx.x, 0, g.nbatch);
    if (b < 0)
        return;
    const int e0 = bn.bptr[b], nb = bn.bptr[b + 1] - e0;
    const int g0 = bn.bgptr[b], ngb = bn.bgptr[b + 1] - g0;
    int ib[3];
    batch_coords(g, b, ib);

    for (int k = tid; k < g.nrad; k += NT)
        s_rad[k] = bs.rad[k];
    for (int k = tid; k < g.nspecies; k += NT)
        s_sp[k] = bs.sp[k];
    for (int a = tid; a < nb; a += NT) {
        const int atom = bn.ent_atom[e0 + a];
        s_atom[a] = atom;
        s_spc[a] = bs.spc[atom];
        s_F[a][0] = s_F[a][1] = s_F[a][2] = 0.0;
    }
    if constexpr (!HONLY)
        for (int k = tid; k < ngb * ngb; k += NT) {
            const int ra = k / ngb, rb = k % ngb;
            const int ga = bn.bgrp[g0 + ra], gb = bn.bgrp[g0 + rb];
            s_ptab[k] = (ra <= rb) ? bn.pair_index[(size_t)ga * g.ngroup + gb] : -1;
        }
    for (int p = tid; p < P; p += NT) {
        int n[3];
        s_w[p] = batch_point(g, ib, p, n) ? wscale * W[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] : 0.0;
    }
    __syncthreads();
    // row offsets of the atoms (an inclusive scan of their orbital counts) and
    // their group ranks (atoms are increasing, so the rank of an atom's group
    // among the batch's groups counts the group changes before it); nb <= 64
    if (wave == 0) {
        int v = lane < nb ? s_sp[s_spc[lane]].norb : 0;
        int c = (lane > 0 && lane < nb && s_atom[lane] / kGroup != s_atom[lane - 1] / kGroup) ? 1 : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(v, o), tc = __shfl_up(c, o);
            if (lane >= o) {
                v += t;
                c += tc;
            }
        }
        if (lane < nb) {
            s_off[lane + 1] = v;
            s_grank[lane] = c;
        }
        if (lane == 0)
            s_off[0] = 0;
    }
    __syncthreads();
    if constexpr (!HONLY)
        for (int k = tid; k < nb * nb; k += NT) {
            const int x = k / nb, y = k % nb;
            const bool le = x <= y;
            const int lo = le ? x : y, hi = le ? y : x;
            const int pr = s_ptab[s_grank[lo] * ngb + s_grank[hi]];
            s_bb[k] = (pr * 16 + (s_atom[lo] % kGroup) * 4 + s_atom[hi] % kGroup) * 2 + (le ? 0 : 1);
        }
    const int nrow = s_off[nb];
    const int nrp = (nrow + 15) & ~15;  // packed rows incl. the padding of the last tile
    for (int r = tid; r < nrp; r += NT) {
        int code = -1;
        if (r < nrow) {
            int lo = 0, hi = nb;  // last a with off[a] <= r
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_off[mid] <= r)
                    lo = mid;
                else
                    hi = mid;
            }
            code = (lo << 16) | (s_grank[lo] << 8) | ((s_atom[lo] % kGroup) << 4) | (r - s_off[lo]);
        }
        s_row[r] = code;
    }

    // ---- stage the folded orbitals of every atom at every batch point ----
    for (int idx = tid; idx < nb * P; idx += NT) {
        const int a = idx / P, p = idx % P;
        const int e = e0 + a;
        const int atom = s_atom[a];
        // orbital o of this point at row[kPitch o]
        T *row = s_phi + (size_t)(a * NS + (p >> 4)) * kTile + (p & 15);
        int n[3];
        const bool valid = batch_point(g, ib, p, n);
        const DevSpecies &S = s_sp[s_spc[a]];
        const int zlo = valid ? S.norb : 0;
        for (int o = zlo; o < kMaxOrb; ++o)
            row[kPitch * o] = (T)0;
        if (valid) {
            const int io = bn.ent_img[e];
            const int cnt = bn.ent_img[e + 1] - io;
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            double r[3];
            mesh_cart(g, n, r);
            eval_orbitals<T, kPitch>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, cnt, bn.img[io], io,
                                     bn.img, r, row);
        }
    }
    __syncthreads();
    // tile s2 of atom slot x: element (orbital o, point q) at [kPitch o + q]
    auto tile = [&](int x, int s2) -> T * { return s_phi + (size_t)(x * NS + s2) * kTile; };

    if constexpr (H16) {
        // ---- 16-bit H (as k_H_batch16): per atom the hi (and lo) planes of
        // psi = sqrt|w| phi, then every block (ia <= ja) in contiguous ranges
        // over the waves, the sign of w a bit flip of the left operand ----
        constexpr bool F16 = HMODE == kModeF16 || HMODE == kModeF16x3;
        constexpr bool SPLIT = HMODE == kModeBF16x3 || HMODE == kModeF16x3;
        constexpr float kScale = F16 ? 256.0f : 1.0f;
        constexpr float kUnscale = 1.0f / (kScale * kScale);
        u4v *s_pl = reinterpret_cast<u4v *>(s_dyn + h16_plane_offset(sizeof(T), nbmax, P));  // [atom][hi, lo][lane]
        for (int a = wave; a < nb; a += NW) {
            const float *ta = reinterpret_cast<const float *>(tile(a, 0));
            unsigned hi[8], lo[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int p = 8 * lk + j;
                const float sw = (float)(sqrt(fabs(s_w[p])) * (double)kScale);
                split16<F16>(ta[(p >> 4) * kTile + kPitch * li + (p & 15)] * sw, hi[j], lo[j]);
            }
            u4v H, L;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                H[d] = hi[2 * d] | (hi[2 * d + 1] << 16);
                L[d] = lo[2 * d] | (lo[2 * d + 1] << 16);
            }
            s_pl[(2 * a) * 64 + lane] = H;
            s_pl[(2 * a + 1) * 64 + lane] = L;
        }
        u4v neg;
#pragma unroll
        for (int d = 0; d < 4; ++d)
            neg[d] = ((s_w[8 * lk + 2 * d] < 0.0 ? 1u : 0u) << 15) | ((s_w[8 * lk + 2 * d + 1] < 0.0 ? 1u : 0u) << 31);
        __syncthreads();
        const int nblk = nb * (nb + 1) / 2;
        const int k0 = wave * nblk / NW, k1 = (wave + 1) * nblk / NW;
        int ia = 0, ja = 0;
        tri_advance(ia, ja, k0, nb);
        const int mm = block_pitch(mno, sizeof(float));
        // this wave's block in LDS (row-major, pitch mno), streamed out as
        // one contiguous run of 16-byte stores
        float *s_hb = reinterpret_cast<float *>(s_dyn + h16_plane_offset(sizeof(T), nbmax, P) +
                                                2 * 64 * 16 * (size_t)nbmax) +
                      kMaxOrb * kMaxOrb * wave;
        // the left operands stay in registers while the blocks share atom ia
        int cur = -1, nI = 0;
        u4v aH = u4v{0u, 0u, 0u, 0u}, aL = aH;
        for (int k = k0; k < k1; ++k) {
            if (ia != cur) {
                aH = s_pl[(2 * ia) * 64 + lane] ^ neg;
                if (SPLIT)
                    aL = s_pl[(2 * ia + 1) * 64 + lane] ^ neg;
                nI = s_sp[s_spc[ia]].norb;
                cur = ia;
            }
            const u4v bH = s_pl[(2 * ja) * 64 + lane];
            f4 acc = f4{0.0f, 0.0f, 0.0f, 0.0f};
            acc = mma16<F16>(aH, bH, acc);
            if (SPLIT) {
                const u4v bL = s_pl[(2 * ja + 1) * 64 + lane];
                acc = mma16<F16>(aH, bL, acc);
                acc = mma16<F16>(aL, bH, acc);
            }
            const int nJ = s_sp[s_spc[ja]].norb;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 4 * lk + v;
                if (row < nI && li < nJ)
                    s_hb[row * mno + li] = acc[v] * kUnscale;
            }
            // (wave-level fences: the reads below see the writes above, and
            // the next block's writes follow them)
            wave_lds_sync();
            if (4 * lane < mm) {
                f4 *o = reinterpret_cast<f4 *>(part) + ((size_t)(boff[b] - boff[b0] + k) * mm >> 2);
                __builtin_nontemporal_store(*reinterpret_cast<const f4 *>(s_hb + 4 * lane), o + lane);
            }
            wave_lds_sync();
            if (++ja == nb) {
                ++ia;
                ja = ia;
            }
        }
    } else if constexpr (HB) {
        // ---- H over the packed rows: tile pairs (ti <= tj) of 16 packed
        // rows, in contiguous ranges over the waves.  Output element (packed
        // row r, packed column c) is element (ox, oy) of atom-pair block
        // (x, y); it is stored when x < y, or x == y and ox <= oy (the upper
        // triangle of a diagonal block, the part the reduction reads), at the
        // block's partial.  Each element is the same 32-point dot product as
        // in k_H_batch, accumulated in the same order. ----
        const int ntile = nrp >> 4;
        const int npr = ntile * (ntile + 1) / 2;
        const int k0 = wave * npr / NW, k1 = (wave + 1) * npr / NW;
        int ti = 0, tj = 0;
        tri_advance(ti, tj, k0, ntile);
        const int mm = block_pitch(mno, sizeof(T));
        T *pb = part + (size_t)(boff[b] - boff[b0]) * mm;  // this batch's block partials
        // this lane's points 4 kk + lk: weight, and the point's place in a tile row
        T wl[P / 4];
        int po[P / 4];
#pragma unroll
        for (int kk = 0; kk < P / 4; ++kk) {
            const int p = 4 * kk + lk;
            wl[kk] = (T)s_w[p];
            po[kk] = (p >> 4) * kTile + (p & 15);
        }
        // operand row li of tile t: phi of packed row 16 t + li.  Rows past
        // the last orbital read row (0, 0): the products of such rows and
        // columns are never stored, and no select waits for the loads
        auto oprow = [&](int t, T (&v8)[P / 4], bool weighted) {
            const int c = max(s_row[16 * t + li], 0);
            const T *pr = tile(c >> 16, 0) + kPitch * (c & 15);
#pragma unroll
            for (int kk = 0; kk < P / 4; ++kk) {
                const T f = pr[po[kk]];
                v8[kk] = weighted ? wl[kk] * f : f;
            }
        };
        int cur = -1;
        T aw[P / 4];
        // per output row of this lane: key 16 x + ox (larger than every
        // column key past the last orbital), partial offset
        int rkey[4], rb[4];
        for (int k = k0; k < k1; ++k) {
            if (ti != cur) {
                oprow(ti, aw, true);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = s_row[16 * ti + MM<T>::row(lk, v)];
                    const int x = c >> 16, ox = c & 15;
                    rkey[v] = c >= 0 ? 16 * x + ox : 0x7fffffff;
                    // block (x, y) is number x nb - x (x - 1) / 2 + (y - x) of the triangle
                    rb[v] = (x * nb - x * (x - 1) / 2 - x) * mm + ox * mno;
                }
                cur = ti;
            }
            T bv[P / 4];
            oprow(tj, bv, false);
            typename MM<T>::acc hc = MM<T>::zero();
#pragma unroll
            for (int kk = 0; kk < P / 4; ++kk)
                hc = MM<T>::mma(aw[kk], bv[kk], hc);
            const int cc = s_row[16 * tj + li];
            const int ckey = cc >= 0 ? 16 * (cc >> 16) + (cc & 15) : -1;
            const int cb = (cc >> 16) * mm + (cc & 15);
            // stored when both rows are orbitals (a padding column's key is
            // -1) and the element lies in the blocks' upper triangle
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (rkey[v] <= ckey)
                    store_partial(pb + rb[v] + cb, hc[v]);
            if (++tj == ntile) {
                ++ti;
                tj = ti;
            }
        }
    }
    if constexpr (HONLY)
        return;

    if constexpr (T16) {
        // phase A's right operands as FP16 hi/lo planes over the H planes
        // (every wave is past them): lane (j, k0) of point tile s2 of atom y
        // holds phi_y at point 16 s2 + j of slots k0 + 4 m, m = 0..3
        __syncthreads();
        u4v *s_tp = reinterpret_cast<u4v *>(s_dyn + h16_plane_offset(sizeof(T), nbmax, P));  // [atom][tile][lane]
        for (int k = tid; k < nb * NS * 64; k += NT) {
            const int ln = k & 63, y = k / (NS * 64), s2 = (k >> 6) % NS;
            const T *tp = tile(y, s2) + (ln & 15);
            const int k0 = ln >> 4;
            s_tp[k] = split4_f16(tp[kPitch * k0], tp[kPitch * (k0 + 4)], tp[kPitch * (k0 + 8)], tp[kPitch * (k0 + 12)]);
        }
        __syncthreads();
    }

    // ---- phase A ----
    const int ntile = nrp >> 4;
    double rp[NS];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2)
        rp[s2] = 0.0;
    typename MM<T>::acc acc[KU][NS];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2)
            acc[u][s2] = MM<T>::zero();
        const int ti = wave + NW * u;
        if (ti >= ntile)
            continue;
        // this lane's output row (x, ox): A[i][k] = S2[row 16 ti + i][(y, 4 j + k)]
        const int rc = s_row[16 * ti + li];
        const bool rok = rc >= 0;
        const int x = rok ? rc >> 16 : 0, ox = rok ? rc & 15 : 0;
        // the A values of atom y: S2[(x, ox)][(y, 4 j + lk)] sits in the packed
        // block of the slot-ordered pair (orientation 0 when x <= y) at
        // 16 (4 j + lk) + ox
        auto load = [&](T (&a4)[4], int y) {
            const T *f = pk + (size_t)s_bb[x * nb + y] * 256 + 16 * lk + ox;
            // (rows past the last orbital read the finite values of row
            // (0, 0): their T is discarded; no select here, which would wait
            // for the loads where they are issued)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                a4[j] = f[64 * j];
        };
        auto mblock = [&](const T (&a4)[4], int y) {
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                const T *pB = tile(y, s2) + kPitch * lk + li;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[u][s2] = MM<T>::mma(a4[j], pB[4 * kPitch * j], acc[u][s2]);
            }
        };
        // three register sets in rotation: an atom's D values are loaded two
        // atoms ahead of their use (past the end, the last atom is reloaded)
        auto at = [&](int y) { return y < nb ? y : nb - 1; };
        if constexpr (T16) {
            // the 16-byte hi/lo form of the same packed values (lane
            // 16 lk + ox of the block), right operands from the planes; K
            // order k0 + 4 m on both operands
            const u4v *pk16 = reinterpret_cast<const u4v *>(pk);
            const u4v *s_tp = reinterpret_cast<const u4v *>(s_dyn + h16_plane_offset(sizeof(T), nbmax, P));
            auto load16 = [&](u4v &a, int y) { a = pk16[(size_t)s_bb[x * nb + y] * 64 + 16 * lk + ox]; };
            auto mblock16 = [&](const u4v &a, int y) {
                const u2v aH = u2v{a.x, a.y}, aL = u2v{a.z, a.w};
#pragma unroll
                for (int s2 = 0; s2 < NS; ++s2) {
                    const u4v b = s_tp[(y * NS + s2) * 64 + lane];
                    const u2v bH = u2v{b.x, b.y}, bL = u2v{b.z, b.w};
                    acc[u][s2] = mma16k16(aH, bH, acc[u][s2]);
                    acc[u][s2] = mma16k16(aH, bL, acc[u][s2]);
                    acc[u][s2] = mma16k16(aL, bH, acc[u][s2]);
                }
            };
            u4v fa, fb, fc;
            load16(fa, 0);
            load16(fb, at(1));
            int ja = 0;
            for (; ja + 2 < nb; ja += 3) {
                load16(fc, ja + 2);
                mblock16(fa, ja);
                load16(fa, at(ja + 3));
                mblock16(fb, ja + 1);
                load16(fb, at(ja + 4));
                mblock16(fc, ja + 2);
            }
            if (ja < nb)
                mblock16(fa, ja);
            if (ja + 1 < nb)
                mblock16(fb, ja + 1);
            // both operands carried a 2^8 scale
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2)
                acc[u][s2] *= 1.0f / 65536.0f;
        } else {
            T fa[4], fb[4], fc[4];
            load(fa, 0);
            load(fb, at(1));
            int ja = 0;
            for (; ja + 2 < nb; ja += 3) {
                load(fc, ja + 2);
                mblock(fa, ja);
                load(fa, at(ja + 3));
                mblock(fb, ja + 1);
                load(fb, at(ja + 4));
                mblock(fc, ja + 2);
            }
            if (ja < nb)
                mblock(fa, ja);
            if (ja + 1 < nb)
                mblock(fb, ja + 1);
        }
        if (RHO) {
            // phi at the output rows of this lane (zero for padding rows)
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                double dot = 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = s_row[16 * ti + MM<T>::row(lk, v)];
                    const T ph = c >= 0 ? tile(c >> 16, s2)[kPitch * (c & 15) + li] : (T)0;
                    dot += (double)acc[u][s2][v] * (double)ph;
                }
                rp[s2] += dot;
            }
        }
    }
    if (RHO) {
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) {
            double v = rp[s2];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lane < 16)
                s_red[wave][16 * s2 + lane] = v;
        }
    }
    __syncthreads();  // every wave is done with Phi
#pragma unroll
    for (int u = 0; u < KU; ++u) {
        const int ti = wave + NW * u;
        if (ti >= ntile)
            continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = s_row[16 * ti + MM<T>::row(lk, v)];
            if (c >= 0)
#pragma unroll
                for (int s2 = 0; s2 < NS; ++s2)
                    tile(c >> 16, s2)[kPitch * (c & 15) + li] = acc[u][s2][v];
        }
    }
    __syncthreads();

    // ---- phase B: dE/dR_I partial = -sum_p w_p grad phi_I(p) . T_I(p) ----
    // item (atom a, point p) = a P + p: the P items of an atom are P
    // consecutive lanes of one wave (P divides 64)
    for (int base = wave * 64; base < nb * P; base += NT) {
        const int idx = base + lane;
        const int a = idx / P, p = idx % P;
        double fx[3] = {0.0, 0.0, 0.0};
        int n[3];
        if (idx < nb * P && batch_point(g, ib, p, n)) {
            const int e = e0 + a;
            const int atom = s_atom[a];
            const DevSpecies &S = s_sp[s_spc[a]];
            const double X[3] = {bs.xw[3 * atom], bs.xw[3 * atom + 1], bs.xw[3 * atom + 2]};
            const int io = bn.ent_img[e];
            const int cnt = bn.ent_img[e + 1] - io;
            double r[3];
            mesh_cart(g, n, r);
            grad_dot_all<T, kPitch>(g, s_rad, S.rad0, S.rad0 + S.nrad, S.rc, bs.coef, X, cnt, bn.img[io], io,
                                    bn.img, r, tile(a, p >> 4) + (p & 15), s_w[p], fx);
        }
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            double v = fx[x];
#pragma unroll
            for (int o = P / 2; o > 0; o >>= 1)
                v += __shfl_xor(v, o);
            fx[x] = v;
        }
        if (idx < nb * P && p == 0) {
            s_F[a][0] = -fx[0];
            s_F[a][1] = -fx[1];
            s_F[a][2] = -fx[2];
        }
    }
    __syncthreads();
    for (int k = tid; k < nb * 3; k += NT)
        out[(size_t)(e0 + k / 3) * 3 + k % 3] = s_F[k / 3][k % 3];
    if (RHO)
        for (int p = tid; p < P; p += NT) {
            int n[3];
            if (batch_point(g, ib, p, n)) {
                double v = s_red[0][p];
                for (int w = 1; w < NW; ++w)
                    v += s_red[w][p];
                rho2[(n[0] * g.N[1] + n[1]) * g.N[2] + n[2]] = 0.5 * v;
            }
        }
}

template <bool RHO, typename T, int P, int KU, int HB = 0, bool T16 = HB == kModeF16x3 + 1, bool HONLY = false>
static hipError_t launch_packed_k(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                                  size_t lds, const void *pk, const double *W, double wscale, double *out,
                                  double *rho2, int b0 = 0, int b1 = 0, const int *boff = nullptr, int mno = 0,
                                  void *part = nullptr)
{
    hipError_t e = hipFuncSetAttribute((const void *)k_force_packed<RHO, T, P, KU, HB, T16, HONLY>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    const int nbat = HB ? b1 - b0 : g.nbatch;
    hipLaunchKernelGGL((k_force_packed<RHO, T, P, KU, HB, T16, HONLY>), dim3(xcd_grid(nbat)), dim3(64 * kForceWaves), lds, s,
                       g, bn, b, nbmax, static_cast<const T *>(pk), W, wscale, out, rho2, b0, b1, boff, mno,
                       static_cast<T *>(part));
    return hipGetLastError();
}

// the packed form while every wave holds at most 3 row tiles (otherwise the
// per-atom form, whose registers do not grow with the atom count)
template <bool RHO, typename T, int P>
static hipError_t launch_force_p(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int mno,
                                 const void *pk, const double *W, double wscale, double *out, double *rho2)
{
    const int rows = (nbmax * mno + 15) & ~15;
    const int ku = (rows / 16 + kForceWaves - 1) / kForceWaves;
    const size_t lds = sizeof(T) * (size_t)nbmax * (P / 16) * kTile + sizeof(int) * (size_t)nbmax * nbmax;
    if (lds + 20480 > 163840)  // with the kernel's static LDS
        return launch_batch_p<RHO ? kRhoForce : kForce, T, P>(s, g, bn, b, nbmax, pk, W, wscale, out, rho2);
    switch (ku) {
    case 0:
    case 1: return launch_packed_k<RHO, T, P, 1>(s, g, bn, b, nbmax, lds, pk, W, wscale, out, rho2);
    case 2: return launch_packed_k<RHO, T, P, 2>(s, g, bn, b, nbmax, lds, pk, W, wscale, out, rho2);
    case 3: return launch_packed_k<RHO, T, P, 3>(s, g, bn, b, nbmax, lds, pk, W, wscale, out, rho2);
    default: return launch_batch_p<RHO ? kRhoForce : kForce, T, P>(s, g, bn, b, nbmax, pk, W, wscale, out, rho2);
    }
}

template <bool RHO, typename T>
static hipError_t launch_force_t(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int mno,
                                 const void *pk, const double *W, double wscale, double *out, double *rho2)
{
    if (g.P == 32)
        return launch_force_p<RHO, T, 32>(s, g, bn, b, nbmax, mno, pk, W, wscale, out, rho2);
    if (g.P == 16)
        return launch_force_p<RHO, T, 16>(s, g, bn, b, nbmax, mno, pk, W, wscale, out, rho2);
    return hipErrorInvalidValue;
}

hipError_t launch_rho_batch(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                            const void *pk, double *rho)
{
    return f32 ? launch_batch_t<kRho, float>(s, g, bn, b, nbmax, pk, nullptr, 0.0, rho, nullptr)
               : launch_batch_t<kRho, double>(s, g, bn, b, nbmax, pk, nullptr, 0.0, rho, nullptr);
}

// the fused pass's LDS and row tiles per wave for this plan and H mode, or 0
// if it does not apply (16-bit H: 32-point batches, FP32 tiles)
template <typename T, int P>
static int packed_ku(int nbmax, int mno, int mode, size_t *lds)
{
    const int rows = (nbmax * mno + 15) & ~15;
    const int ku = (rows / 16 + kForceWaves - 1) / kForceWaves;
    *lds = sizeof(T) * (size_t)nbmax * (P / 16) * kTile + sizeof(int) * (size_t)nbmax * nbmax;
    if (mode > kModeF32) {
        if (P != 32)
            return 0;
        // the hi/lo planes (later phase A's), then one block per wave
        *lds = h16_plane_offset(sizeof(T), nbmax, P) + 2 * 64 * 16 * (size_t)nbmax +
               sizeof(float) * kMaxOrb * kMaxOrb * kForceWaves;
    }
    return (*lds + 24576 > 163840 || ku > 3) ? 0 : (ku < 1 ? 1 : ku);
}

template <typename T, int P, int HB>
static hipError_t launch_hrf_m(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int mno,
                               const void *pk, const double *W, double wscale, double *Fent, double *rho, int b0,
                               int b1, const int *boff, void *part)
{
    size_t lds = 0;
    switch (packed_ku<T, P>(nbmax, mno, HB - 1, &lds)) {
    case 1: return launch_packed_k<true, T, P, 1, HB>(s, g, bn, b, nbmax, lds, pk, W, wscale, Fent, rho, b0, b1, boff, mno, part);
    case 2: return launch_packed_k<true, T, P, 2, HB>(s, g, bn, b, nbmax, lds, pk, W, wscale, Fent, rho, b0, b1, boff, mno, part);
    case 3: return launch_packed_k<true, T, P, 3, HB>(s, g, bn, b, nbmax, lds, pk, W, wscale, Fent, rho, b0, b1, boff, mno, part);
    default: return hipErrorNotSupported;
    }
}

bool H_rho_force_fits(int mode, int P, int nbmax, int mno)
{
    size_t lds = 0;
    if (P != 32 && P != 16)
        return false;
    if (mode != kModeF64)
        return (P == 32 ? packed_ku<float, 32>(nbmax, mno, mode, &lds) : packed_ku<float, 16>(nbmax, mno, mode, &lds)) > 0;
    return (P == 32 ? packed_ku<double, 32>(nbmax, mno, mode, &lds) : packed_ku<double, 16>(nbmax, mno, mode, &lds)) > 0;
}

hipError_t launch_H_rho_force(hipStream_t s, int mode, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                              int mno, const void *pk, const double *W, double wscale, double *Fent, double *rho,
                              int b0, int b1, const int *boff, void *part)
{
    if (b1 <= b0)
        return hipSuccess;
#define GINT_HRF(T, P, HB) launch_hrf_m<T, P, HB>(s, g, bn, b, nbmax, mno, pk, W, wscale, Fent, rho, b0, b1, boff, part)
    if (g.P == 32) {
        switch (mode) {
        case kModeF64: return GINT_HRF(double, 32, kModeF64 + 1);
        case kModeF32: return GINT_HRF(float, 32, kModeF32 + 1);
        case kModeBF16: return GINT_HRF(float, 32, kModeBF16 + 1);
        case kModeF16: return GINT_HRF(float, 32, kModeF16 + 1);
        case kModeBF16x3: return GINT_HRF(float, 32, kModeBF16x3 + 1);
        case kModeF16x3: return GINT_HRF(float, 32, kModeF16x3 + 1);
        default: return hipErrorInvalidValue;
        }
    }
    if (g.P == 16) {
        switch (mode) {
        case kModeF64: return GINT_HRF(double, 16, kModeF64 + 1);
        case kModeF32: return GINT_HRF(float, 16, kModeF32 + 1);
        default: return hipErrorNotSupported;
        }
    }
#undef GINT_HRF
    return hipErrorNotSupported;
}

// H alone through the fused kernel's packed-row H loop: its tiles and the
// slot-pair table in LDS; hipErrorNotSupported (nothing launched) where they
// do not fit
template <typename T, int P, int HB>
static hipError_t launch_H_packed_t(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int b0,
                                    int b1, const double *W, double wscale, const int *boff, int mno, void *part)
{
    const size_t lds = sizeof(T) * (size_t)nbmax * (P / 16) * kTile + sizeof(int) * (size_t)nbmax * nbmax;
    if (nbmax > kMaxBatchAtoms || lds + 24576 > 163840)
        return hipErrorNotSupported;
    return launch_packed_k<false, T, P, 1, HB, false, true>(s, g, bn, b, nbmax, lds, nullptr, W, wscale, nullptr,
                                                            nullptr, b0, b1, boff, mno, part);
}

static hipError_t launch_H_packed(hipStream_t s, int mode, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                                  int b0, int b1, const double *W, double wscale, const int *boff, int mno,
                                  void *part)
{
    if (mode == kModeF32)
        return g.P == 32   ? launch_H_packed_t<float, 32, kModeF32 + 1>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff,
                                                                        mno, part)
               : g.P == 16 ? launch_H_packed_t<float, 16, kModeF32 + 1>(s, g, bn, b, nbmax, b0, b1, W, wscale, boff,
                                                                        mno, part)
                           : hipErrorNotSupported;
    return hipErrorNotSupported;
}

bool force_h16_fits(int P, int nbmax, int mno)
{
    size_t lds = 0;
    return P == 32 && packed_ku<float, 32>(nbmax, mno, kModeF16x3, &lds) > 0;
}

// the packed form with the 16-bit T (no H: the H planes' LDS holds the T planes)
template <bool RHO>
static hipError_t launch_force_h16(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int mno,
                                   const void *pk, const double *W, double wscale, double *out, double *rho2)
{
    size_t lds = 0;
    if (g.P != 32)
        return hipErrorNotSupported;
    switch (packed_ku<float, 32>(nbmax, mno, kModeF16x3, &lds)) {
    case 1: return launch_packed_k<RHO, float, 32, 1, 0, true>(s, g, bn, b, nbmax, lds, pk, W, wscale, out, rho2);
    case 2: return launch_packed_k<RHO, float, 32, 2, 0, true>(s, g, bn, b, nbmax, lds, pk, W, wscale, out, rho2);
    case 3: return launch_packed_k<RHO, float, 32, 3, 0, true>(s, g, bn, b, nbmax, lds, pk, W, wscale, out, rho2);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_force_batch(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                              int mno, const void *pk, const double *W, double wscale, double *Fent, double *rho,
                              bool h16)
{
    if (h16)
        return rho ? launch_force_h16<true>(s, g, bn, b, nbmax, mno, pk, W, wscale, Fent, rho)
                   : launch_force_h16<false>(s, g, bn, b, nbmax, mno, pk, W, wscale, Fent, nullptr);
    if (rho)
        return f32 ? launch_force_t<true, float>(s, g, bn, b, nbmax, mno, pk, W, wscale, Fent, rho)
                   : launch_force_t<true, double>(s, g, bn, b, nbmax, mno, pk, W, wscale, Fent, rho);
    return f32 ? launch_force_t<false, float>(s, g, bn, b, nbmax, mno, pk, W, wscale, Fent, nullptr)
               : launch_force_t<false, double>(s, g, bn, b, nbmax, mno, pk, W, wscale, Fent, nullptr);
}

// dE/dR per atom: fixed-order sum of its per-(batch, atom) partials over the
// batches of its group's list.
__global__ __launch_bounds__(256) void k_force_reduce(const int *__restrict__ aptr, const int *__restrict__ aent,
                                                      const int *__restrict__ perm, const double *__restrict__ Fent,
                                                      double *__restrict__ dEdR)
{
    __shared__ double red[3][256];
    const int ii = blockIdx.x;
    // the atom's entries in batch order (its list of the pair-block build)
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = aptr[ii] + threadIdx.x; k < aptr[ii + 1]; k += 256) {
        const int e = aent[k];
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
        dEdR[3 * perm[ii] + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_force_reduce(hipStream_t s, int natom, const int *aptr, const int *aent, const int *perm,
                               const double *Fent, double *dEdR)
{
    if (natom <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_force_reduce, dim3(natom), dim3(256), 0, s, aptr, aent, perm, Fent, dEdR);
    return hipGetLastError();
}

}  // namespace gint
