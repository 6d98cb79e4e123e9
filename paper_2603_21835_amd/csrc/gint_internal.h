// gint_internal.h -- device-side views and launchers shared by the host API
// (gint_api.hip) and the kernels (gint_kernels.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gint {

constexpr int kMaxOrb = 16;       // orbital slots per atom (l <= 2)
constexpr int kMaxRad = 16;       // radials per species
constexpr int kGroup = 4;         // atoms per group (output tile = 4x4 atom blocks)
constexpr int kMaxP = 32;         // mesh points per batch
constexpr int kMaxAtoms = 16384;
constexpr int kMaxRadTotal = 64;  // radials over all species (staged in LDS)
constexpr int kMaxSpecies = 16;
constexpr int kMaxBatchAtoms = 64;   // atoms reaching one mesh batch
constexpr int kMaxBatchGroups = 32;  // atom groups reaching one mesh batch
constexpr int kXcd = 8;           // XCDs: workgroup i runs on XCD i % kXcd
constexpr int kRow = 16;          // elements per staged (slot, point) row in LDS (H kernels)
constexpr double kRTiny = 1e-12;  // |d| below this: the atom's own position

// Mesh, lattice and batch shape.  Batches tile the mesh with bs[0] x bs[1] x
// bs[2] points (n3 fastest inside a batch); edge batches are partial.
struct Geo {
    double lat[9];  // rows a1, a2, a3
    double rec[9];  // rows b_i, a_i . b_j = delta_ij
    double h[9];    // mesh steps: rows a_i / N_i
    int N[3];
    int bs[3];
    int nb[3];
    int bt[3];   // batches per tile along each axis (divides nb): batch ids run tile by tile
    int P;       // bs[0]*bs[1]*bs[2]
    int nbatch;  // nb[0]*nb[1]*nb[2]
    int ortho;   // lattice rows are along the cartesian axes
    int natom;
    int ngroup;  // ceil(natom / kGroup)
    int nrad;    // radials over all species
    int nspecies;
};

struct DevRadial {
    double dr, inv_dr, rc;
    int l, nr, orb0;  // orb0: first orbital slot of this radial inside the atom
    int coef_off;     // offset (doubles) of the (nr-1) x 4 coefficient table
    int knot_off;     // offset (doubles) of the knot values
};

struct DevSpecies {
    int rad0, nrad, norb;
    double rc;                   // largest cutoff of the species
    signed char orb_rad[kMaxOrb];  // radial (global index) owning each orbital
    signed char orb_m[kMaxOrb];    // m of each orbital
};

// Binning lists (all device pointers).
struct Bins {
    const int *bptr;        // nbatch+1: entries of each batch
    const int *ent_atom;    // internal atom id, increasing within a batch
    const int *ent_img;     // nent+1: image offsets of each entry
    const int *img;         // packed signed 8-bit lattice multiples (n1, n2, n3)
    const int *bgptr;       // nbatch+1: distinct groups of each batch
    const int *bgrp;        // group ids, increasing within a batch
    const int *gptr;        // ngroup+1: batches of each group
    const int *gbatch;      // batch ids, increasing within a group
    const int *pairA;       // npair
    const int *pairB;       // npair
    const int *pair_index;  // ngroup*ngroup -> pair id or -1 (A <= B)
};

// Per-atom lists for the point-stationary H path.
// Caller's list of lattice vectors for the H(R) blocks: rmap over the box
// |n_k| <= ext[k] gives the list index of R = (n1, n2, n3), or -1.
struct HRMap {
    const int *rmap;
    int ext[3];
};
constexpr int kHRBox = 31;  // |n_k| of the lattice vectors of the H(R) blocks

struct AtomLists {
    const int *aptr;   // natom+1: entries of each atom
    const int *aent;   // entry indices, increasing (= increasing batch)
    const int *abat;   // batch of each of those entries
    const int *pptr;   // natom+1: partners of each atom
    const int *plist;  // owned partner atoms, increasing
};

struct Basis {
    const DevRadial *rad;
    const DevSpecies *sp;
    const double *coef;
    const int *spc;      // species of each internal atom
    const double *xw;    // wrapped cartesian position of each internal atom
    const int *perm;     // internal -> input atom
    const int *inv_perm; // input -> internal atom
    const int *orb0;     // input atom -> first orbital (natom+1)
    const int *orb_atom; // orbital -> input atom
};

// ---- launchers (gint_kernels.hip); each returns hipGetLastError() ----
hipError_t launch_spline(hipStream_t s, int nrad, const DevRadial *rad, const double *knots,
                         const double *s0, const double *sn, double *coef, double *scratch);
hipError_t launch_wrap(hipStream_t s, const Geo &g, const double *pos_in, double *xw_in,
                       unsigned long long *keys);
hipError_t launch_sort_perm(hipStream_t s, int natom, unsigned long long *keys, int *perm,
                            int *inv_perm);
hipError_t launch_gather_internal(hipStream_t s, int natom, const int *perm, const double *xw_in,
                                  const int *spc_in, double *xw, int *spc);
hipError_t launch_bin_count(hipStream_t s, const Geo &g, const Basis &b, int *cnt_e, int *cnt_i,
                            int *cnt_g);
hipError_t launch_bin_fill(hipStream_t s, const Geo &g, const Basis &b, const int *bptr,
                           const int *iptr, const int *bgptr, int *ent_atom, int *ent_img, int *img,
                           int *bgrp);
// exclusive scan (out: n + 1 ints, out[n] = total); tmp: scan_tmp_ints(n) ints
int scan_tmp_ints(long long n);
hipError_t launch_scan_i32(hipStream_t s, const int *in, long long n, int *out, int *tmp);
int group_chunks(const Geo &g);  // chunks of the per-group batch list construction
hipError_t launch_group_count(hipStream_t s, const Geo &g, const int *bgptr, const int *bgrp,
                              int *cnt /* ngroup * group_chunks */);
hipError_t launch_group_fill(hipStream_t s, const Geo &g, const int *bgptr, const int *bgrp, const int *off,
                             int *gbatch, int *gptr);
hipError_t launch_fill_i32(hipStream_t s, int *p, long long n, int v);
hipError_t launch_pair_mark(hipStream_t s, const Geo &g, const int *bgptr, const int *bgrp,
                            int *mark);
hipError_t launch_pair_list(hipStream_t s, int ngroup, const int *mark, const int *mark_scan,
                            int *pair_index, int *pairA, int *pairB);
hipError_t launch_support_count(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b,
                                double *sums /* 2 per block */, int nblocks);

// Contractions (gint_contract.hip).
// f32 selects FP32 orbital tiles, packed D and H partials (else FP64).
// Elements between consecutive H block partials: mno * mno rounded up to
// whole 128-byte lines, so that every block starts on a line of its own and
// its stores and loads never share a line with a neighbouring block.
__host__ __device__ inline int block_pitch(int mno, int esz)
{
    const int v = 128 / esz;
    return (mno * mno + v - 1) / v * v;
}
// arithmetic modes of the H kernel (values of gint_precision)
constexpr int kModeF64 = 0, kModeF32 = 1, kModeBF16 = 2, kModeF16 = 3, kModeBF16x3 = 4, kModeF16x3 = 5;
// H(R) blocks (gint_hr.hip): per-image atom and wrap-shift tables, then the
// per-batch kernel adding into HR[nR][norb][norb]
hipError_t launch_HR_prep(hipStream_t s, const Geo &g, long long nent, const int *ent_atom, const int *ent_img,
                          int *img_atom, const int *perm, const double *pos_in, const double *xw, int *wsh);
hipError_t launch_iota(hipStream_t s, long long n, int *a);
hipError_t launch_HR_keys(hipStream_t s, int nbatch, const int *iptr, const int *boff, const int *img_atom,
                          const int *img, const int *perm, const int *wsh, int natom, unsigned long long *key,
                          int *code, int *bad);
hipError_t launch_seg(hipStream_t s, long long n, const unsigned long long *key, int *flag, int *fscan, int *tstart,
                      unsigned long long *tkey, bool fill);
hipError_t sort_HR_keys(hipStream_t s, void *tmp, size_t &tmp_bytes, const unsigned long long *key_in,
                        unsigned long long *key_out, const int *code_in, int *code_out, int n, int end_bit);
// fixed-order sums of the H(R) block partials, one wave per canonical triple
hipError_t launch_HR_reduce(hipStream_t s, bool f32, int ntri, const int *order, const unsigned long long *tkey,
                            const int *tstart, const int *list, int natom, const HRMap &m, const Basis &b, int mno,
                            int norb, const void *part, double *HR);
// D(R) blocks of the rho and force contractions packed per canonical (I, J, R)
// triple: etri[entry] = 2 t + o for every unfolded block entry (batch b's
// entries from boff[b], image pairs a <= c in row-major order), nz[t] = 0
// where neither R nor -R is listed, spk[2 t + o] = 16 x 16 doubles of S_IJ(R)
// = D_IJ(R) + D_JI(-R)^T (o = 0) or its transpose (o = 1) in MFMA A-operand
// lane order
struct PackedS {
    const int *etri;
    const int *boff;
    const int *nz;
    const double *spk;
};
hipError_t launch_entry_tri(hipStream_t s, long long n, const int *code, const int *fscan, int *etri);
hipError_t launch_S_pack(hipStream_t s, int ntri, const unsigned long long *tkey, int natom, const int *orb0,
                         const HRMap &m, int norb, const double *DR, double *spk, int *nz);
// ps == nullptr: each lane gathers its D(R) elements instead
hipError_t launch_rhoR_batch(hipStream_t s, bool f32, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                             const int *img, const Basis &b, const int *wsh, const HRMap &m, int norb,
                             const double *DR, const PackedS *ps, double *rho);
hipError_t launch_Hk(hipStream_t s, long long nel, int nR, int nk, const double *ph, const double *HR, double *Hk);
// spherical-grid projector overlaps (gint_sphere.hip)
hipError_t launch_pb_images(hipStream_t s, const Geo &g, const Basis &b, int npa, const int *pint, const double *prb,
                            const int *m, int *cnt, const int *off, int *img);
hipError_t launch_psibeta(hipStream_t s, const Geo &g, const Basis &b, const DevRadial *prad, const DevSpecies *psp,
                          const double *pcoef, int nprad, int npa, const int *pint, const int *pin, const int *prow,
                          const int4 *ent, int nent, const int *img, const double *pos, int nang, const double *ang,
                          int nrq, const double *rq, const double *A, int nps, void *tab, int norb, double *Q);
// moving-basis matrix DK (gint_dphi.hip): one workgroup per owned atom pair
// over the pair's block list; DK must be zero beforehand
size_t DK_pairs_lds(int P);
hipError_t launch_DK_desc(hipStream_t s, long long n, int nbatch, const int *list, const int *boff, const int *bptr,
                          int4 *desc);
hipError_t launch_DK_pairs(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, const double *W, double wscale,
                           int npair, const int *order, const int *pown, const int *plist, const int *lptr,
                           const int4 *desc, int norb, double *DK);
// limits of the allocation-free H(k) (its workspace is a fixed device array)
constexpr int kHkNaMaxPhase = 65536, kHkNaMaxK = 8192, kHkNaMaxR = 8192;
// H(k) with the phases and staged inputs in the device array of gint_hr.hip
// (no device allocation; synchronises s once after staging R and kfrac);
// hipErrorInvalidValue beyond the limits above
hipError_t Hk_noalloc(hipStream_t s, int device, long long nel, int nR, const int *R, int nk, const double *kfrac,
                      const double *HR, double *Hk);
hipError_t launch_forceR_batch(hipStream_t s, bool f32, const Geo &g, int nbmax, const int *iptr,
                               const int *img_atom, const int *img, const Basis &b, const int *wsh, const HRMap &m,
                               int norb, const double *DR, const PackedS *ps, const double *W, double wscale,
                               double *Fimg);
hipError_t launch_forceR_reduce(hipStream_t s, int natom, const int *aptr, const int *aent, const int *ent_img,
                                const int *perm, const double *Fimg, double *dEdR);
hipError_t launch_HR_mark(hipStream_t s, const Geo &g, const int *iptr, const int *img_atom, const int *img,
                          const int *wsh, int M, int *mark);
hipError_t launch_HR_batch(hipStream_t s, bool f32, const Geo &g, int nbmax, const int *iptr, const int *img_atom,
                           const int *img, const Basis &b, const int *wsh, const double *W, double wscale,
                           const HRMap &m, int norb, double *HR);
hipError_t launch_H_batch(hipStream_t s, int mode, const Geo &g, const Bins &bn, const Basis &b, int nbmax, int b0,
                          int b1, const double *W, double wscale, const int *boff, int mno, void *part);
// H block partials of slab si summed per owned pair (I = pown[p], J = plist[p])
// over its list entries lsl[p (nslab + 1) + si] .. lsl[... + si + 1]; pairs
// launched in the order order[] (nullptr: index order)
hipError_t launch_H_pairreduce(hipStream_t s, bool f32, int npair, const int *order, const int *pown,
                               const int *plist, const int *lsl, int nslab, int si, const int *list, const Basis &b,
                               int mno, int norb, const void *part, int q0, int accumulate, double *H);
// the smaller entry count of each owned pair's two atoms (a bound on its
// block list), and the compaction of lists written at those bounds' offsets
hipError_t launch_pair_ub(hipStream_t s, int natom, int npair, const int *aptr, const int *pptr, const int *plist,
                          int *ub);
hipError_t launch_list_compact(hipStream_t s, int npair, const int *uptr, const int *lptr, const int *cnt,
                               const int *src, int *dst);
hipError_t launch_pair_blocks(hipStream_t s, int natom, int npair, const int *aptr, const int *aent,
                              const int *abat, const int *bptr, const int *boff, const int *pptr, const int *plist,
                              int *lcnt, const int *lptr, int *list);
// items (owned pairs, H(R) triples) sorted by the length of their list
// range ptr[i stride] .. ptr[i stride + span], heaviest first (stable), into
// order[n]; tmp == nullptr: tmp_bytes receives the scratch size
hipError_t launch_item_order(hipStream_t s, void *tmp, size_t &tmp_bytes, int n, int stride, int span, const int *ptr,
                             int *cost, int *cost2, int *idx, int *order);
hipError_t launch_pair_slabs(hipStream_t s, int natom, int npair, const int *pptr, const int *lptr, const int *list,
                             int nslab, const int *slab_q, int *pown, int *lsl);
hipError_t launch_fill_f64(hipStream_t s, double *p, long long n, double v);
hipError_t launch_block_count(hipStream_t s, int nbatch, const int *bptr, int *cnt);
hipError_t launch_atom_count(hipStream_t s, int natom, const int *gptr, const int *gbatch, const int *bptr,
                             const int *ent_atom, int *acnt);
hipError_t launch_atom_fill(hipStream_t s, int natom, const int *gptr, const int *gbatch, const int *bptr,
                            const int *ent_atom, const int *aptr, int *aent, int *abat);
hipError_t launch_partners(hipStream_t s, const Geo &g, const Basis &b, double brad, const int *pptr,
                           int *pcnt, int *plist);
hipError_t launch_pack_S2(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int npair,
                          const double *D, int norb, void *pk);
// the same fragments as FP16 hi/lo planes (each value scaled by 2^8): per
// block and orientation 64 lanes of 16 bytes, lane (i, k0) holding (i, k0 + 4 m)
hipError_t launch_pack_S2_h16(hipStream_t s, const Geo &g, const Bins &bn, const Basis &b, int npair,
                              const double *D, int norb, void *pk);
size_t batch_lds_bytes(int nbmax, int P, bool f32);
hipError_t launch_rho_batch(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                            const void *pk, double *rho);
// h16: T on FP16 hi/lo matrix cores from the 16-bit packed form
// (launch_pack_S2_h16), possible where force_h16_fits says so
bool force_h16_fits(int P, int nbmax, int mno);
hipError_t launch_force_batch(hipStream_t s, bool f32, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                              int mno, const void *pk, const double *W, double wscale, double *Fent,
                              double *rho /* NULL, or rho as well */, bool h16 = false);
// H blocks of batches b0 .. b1 - 1 (into part, as launch_H_batch) together
// with rho and the force partials of the same batches, from one evaluation of
// the orbital tiles (mode: the H arithmetic, kModeF64 .. kModeF16x3);
// H_rho_force_fits says whether the plan's batches fit the fused pass
bool H_rho_force_fits(int mode, int P, int nbmax, int mno);
hipError_t launch_H_rho_force(hipStream_t s, int mode, const Geo &g, const Bins &bn, const Basis &b, int nbmax,
                              int mno, const void *pk, const double *W, double wscale, double *Fent, double *rho,
                              int b0, int b1, const int *boff, void *part);
// dE/dR of every atom: its entry partials Fent summed in batch order (its
// atom list aptr / aent), written at the atom's input index
hipError_t launch_force_reduce(hipStream_t s, int natom, const int *aptr, const int *aent, const int *perm,
                               const double *Fent, double *dEdR);
hipError_t launch_max_i32(hipStream_t s, const int *a, long long n, int *out);

}  // namespace gint
