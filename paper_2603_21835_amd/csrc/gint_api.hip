// gint_api.hip -- host side of the C ABI declared in include/gint.h:
// argument validation, the plan (GintInfo role: geometry, basis tables and
// the batch/atom lists), and dispatch of the kernels in gint_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/gint.h"
#include "gint_internal.h"

using namespace gint;

namespace {

constexpr unsigned kMagic = 0x47494e54u;  // "GINT"
thread_local std::string g_last_error;
// failure injection for tests of the error paths: the next n list rebuilds
// fail with GINT_ENOMEM before touching the device (gint_test_fail_rebuilds)
int g_fail_rebuilds = 0;
// rho and the force from D(R) gather their D(R) elements instead of reading
// packed blocks (gint_test_DR_gather)
int g_dr_gather = 0;

gint_status fail(gint_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIPCHK(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(e_ == hipErrorOutOfMemory ? GINT_ENOMEM : GINT_EDEVICE, "%s failed: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);                             \
    } while (0)

#define STCHK(call)                 \
    do {                            \
        gint_status s_ = (call);    \
        if (s_ != GINT_OK)          \
            return s_;              \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf()
    {
        if (p)
            (void)hipFree(p);
    }
    gint_status ensure(size_t need)
    {
        if (need == 0)
            need = 256;
        if (need <= bytes)
            return GINT_OK;
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            bytes = 0;
        }
        hipError_t e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(GINT_ENOMEM, "hipMalloc(%zu) failed: %s", need, hipGetErrorString(e));
        }
        bytes = need;
        return GINT_OK;
    }
    template <typename T>
    T *as() const
    {
        return static_cast<T *>(p);
    }
};

}  // namespace

struct gint_plan_s {
    unsigned magic = kMagic;
    // set when a failed re-tune could not restore the previous lists: every
    // call but gint_plan_destroy then returns GINT_ESTATE
    bool broken = false;
    int device = 0;
    hipStream_t stream = nullptr;
    // second stream of gint_H_rho_force (created on first use) and its
    // fork / join events
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    gint_precision prec = GINT_FP64;
    Geo geo{};
    int natom = 0, norb = 0, nrad = 0, nspecies = 0;
    double dV = 0.0;
    double rc_max = 0.0;
    long long hbudget_req = 0;  // H partial-buffer budget in bytes (0 = automatic)
    long long nblock = 0;       // H block partials over all batches
    void *ext_hpart = nullptr;  // H partial buffer lent by a batch (shared by its chain)
    size_t ext_hpart_bytes = 0;
    long long gen = 0;          // bumped whenever the lists are rebuilt
    int mno = 0;                // most orbitals of any species
    double brad = 0.0;          // radius of a full batch's point box
    std::vector<int> slab;      // batch ranges [slab[i], slab[i+1]) of the H path
    long long nent = 0, nimg = 0, ngb = 0, npair = 0, ngbatch = 0;

    // basis and atoms
    DevBuf rad, sp, knots, s0, sn, coef, scratch;
    DevBuf spc_in, spc, pos_in, xw_in, xw, keys, perm, inv_perm, orb0, orb_atom;
    // binning lists
    DevBuf cnt_e, cnt_i, cnt_g, cnt_s, bptr, iptr, bgptr, soff, maxv;
    DevBuf ent_atom, ent_img, img, bgrp;
    DevBuf gcnt, gcoff, gptr, gbatch;
    DevBuf mark, mscan, pair_index, pairA, pairB;
    // work buffers
    DevBuf Hpart, S2pk, Fent, sums, readback;
    DevBuf cnt_blk, boff, acnt, aptr, aent, abat, pcnt, pptr, plist, lcnt, lptr, blist;
    DevBuf ucnt, uptr, blist_ub;  // per-pair list bounds, their offsets, the lists at those offsets
    DevBuf pown, lsl, slabq;  // owner of each owned pair; slab ranges of its block list
    DevBuf dk_desc;           // per block-list entry: batch and the two entries (gint_build_DK)
    long long nlist = 0;      // entries of the pairs' block lists
    long long dk_gen = -1;    // list generation of dk_desc
    DevBuf scan_tmp;          // tile sums of the list scans
    // H(R) blocks: internal atom of each image, wrap shift of each atom,
    // the caller's R list as a box map (rebuilt when the lists or the list
    // change)
    DevBuf img_atom, wsh, rmap;
    long long hr_gen = -1;     // list generation of img_atom / wsh / nbmax_img
    long long hrfix_gen = -1;  // list generation of the sorted triples
    int nbmax_img = 0;
    std::vector<int> hr_key;
    // fixed-order H(R): per-image identity entries, per-batch block offsets
    // of the unfolded images, sorted triple keys and their runs
    DevBuf hk_phase;  // (cos, sin) phases of gint_HR_to_Hk
    DevBuf Fimg;      // per-(batch, image) force partials of gint_forceR
    DevBuf img_id, cnt_u, boff_u, hkey, hkey2, hcode, hcode2, hflag, hfscan, tstart, tkey, sort_tmp, hbad;
    long long nblock_u = 0;
    int ntri = 0;
    long long hblk_gen = -1;   // list generation of img_id / boff_u / nblock_u
    long long htri_gen = -1;   // list generation of the sorted triples (or of their failure)
    bool htri_bad = false;     // an image pair spans more than kHRBox cells: no triples
    // packed D(R) blocks of gint_build_rhoR / gint_forceR: triple of every
    // block entry (per geometry), packed S and its nonzero flags (per call)
    DevBuf etri, spk, snz;
    long long etri_gen = -1;
    bool hr_fixed = false;  // the partials fit the budget: sorted-triple path
    size_t hbudget_eff = 0;  // partial-buffer budget of the last list build
    int npair_owned = 0;          // owned atom pairs (entries of plist)
    // owned pairs heaviest first (block count over all slabs): launch order of
    // the per-pair reductions and of D_K; pord holds [idx | order], pcost
    // [cost | sorted cost]
    DevBuf pcost, pord, psort_tmp;
    // canonical H(R) triples heaviest first, laid out like pcost / pord
    DevBuf tcost, tord, tsort_tmp;
    std::vector<int> slab_q;      // first block partial of each slab (+ end)
    int nbmax = 0, ngbmax = 0;  // most atoms / atom groups reaching one batch

    // optional per-kernel timing (events on the plan's stream)
    bool timing = false;
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> event_pool;
    double timed_ms[GINT_NKERNEL] = {0};
    int timed_n[GINT_NKERNEL] = {0};

    ~gint_plan_s()
    {
        if (aux) {
            (void)hipStreamSynchronize(aux);
            (void)hipStreamDestroy(aux);
        }
        if (ev_fork)
            (void)hipEventDestroy(ev_fork);
        if (ev_join)
            (void)hipEventDestroy(ev_join);
        for (auto &m : marks) {
            (void)hipEventDestroy(m.a);
            (void)hipEventDestroy(m.b);
        }
        for (auto e : event_pool)
            (void)hipEventDestroy(e);
    }

    bool f32() const { return prec != GINT_FP64; }  // FP32 tiles for all but FP64
    void *hpart() const { return ext_hpart ? ext_hpart : Hpart.p; }
    const int *porder() const { return npair_owned > 0 ? pord.as<int>() + npair_owned + 1 : nullptr; }
    AtomLists atom_lists() const
    {
        AtomLists a;
        a.aptr = aptr.as<int>();
        a.aent = aent.as<int>();
        a.abat = abat.as<int>();
        a.pptr = pptr.as<int>();
        a.plist = plist.as<int>();
        return a;
    }
    Basis basis() const
    {
        Basis b;
        b.rad = rad.as<DevRadial>();
        b.sp = sp.as<DevSpecies>();
        b.coef = coef.as<double>();
        b.spc = spc.as<int>();
        b.xw = xw.as<double>();
        b.perm = perm.as<int>();
        b.inv_perm = inv_perm.as<int>();
        b.orb0 = orb0.as<int>();
        b.orb_atom = orb_atom.as<int>();
        return b;
    }
    Bins bins() const
    {
        Bins b;
        b.bptr = bptr.as<int>();
        b.ent_atom = ent_atom.as<int>();
        b.ent_img = ent_img.as<int>();
        b.img = img.as<int>();
        b.bgptr = bgptr.as<int>();
        b.bgrp = bgrp.as<int>();
        b.gptr = gptr.as<int>();
        b.gbatch = gbatch.as<int>();
        b.pairA = pairA.as<int>();
        b.pairB = pairB.as<int>();
        b.pair_index = pair_index.as<int>();
        return b;
    }
};

namespace {

bool finite3(const double *p, long long n)
{
    for (long long i = 0; i < n; ++i)
        if (!std::isfinite(p[i]))
            return false;
    return true;
}

gint_status check_plan(gint_plan p)
{
    if (!p)
        return fail(GINT_EINVAL, "plan is NULL");
    if (p->magic != kMagic)
        return fail(GINT_ESTATE, "plan is destroyed or corrupted");
    if (p->broken)
        return fail(GINT_ESTATE, "plan lost its lists in a failed gint_plan_tune; only gint_plan_destroy is valid");
    return GINT_OK;
}

// Select the device the plan lives on; refuse anything that is not gfx950.
gint_status device_ok(int *dev)
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0)
        return fail(GINT_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    HIPCHK(hipGetDevice(dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, *dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GINT_EDEVICE, "device %d is %s; this library is built for gfx950 only", *dev, prop.gcnArchName);
    return GINT_OK;
}

void set_batch(Geo &g, const int bs[3])
{
    for (int k = 0; k < 3; ++k) {
        g.bs[k] = bs[k];
        g.nb[k] = (g.N[k] + bs[k] - 1) / bs[k];
    }
    g.P = bs[0] * bs[1] * bs[2];
    g.nbatch = g.nb[0] * g.nb[1] * g.nb[2];
    // compact tiles of batches: a contiguous range of batch ids is a compact
    // region of the mesh (the atoms, and D blocks, it needs overlap)
    for (int k = 0; k < 3; ++k)
        g.bt[k] = g.nb[k] % 4 == 0 ? 4 : (g.nb[k] % 2 == 0 ? 2 : 1);
}

// Radius of the bounding sphere of a full batch's point box.
double batch_radius(const Geo &g)
{
    double rad = 0.0;
    for (int m = 0; m < 8; ++m) {
        double x[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 3; ++k) {
            const double sgn = (m >> k) & 1 ? 0.5 : -0.5;
            const double f = sgn * (double)(g.bs[k] - 1) / g.N[k];
            for (int c = 0; c < 3; ++c)
                x[c] += f * g.lat[3 * k + c];
        }
        rad = std::max(rad, std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]));
    }
    return rad;
}

// Largest lattice multiple any batch can need, given the batch shape.
double max_image_index(const Geo &g, double rc)
{
    double m = 0.0;
    double sd[3] = {(double)g.bs[0] / g.N[0], (double)g.bs[1] / g.N[1], (double)g.bs[2] / g.N[2]};
    double x[3];
    for (int k = 0; k < 3; ++k)
        x[k] = sd[0] * g.lat[k] + sd[1] * g.lat[3 + k] + sd[2] * g.lat[6 + k];
    const double rad = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (int i = 0; i < 3; ++i) {
        const double bn =
            std::sqrt(g.rec[3 * i] * g.rec[3 * i] + g.rec[3 * i + 1] * g.rec[3 * i + 1] + g.rec[3 * i + 2] * g.rec[3 * i + 2]);
        m = std::max(m, (rc + rad) * bn + 2.0);
    }
    return m;
}

hipEvent_t take_event(gint_plan p)
{
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Fold finished marks into the totals and recycle their events.
gint_status drain_marks(gint_plan p)
{
    if (p->marks.empty())
        return GINT_OK;
    HIPCHK(hipStreamSynchronize(p->stream));
    for (auto &m : p->marks) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, m.a, m.b));
        p->timed_ms[m.kind] += ms;
        p->timed_n[m.kind] += 1;
        p->event_pool.push_back(m.a);
        p->event_pool.push_back(m.b);
    }
    p->marks.clear();
    return GINT_OK;
}

// Run `launch` (returns hipError_t), bracketed by events when timing is on.
template <typename F>
gint_status timed_on(gint_plan p, hipStream_t st, int kind, F launch)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (p->timing) {
        if (p->marks.size() > 4096)
            STCHK(drain_marks(p));
        a = take_event(p);
        b = take_event(p);
        if (!a || !b)
            return fail(GINT_EDEVICE, "hipEventCreate failed");
        HIPCHK(hipEventRecord(a, st));
    }
    HIPCHK(launch());
    if (p->timing) {
        HIPCHK(hipEventRecord(b, st));
        p->marks.push_back({kind, a, b});
    }
    return GINT_OK;
}

template <typename F>
gint_status timed(gint_plan p, int kind, F launch)
{
    return timed_on(p, p->stream, kind, launch);
}

// exclusive scan of n ints on stream st (out: n + 1 ints)
gint_status scan_i32(gint_plan p, hipStream_t st, const int *in, long long n, int *out)
{
    STCHK(p->scan_tmp.ensure(sizeof(int) * (size_t)scan_tmp_ints(n)));
    HIPCHK(launch_scan_i32(st, in, n, out, p->scan_tmp.as<int>()));
    return GINT_OK;
}

template <typename T>
gint_status read_scalar(gint_plan p, const T *dev, T *host)
{
    HIPCHK(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return GINT_OK;
}

// Rebuild every list that depends on the atom positions (GintInfo).
gint_status rebuild_lists(gint_plan p, bool resort)
{
    if (g_fail_rebuilds > 0) {
        --g_fail_rebuilds;
        return fail(GINT_ENOMEM, "list rebuild failed (injected by gint_test_fail_rebuilds)");
    }
    Geo &g = p->geo;
    hipStream_t s = p->stream;
    const int na = p->natom;
    HIPCHK(launch_wrap(s, g, p->pos_in.as<double>(), p->xw_in.as<double>(),
                       resort ? p->keys.as<unsigned long long>() : nullptr));
    if (resort)
        HIPCHK(launch_sort_perm(s, na, p->keys.as<unsigned long long>(), p->perm.as<int>(), p->inv_perm.as<int>()));
    HIPCHK(launch_gather_internal(s, na, p->perm.as<int>(), p->xw_in.as<double>(), p->spc_in.as<int>(),
                                  p->xw.as<double>(), p->spc.as<int>()));

    const long long nb = g.nbatch;
    STCHK(p->cnt_e.ensure(sizeof(int) * nb));
    STCHK(p->cnt_i.ensure(sizeof(int) * nb));
    STCHK(p->cnt_g.ensure(sizeof(int) * nb));
    STCHK(p->bptr.ensure(sizeof(int) * (nb + 1)));
    STCHK(p->iptr.ensure(sizeof(int) * (nb + 1)));
    STCHK(p->bgptr.ensure(sizeof(int) * (nb + 1)));
    const Basis B = p->basis();
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_bin_count(s, g, B, p->cnt_e.as<int>(), p->cnt_i.as<int>(), p->cnt_g.as<int>());
    }));
    STCHK(scan_i32(p, s, p->cnt_e.as<int>(), nb, p->bptr.as<int>()));
    STCHK(scan_i32(p, s, p->cnt_i.as<int>(), nb, p->iptr.as<int>()));
    STCHK(scan_i32(p, s, p->cnt_g.as<int>(), nb, p->bgptr.as<int>()));
    // totals (counts are far below 2^31 for any mesh this library accepts,
    // but the image total is checked explicitly)
    int tot[5];
    STCHK(p->maxv.ensure(2 * sizeof(int)));
    HIPCHK(launch_max_i32(s, p->cnt_e.as<int>(), nb, p->maxv.as<int>()));
    HIPCHK(launch_max_i32(s, p->cnt_g.as<int>(), nb, p->maxv.as<int>() + 1));
    HIPCHK(hipMemcpyAsync(&tot[0], p->bptr.as<int>() + nb, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tot[1], p->iptr.as<int>() + nb, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tot[2], p->bgptr.as<int>() + nb, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tot[3], p->maxv.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (tot[0] < 0 || tot[1] < 0 || tot[2] < 0)
        return fail(GINT_EUNSUPPORTED, "binning lists exceed 2^31 entries");
    p->nent = tot[0];
    p->nimg = tot[1];
    p->ngb = tot[2];
    p->nbmax = tot[3];
    p->ngbmax = tot[4];
    if (p->nbmax > kMaxBatchAtoms || p->ngbmax > kMaxBatchGroups)
        return fail(GINT_EUNSUPPORTED, "%d atoms / %d atom groups reach one mesh batch (max %d / %d); use a smaller batch",
                    p->nbmax, p->ngbmax, kMaxBatchAtoms, kMaxBatchGroups);
    {
        // LDS of the point-stationary kernels: every atom of a batch at once
        const size_t esz = p->f32() ? sizeof(float) : sizeof(double);
        const size_t lds_H = esz * (size_t)p->nbmax * g.P * kRow + 16384;
        if (lds_H > 163840)
            return fail(GINT_EUNSUPPORTED, "%d atoms reach one %d-point batch: %zu bytes of LDS; use a smaller batch",
                        p->nbmax, g.P, lds_H);
    }
    STCHK(p->ent_atom.ensure(sizeof(int) * (p->nent + 1)));
    STCHK(p->ent_img.ensure(sizeof(int) * (p->nent + 1)));
    STCHK(p->img.ensure(sizeof(int) * (p->nimg + 1)));
    STCHK(p->bgrp.ensure(sizeof(int) * (p->ngb + 1)));
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_bin_fill(s, g, B, p->bptr.as<int>(), p->iptr.as<int>(), p->bgptr.as<int>(),
                               p->ent_atom.as<int>(), p->ent_img.as<int>(), p->img.as<int>(), p->bgrp.as<int>());
    }));

    // per-group batch lists
    const int ng = g.ngroup;
    const long long ngc = (long long)ng * group_chunks(g);
    STCHK(p->gcnt.ensure(sizeof(int) * (ngc + 1)));
    STCHK(p->gcoff.ensure(sizeof(int) * (ngc + 1)));
    STCHK(p->gptr.ensure(sizeof(int) * (ng + 1)));
    STCHK(timed(p, GINT_K_BIN,
                [&] { return launch_group_count(s, g, p->bgptr.as<int>(), p->bgrp.as<int>(), p->gcnt.as<int>()); }));
    STCHK(scan_i32(p, s, p->gcnt.as<int>(), ngc, p->gcoff.as<int>()));
    int tg = 0;
    STCHK(read_scalar(p, p->gcoff.as<int>() + ngc, &tg));
    if (tg < 0)
        return fail(GINT_EUNSUPPORTED, "group batch lists exceed 2^31 entries");
    p->ngbatch = tg;
    STCHK(p->gbatch.ensure(sizeof(int) * (p->ngbatch + 1)));
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_group_fill(s, g, p->bgptr.as<int>(), p->bgrp.as<int>(), p->gcoff.as<int>(),
                                 p->gbatch.as<int>(), p->gptr.as<int>());
    }));

    // active group pairs
    const long long nn = (long long)ng * ng;
    STCHK(p->mark.ensure(sizeof(int) * nn));
    STCHK(p->mscan.ensure(sizeof(int) * (nn + 1)));
    STCHK(p->pair_index.ensure(sizeof(int) * nn));
    HIPCHK(launch_fill_i32(s, p->mark.as<int>(), nn, 0));
    STCHK(timed(p, GINT_K_BIN,
                [&] { return launch_pair_mark(s, g, p->bgptr.as<int>(), p->bgrp.as<int>(), p->mark.as<int>()); }));
    STCHK(scan_i32(p, s, p->mark.as<int>(), nn, p->mscan.as<int>()));
    int tp = 0;
    STCHK(read_scalar(p, p->mscan.as<int>() + nn, &tp));
    p->npair = tp;
    STCHK(p->pairA.ensure(sizeof(int) * (p->npair + 1)));
    STCHK(p->pairB.ensure(sizeof(int) * (p->npair + 1)));
    HIPCHK(launch_pair_list(s, ng, p->mark.as<int>(), p->mscan.as<int>(), p->pair_index.as<int>(),
                            p->pairA.as<int>(), p->pairB.as<int>()));

    // point-stationary H: per-batch block offsets, per-atom entry lists and
    // owned-partner lists, and the batch ranges (slabs) whose block partials
    // fit the partial-buffer budget
    STCHK(p->cnt_blk.ensure(sizeof(int) * nb));
    STCHK(p->boff.ensure(sizeof(int) * (nb + 1)));
    HIPCHK(launch_block_count(s, g.nbatch, p->bptr.as<int>(), p->cnt_blk.as<int>()));
    STCHK(scan_i32(p, s, p->cnt_blk.as<int>(), nb, p->boff.as<int>()));
    // (na: atom count, set above)
    STCHK(p->acnt.ensure(sizeof(int) * na));
    STCHK(p->aptr.ensure(sizeof(int) * (na + 1)));
    STCHK(p->aent.ensure(sizeof(int) * (p->nent + 1)));
    STCHK(p->abat.ensure(sizeof(int) * (p->nent + 1)));
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_atom_count(s, na, p->gptr.as<int>(), p->gbatch.as<int>(), p->bptr.as<int>(),
                                 p->ent_atom.as<int>(), p->acnt.as<int>());
    }));
    STCHK(scan_i32(p, s, p->acnt.as<int>(), na, p->aptr.as<int>()));
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_atom_fill(s, na, p->gptr.as<int>(), p->gbatch.as<int>(), p->bptr.as<int>(),
                                p->ent_atom.as<int>(), p->aptr.as<int>(), p->aent.as<int>(), p->abat.as<int>());
    }));
    STCHK(p->pcnt.ensure(sizeof(int) * na));
    STCHK(p->pptr.ensure(sizeof(int) * (na + 1)));
    const Basis B2 = p->basis();
    STCHK(timed(p, GINT_K_BIN, [&] { return launch_partners(s, g, B2, p->brad, nullptr, p->pcnt.as<int>(), nullptr); }));
    STCHK(scan_i32(p, s, p->pcnt.as<int>(), na, p->pptr.as<int>()));
    // the block total and the owned-pair count (the per-batch block offsets
    // come to the host only when H needs more than one slab, below)
    int tblk = 0, tpart = 0;
    HIPCHK(hipMemcpyAsync(&tblk, p->boff.as<int>() + nb, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&tpart, p->pptr.as<int>() + na, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (tblk < 0 || tpart < 0)
        return fail(GINT_EUNSUPPORTED, "block lists exceed 2^31 entries");
    p->nblock = tblk;
    STCHK(p->plist.ensure(sizeof(int) * (tpart + 1)));
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_partners(s, g, B2, p->brad, p->pptr.as<int>(), p->pcnt.as<int>(), p->plist.as<int>());
    }));
    // block lists of the owned pairs (batch order) for the H reduction: one
    // intersection pass writes each list at the offset of its bound (the
    // smaller of the two atoms' entry counts) and its length; the lists are
    // then compacted
    p->npair_owned = tpart;
    STCHK(p->lcnt.ensure(sizeof(int) * (tpart + 1)));
    STCHK(p->lptr.ensure(sizeof(int) * (tpart + 1)));
    STCHK(p->ucnt.ensure(sizeof(int) * (tpart + 1)));
    STCHK(p->uptr.ensure(sizeof(int) * (tpart + 1)));
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_pair_ub(s, na, tpart, p->aptr.as<int>(), p->pptr.as<int>(), p->plist.as<int>(),
                              p->ucnt.as<int>());
    }));
    STCHK(scan_i32(p, s, p->ucnt.as<int>(), tpart, p->uptr.as<int>()));
    int tub = 0;
    HIPCHK(hipMemcpyAsync(&tub, p->uptr.as<int>() + tpart, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (tub < 0)
        return fail(GINT_EUNSUPPORTED, "pair block lists exceed 2^31 entries");
    STCHK(p->blist_ub.ensure(sizeof(int) * ((size_t)tub + 1)));
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_pair_blocks(s, na, tpart, p->aptr.as<int>(), p->aent.as<int>(), p->abat.as<int>(),
                                  p->bptr.as<int>(), p->boff.as<int>(), p->pptr.as<int>(), p->plist.as<int>(),
                                  p->lcnt.as<int>(), p->uptr.as<int>(), p->blist_ub.as<int>());
    }));
    STCHK(scan_i32(p, s, p->lcnt.as<int>(), tpart, p->lptr.as<int>()));
    int tlist = 0;
    HIPCHK(hipMemcpyAsync(&tlist, p->lptr.as<int>() + tpart, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (tlist < 0)
        return fail(GINT_EUNSUPPORTED, "pair block lists exceed 2^31 entries");
    p->nlist = tlist;
    STCHK(p->blist.ensure(sizeof(int) * ((size_t)tlist + 1)));
    STCHK(timed(p, GINT_K_BIN, [&] {
        return launch_list_compact(s, tpart, p->uptr.as<int>(), p->lptr.as<int>(), p->lcnt.as<int>(),
                                   p->blist_ub.as<int>(), p->blist.as<int>());
    }));
    const size_t esz = p->f32() ? sizeof(float) : sizeof(double);
    const size_t blk_bytes = esz * (size_t)block_pitch(p->mno, (int)esz);
    size_t budget = p->hbudget_req > 0 ? (size_t)p->hbudget_req : (size_t)64 << 30;
    if (p->ext_hpart)
        budget = p->ext_hpart_bytes;
    else if (p->hbudget_req <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && fr / 3 < budget)
            budget = fr / 3;
    }
    p->hbudget_eff = budget;
    p->slab.assign(1, 0);
    p->slab_q.assign(1, 0);
    long long most = 0;
    if (nb > 0 && (long long)(budget / blk_bytes) >= (long long)tblk) {
        // every partial fits: one slab
        p->slab.push_back((int)nb);
        p->slab_q.push_back(tblk);
        most = tblk;
    } else {
        std::vector<int> hboff(nb + 1);
        HIPCHK(hipMemcpyAsync(hboff.data(), p->boff.p, sizeof(int) * (nb + 1), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        // a range holds at least one whole batch
        long long per_slab = (long long)(budget / blk_bytes);
        for (int b = 0; b < nb; ++b)
            per_slab = std::max(per_slab, (long long)hboff[b + 1] - hboff[b]);
        for (int b = 0; b < nb;) {
            int e = b;
            while (e < nb && (long long)hboff[e + 1] - hboff[b] <= per_slab)
                ++e;
            if (e == b)
                ++e;
            most = std::max(most, (long long)hboff[e] - hboff[b]);
            p->slab.push_back(e);
            p->slab_q.push_back(hboff[e]);
            b = e;
        }
    }
    {
        const int ns = (int)p->slab.size() - 1;
        STCHK(p->slabq.ensure(sizeof(int) * (ns + 1)));
        STCHK(p->pown.ensure(sizeof(int) * (tpart + 1)));
        STCHK(p->lsl.ensure(sizeof(int) * ((size_t)tpart * (ns + 1) + 1)));
        HIPCHK(hipMemcpyAsync(p->slabq.p, p->slab_q.data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice, s));
        STCHK(timed(p, GINT_K_BIN, [&] {
            return launch_pair_slabs(s, na, tpart, p->pptr.as<int>(), p->lptr.as<int>(), p->blist.as<int>(), ns,
                                     p->slabq.as<int>(), p->pown.as<int>(), p->lsl.as<int>());
        }));
        STCHK(p->pcost.ensure(sizeof(int) * 2 * ((size_t)tpart + 1)));
        STCHK(p->pord.ensure(sizeof(int) * 2 * ((size_t)tpart + 1)));
        size_t tb = 0;
        HIPCHK(launch_item_order(s, nullptr, tb, tpart, ns + 1, ns, nullptr, nullptr, nullptr, nullptr, nullptr));
        STCHK(p->psort_tmp.ensure(tb));
        STCHK(timed(p, GINT_K_BIN, [&] {
            return launch_item_order(s, p->psort_tmp.p, tb, tpart, ns + 1, ns, p->lsl.as<int>(), p->pcost.as<int>(),
                                     p->pcost.as<int>() + tpart + 1, p->pord.as<int>(),
                                     p->pord.as<int>() + tpart + 1);
        }));
        HIPCHK(hipStreamSynchronize(s));  // slab_q (host) outlives the copy
    }
    if (p->ext_hpart) {
        if (blk_bytes * (size_t)most > p->ext_hpart_bytes)
            return fail(GINT_ENOMEM, "a batch of the cell needs %zu bytes of H partials", blk_bytes * (size_t)most);
    } else {
        STCHK(p->Hpart.ensure(blk_bytes * (size_t)std::max(most, 1LL)));
    }
    ++p->gen;
    STCHK(p->S2pk.ensure(esz * 16 * 512 * (size_t)p->npair));
    STCHK(p->Fent.ensure(sizeof(double) * 3 * (size_t)(p->nent + 1)));
    return GINT_OK;
}

gint_status validate_species(int nspecies, const gint_species *species, double *rc_max)
{
    if (nspecies <= 0 || !species)
        return fail(GINT_EINVAL, "nspecies must be >= 1 and species non-NULL");
    if (nspecies > kMaxSpecies)
        return fail(GINT_EUNSUPPORTED, "%d species (max %d)", nspecies, kMaxSpecies);
    int nrad_total = 0;
    for (int s = 0; s < nspecies; ++s)
        nrad_total += species[s].nradial > 0 ? species[s].nradial : 0;
    if (nrad_total > kMaxRadTotal)
        return fail(GINT_EUNSUPPORTED, "%d radials over all species (max %d)", nrad_total, kMaxRadTotal);
    *rc_max = 0.0;
    for (int s = 0; s < nspecies; ++s) {
        const gint_species &S = species[s];
        if (S.nradial <= 0 || !S.radial)
            return fail(GINT_EINVAL, "species %d has no radials", s);
        if (S.nradial > kMaxRad)
            return fail(GINT_EUNSUPPORTED, "species %d has %d radials (max %d)", s, S.nradial, kMaxRad);
        int norb = 0;
        for (int k = 0; k < S.nradial; ++k) {
            const gint_radial &R = S.radial[k];
            if (R.l < 0)
                return fail(GINT_EINVAL, "species %d radial %d: l < 0", s, k);
            if (R.l > 2)
                return fail(GINT_EUNSUPPORTED, "species %d radial %d: l = %d (max 2)", s, k, R.l);
            if (R.nr < 4)
                return fail(GINT_EINVAL, "species %d radial %d: nr = %d (need >= 4)", s, k, R.nr);
            if (!(R.dr > 0.0) || !std::isfinite(R.dr))
                return fail(GINT_EINVAL, "species %d radial %d: dr must be positive", s, k);
            if (!R.f)
                return fail(GINT_EINVAL, "species %d radial %d: f is NULL", s, k);
            if (!finite3(R.f, R.nr) || !std::isfinite(R.dfdr_0) || !std::isfinite(R.dfdr_rc))
                return fail(GINT_EINVAL, "species %d radial %d: non-finite table", s, k);
            norb += 2 * R.l + 1;
            *rc_max = std::max(*rc_max, (R.nr - 1) * R.dr);
        }
        if (norb > kMaxOrb)
            return fail(GINT_EUNSUPPORTED, "species %d has %d orbitals (max %d)", s, norb, kMaxOrb);
    }
    return GINT_OK;
}

gint_status validate_geometry(const double *lattice, const int *grid, Geo &g)
{
    if (!lattice || !grid)
        return fail(GINT_EINVAL, "lattice and grid must be non-NULL");
    if (!finite3(lattice, 9))
        return fail(GINT_EINVAL, "lattice has non-finite entries");
    for (int k = 0; k < 3; ++k)
        if (grid[k] < 1)
            return fail(GINT_EINVAL, "grid[%d] = %d must be >= 1", k, grid[k]);
    const long long ng = (long long)grid[0] * grid[1] * grid[2];
    if (ng >= 0x7fffffffLL)
        return fail(GINT_EUNSUPPORTED, "mesh of %lld points exceeds 2^31", ng);
    const double *a1 = lattice, *a2 = lattice + 3, *a3 = lattice + 6;
    const double det = a1[0] * (a2[1] * a3[2] - a2[2] * a3[1]) - a1[1] * (a2[0] * a3[2] - a2[2] * a3[0]) +
                       a1[2] * (a2[0] * a3[1] - a2[1] * a3[0]);
    double scale = 0.0;
    for (int i = 0; i < 9; ++i)
        scale = std::max(scale, std::fabs(lattice[i]));
    if (!(std::fabs(det) > 1e-12 * scale * scale * scale) || scale == 0.0)
        return fail(GINT_EINVAL, "lattice is singular");
    std::memcpy(g.lat, lattice, sizeof(double) * 9);
    const double *A[3] = {a1, a2, a3};
    for (int i = 0; i < 3; ++i) {
        const double *u = A[(i + 1) % 3], *v = A[(i + 2) % 3];
        g.rec[3 * i + 0] = (u[1] * v[2] - u[2] * v[1]) / det;
        g.rec[3 * i + 1] = (u[2] * v[0] - u[0] * v[2]) / det;
        g.rec[3 * i + 2] = (u[0] * v[1] - u[1] * v[0]) / det;
    }
    g.ortho = (lattice[1] == 0.0 && lattice[2] == 0.0 && lattice[3] == 0.0 && lattice[5] == 0.0 &&
               lattice[6] == 0.0 && lattice[7] == 0.0)
                  ? 1
                  : 0;
    for (int k = 0; k < 3; ++k)
        g.N[k] = grid[k];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            g.h[3 * i + k] = lattice[3 * i + k] / grid[i];
    return GINT_OK;
}

}  // namespace

extern "C" {

const char *gint_status_string(gint_status s)
{
    switch (s) {
    case GINT_OK:
        return "GINT_OK";
    case GINT_EINVAL:
        return "GINT_EINVAL: invalid argument";
    case GINT_ENOMEM:
        return "GINT_ENOMEM: allocation failed";
    case GINT_EDEVICE:
        return "GINT_EDEVICE: device unavailable or HIP error";
    case GINT_EUNSUPPORTED:
        return "GINT_EUNSUPPORTED: valid but unsupported request";
    case GINT_ESTATE:
        return "GINT_ESTATE: invalid plan state";
    }
    return "unknown gint_status";
}

const char *gint_last_error(void) { return g_last_error.c_str(); }

static gint_status plan_create(const double lattice[9], const int grid[3], int nspecies, const gint_species *species,
                               int natom, const int *species_of_atom, const double *positions, gint_precision prec,
                               void *hip_stream, void *ext_hpart, size_t ext_hpart_bytes, gint_plan *out);

gint_status gint_plan_create(const double lattice[9], const int grid[3], int nspecies, const gint_species *species,
                             int natom, const int *species_of_atom, const double *positions, gint_precision prec,
                             void *hip_stream, gint_plan *out)
{
    return plan_create(lattice, grid, nspecies, species, natom, species_of_atom, positions, prec, hip_stream, nullptr,
                       0, out);
}

static gint_status plan_create(const double lattice[9], const int grid[3], int nspecies, const gint_species *species,
                               int natom, const int *species_of_atom, const double *positions, gint_precision prec,
                               void *hip_stream, void *ext_hpart, size_t ext_hpart_bytes, gint_plan *out)
{
    if (!out)
        return fail(GINT_EINVAL, "out is NULL");
    Geo g{};
    STCHK(validate_geometry(lattice, grid, g));
    double rc_max = 0.0;
    STCHK(validate_species(nspecies, species, &rc_max));
    if (natom < 1 || natom > kMaxAtoms)
        return fail(GINT_EINVAL, "natom = %d outside [1, %d]", natom, kMaxAtoms);
    if (!species_of_atom || !positions)
        return fail(GINT_EINVAL, "species_of_atom and positions must be non-NULL");
    for (int i = 0; i < natom; ++i)
        if (species_of_atom[i] < 0 || species_of_atom[i] >= nspecies)
            return fail(GINT_EINVAL, "species_of_atom[%d] = %d out of range", i, species_of_atom[i]);
    if (!finite3(positions, 3LL * natom))
        return fail(GINT_EINVAL, "positions have non-finite entries");
    if ((int)prec < GINT_FP64 || (int)prec > GINT_FP16_SPLIT)
        return fail(GINT_EINVAL, "unknown precision %d", (int)prec);
    g.natom = natom;
    g.ngroup = (natom + kGroup - 1) / kGroup;
    const int bs0[3] = {4, 4, 2};
    set_batch(g, bs0);
    if (max_image_index(g, rc_max) >= 126.0)
        return fail(GINT_EUNSUPPORTED, "cutoff spans more than 125 cells");

    // host tables: radials sorted by l (stable), orbital slots, orbital maps
    std::vector<DevRadial> rad;
    std::vector<DevSpecies> sp(nspecies);
    std::vector<double> knots, s0, sn;
    int coef_off = 0;
    for (int s = 0; s < nspecies; ++s) {
        const gint_species &S = species[s];
        sp[s].rad0 = (int)rad.size();
        for (int o = 0; o < kMaxOrb; ++o) {
            sp[s].orb_rad[o] = 0;
            sp[s].orb_m[o] = 0;
        }
        sp[s].nrad = S.nradial;
        sp[s].rc = 0.0;
        int orb = 0;
        for (int l = 0; l <= 2; ++l)
            for (int k = 0; k < S.nradial; ++k) {
                const gint_radial &R = S.radial[k];
                if (R.l != l)
                    continue;
                DevRadial d;
                for (int m = 0; m < 2 * l + 1; ++m) {
                    sp[s].orb_rad[orb + m] = (signed char)rad.size();
                    sp[s].orb_m[orb + m] = (signed char)(m - l);
                }
                d.dr = R.dr;
                d.inv_dr = 1.0 / R.dr;
                d.rc = (R.nr - 1) * R.dr;
                d.l = R.l;
                d.nr = R.nr;
                d.orb0 = orb;
                d.coef_off = coef_off;
                d.knot_off = (int)knots.size();
                coef_off += 4 * (R.nr - 1);
                knots.insert(knots.end(), R.f, R.f + R.nr);
                s0.push_back(R.dfdr_0);
                sn.push_back(R.dfdr_rc);
                rad.push_back(d);
                orb += 2 * l + 1;
                sp[s].rc = std::max(sp[s].rc, d.rc);
            }
        sp[s].norb = orb;
    }
    std::vector<int> orb0(natom + 1);
    int norb = 0;
    for (int i = 0; i < natom; ++i) {
        orb0[i] = norb;
        norb += sp[species_of_atom[i]].norb;
    }
    orb0[natom] = norb;
    std::vector<int> orb_atom(norb);
    for (int i = 0; i < natom; ++i)
        for (int o = orb0[i]; o < orb0[i + 1]; ++o)
            orb_atom[o] = i;

    int dev = 0;
    STCHK(device_ok(&dev));

    gint_plan p = new (std::nothrow) gint_plan_s();
    if (!p)
        return fail(GINT_ENOMEM, "host allocation failed");
    p->device = dev;
    p->stream = (hipStream_t)hip_stream;
    p->ext_hpart = ext_hpart;
    p->ext_hpart_bytes = ext_hpart_bytes;
    p->prec = prec;
    p->geo = g;
    p->natom = natom;
    p->norb = norb;
    p->nrad = (int)rad.size();
    p->geo.nrad = p->nrad;
    p->geo.nspecies = nspecies;
    p->nspecies = nspecies;
    p->rc_max = rc_max;
    for (int s = 0; s < nspecies; ++s)
        p->mno = std::max(p->mno, sp[s].norb);
    p->brad = batch_radius(g);
    p->dV = std::fabs(g.lat[0] * (g.lat[4] * g.lat[8] - g.lat[5] * g.lat[7]) -
                      g.lat[1] * (g.lat[3] * g.lat[8] - g.lat[5] * g.lat[6]) +
                      g.lat[2] * (g.lat[3] * g.lat[7] - g.lat[4] * g.lat[6])) /
            ((double)g.N[0] * g.N[1] * g.N[2]);

    auto upload = [&](DevBuf &b, const void *h, size_t bytes) -> gint_status {
        STCHK(b.ensure(bytes));
        if (bytes)
            HIPCHK(hipMemcpyAsync(b.p, h, bytes, hipMemcpyHostToDevice, p->stream));
        return GINT_OK;
    };
    gint_status st = GINT_OK;
    int npow2 = 1;
    while (npow2 < natom)
        npow2 <<= 1;
    do {
        if ((st = upload(p->rad, rad.data(), sizeof(DevRadial) * rad.size())) != GINT_OK) break;
        if ((st = upload(p->sp, sp.data(), sizeof(DevSpecies) * sp.size())) != GINT_OK) break;
        if ((st = upload(p->knots, knots.data(), sizeof(double) * knots.size())) != GINT_OK) break;
        if ((st = upload(p->s0, s0.data(), sizeof(double) * s0.size())) != GINT_OK) break;
        if ((st = upload(p->sn, sn.data(), sizeof(double) * sn.size())) != GINT_OK) break;
        if ((st = upload(p->spc_in, species_of_atom, sizeof(int) * natom)) != GINT_OK) break;
        if ((st = upload(p->pos_in, positions, sizeof(double) * 3 * natom)) != GINT_OK) break;
        if ((st = upload(p->orb0, orb0.data(), sizeof(int) * (natom + 1))) != GINT_OK) break;
        if ((st = upload(p->orb_atom, orb_atom.data(), sizeof(int) * std::max(norb, 1))) != GINT_OK) break;
        if ((st = p->coef.ensure(sizeof(double) * coef_off)) != GINT_OK) break;
        if ((st = p->scratch.ensure(sizeof(double) * 3 * knots.size())) != GINT_OK) break;
        if ((st = p->spc.ensure(sizeof(int) * natom)) != GINT_OK) break;
        if ((st = p->xw_in.ensure(sizeof(double) * 3 * natom)) != GINT_OK) break;
        if ((st = p->xw.ensure(sizeof(double) * 3 * natom)) != GINT_OK) break;
        if ((st = p->keys.ensure(sizeof(unsigned long long) * npow2)) != GINT_OK) break;
        if ((st = p->perm.ensure(sizeof(int) * natom)) != GINT_OK) break;
        if ((st = p->inv_perm.ensure(sizeof(int) * natom)) != GINT_OK) break;
        hipError_t e = launch_spline(p->stream, p->nrad, p->rad.as<DevRadial>(), p->knots.as<double>(),
                                     p->s0.as<double>(), p->sn.as<double>(), p->coef.as<double>(),
                                     p->scratch.as<double>());
        if (e != hipSuccess) {
            st = fail(GINT_EDEVICE, "spline kernel launch failed: %s", hipGetErrorString(e));
            break;
        }
        if ((st = rebuild_lists(p, true)) != GINT_OK) {
            // so many atoms reach a 32-point batch that its tiles exceed the
            // LDS: FP64 and FP32 plans start with 16-point batches instead
            if (st != GINT_EUNSUPPORTED || (prec != GINT_FP64 && prec != GINT_FP32))
                break;
            const int bs1[3] = {2, 2, 4};
            Geo g1 = p->geo;
            set_batch(g1, bs1);
            if (max_image_index(g1, rc_max) >= 126.0)
                break;
            p->geo = g1;
            p->brad = batch_radius(g1);
            if ((st = rebuild_lists(p, true)) != GINT_OK)
                break;
        }
        e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) {
            st = fail(GINT_EDEVICE, "plan construction failed on the device: %s", hipGetErrorString(e));
            break;
        }
    } while (0);
    if (st != GINT_OK) {
        (void)hipStreamSynchronize(p->stream);
        p->magic = 0;
        delete p;
        return st;
    }
    *out = p;
    return GINT_OK;
}

gint_status gint_plan_set_positions(gint_plan p, const double *positions)
{
    STCHK(check_plan(p));
    if (!positions)
        return fail(GINT_EINVAL, "positions is NULL");
    if (!finite3(positions, 3LL * p->natom))
        return fail(GINT_EINVAL, "positions have non-finite entries");
    HIPCHK(hipSetDevice(p->device));
    HIPCHK(hipMemcpyAsync(p->pos_in.p, positions, sizeof(double) * 3 * p->natom, hipMemcpyHostToDevice, p->stream));
    STCHK(rebuild_lists(p, false));
    return GINT_OK;
}

gint_status gint_plan_tune(gint_plan p, const int batch[3], long long h_budget_bytes)
{
    STCHK(check_plan(p));
    if (!batch)
        return fail(GINT_EINVAL, "batch is NULL");
    for (int k = 0; k < 3; ++k)
        if (batch[k] < 1)
            return fail(GINT_EINVAL, "batch[%d] = %d must be >= 1", k, batch[k]);
    const int P = batch[0] * batch[1] * batch[2];
    if (P != 16 && P != 32)
        return fail(GINT_EINVAL, "batch holds %d points (must be 16 or 32)", P);
    if (P != 32 && p->prec != GINT_FP64 && p->prec != GINT_FP32)
        return fail(GINT_EINVAL, "16-bit modes need 32-point batches (one instruction's K)");
    if (h_budget_bytes < 0)
        return fail(GINT_EINVAL, "h_budget_bytes must be >= 0");
    Geo g = p->geo;
    set_batch(g, batch);
    if (max_image_index(g, p->rc_max) >= 126.0)
        return fail(GINT_EUNSUPPORTED, "cutoff spans more than 125 cells");
    HIPCHK(hipSetDevice(p->device));
    const Geo g_old = p->geo;
    const double brad_old = p->brad;
    const long long hb_old = p->hbudget_req;
    p->geo = g;
    p->brad = batch_radius(g);
    p->hbudget_req = h_budget_bytes;
    const gint_status st = rebuild_lists(p, false);
    if (st != GINT_OK) {
        // keep the plan usable with its previous shape
        const std::string why = g_last_error;
        p->geo = g_old;
        p->brad = brad_old;
        p->hbudget_req = hb_old;
        if (rebuild_lists(p, false) != GINT_OK) {
            p->broken = true;
            return fail(st, "%s (and restoring the previous batch shape failed: the plan is unusable)",
                        why.c_str());
        }
        return fail(st, "%s", why.c_str());
    }
    return GINT_OK;
}

gint_status gint_plan_set_stream(gint_plan p, void *hip_stream)
{
    STCHK(check_plan(p));
    p->stream = (hipStream_t)hip_stream;
    return GINT_OK;
}

static gint_status build_H_impl(gint_plan p, const double *W, double wscale, double *H)
{
    STCHK(check_plan(p));
    if (!W || !H)
        return fail(GINT_EINVAL, "V and H must be non-NULL device pointers");
    HIPCHK(hipSetDevice(p->device));
    const Bins bn = p->bins();
    const Basis B = p->basis();
    STCHK(timed(p, GINT_K_H_FILL,
                [&] { return launch_fill_f64(p->stream, H, (long long)p->norb * p->norb, 0.0); }));
    for (size_t i = 0; i + 1 < p->slab.size(); ++i) {
        const int b0 = p->slab[i], b1 = p->slab[i + 1];
        STCHK(timed(p, GINT_K_H, [&] {
            return launch_H_batch(p->stream, (int)p->prec, p->geo, bn, B, p->nbmax, b0, b1, W, wscale, p->boff.as<int>(),
                                  p->mno, p->hpart());
        }));
        STCHK(timed(p, GINT_K_H_REDUCE, [&] {
            return launch_H_pairreduce(p->stream, p->f32(), p->npair_owned, p->porder(), p->pown.as<int>(),
                                       p->plist.as<int>(), p->lsl.as<int>(), (int)p->slab.size() - 1, (int)i,
                                       p->blist.as<int>(), B, p->mno, p->norb, p->hpart(), p->slab_q[i],
                                       i > 0 ? 1 : 0, H);
        }));
    }
    return GINT_OK;
}

gint_status gint_build_H(gint_plan p, const double *V_dev, double *H_dev)
{
    STCHK(check_plan(p));
    return build_H_impl(p, V_dev, p->dV, H_dev);
}

gint_status gint_build_H_weighted(gint_plan p, const double *w_dev, double *H_dev)
{
    return build_H_impl(p, w_dev, 1.0, H_dev);
}

gint_status gint_build_DK(gint_plan p, const double *W_dev, double *DK_dev)
{
    STCHK(check_plan(p));
    if (!DK_dev)
        return fail(GINT_EINVAL, "DK must be a non-NULL device pointer");
    if (p->geo.P != 16 && p->geo.P != 32)
        return fail(GINT_EUNSUPPORTED, "batch of %d points", p->geo.P);
    HIPCHK(hipSetDevice(p->device));
    const Bins bn = p->bins();
    const Basis B = p->basis();
    STCHK(timed(p, GINT_K_H_FILL,
                [&] { return launch_fill_f64(p->stream, DK_dev, 3LL * p->norb * p->norb, 0.0); }));
    if (p->dk_gen != p->gen) {
        // per list entry: its batch and the two atoms' entries (once per geometry)
        STCHK(p->dk_desc.ensure(sizeof(int4) * (size_t)std::max(p->nlist, 1LL)));
        STCHK(timed(p, GINT_K_BIN, [&] {
            return launch_DK_desc(p->stream, p->nlist, p->geo.nbatch, p->blist.as<int>(), p->boff.as<int>(),
                                  p->bptr.as<int>(), p->dk_desc.as<int4>());
        }));
        p->dk_gen = p->gen;
    }
    STCHK(timed(p, GINT_K_DK, [&] {
        return launch_DK_pairs(p->stream, p->geo, bn, B, W_dev, p->dV, p->npair_owned, p->porder(),
                               p->pown.as<int>(), p->plist.as<int>(), p->lptr.as<int>(), p->dk_desc.as<int4>(),
                               p->norb, DK_dev);
    }));
    return GINT_OK;
}

gint_status gint_build_rho(gint_plan p, const double *D_dev, double *rho_dev)
{
    STCHK(check_plan(p));
    if (!D_dev || !rho_dev)
        return fail(GINT_EINVAL, "D and rho must be non-NULL device pointers");
    HIPCHK(hipSetDevice(p->device));
    const Bins bn = p->bins();
    const Basis B = p->basis();
    STCHK(timed(p, GINT_K_PACK, [&] {
        return launch_pack_S2(p->stream, p->f32(), p->geo, bn, B, (int)p->npair, D_dev, p->norb, p->S2pk.p);
    }));
    STCHK(timed(p, GINT_K_RHO,
                [&] { return launch_rho_batch(p->stream, p->f32(), p->geo, bn, B, p->nbmax, p->S2pk.p, rho_dev); }));
    return GINT_OK;
}

// st: the stream the pass runs on (the plan's, or the second stream of
// gint_H_rho_force)
static gint_status force_impl(gint_plan p, const double *W, double wscale, const double *D, double *dEdR,
                              double *rho = nullptr, hipStream_t st = nullptr)
{
    STCHK(check_plan(p));
    if (!W || !D || !dEdR)
        return fail(GINT_EINVAL, "W, D and dEdR must be non-NULL device pointers");
    HIPCHK(hipSetDevice(p->device));
    if (!st)
        st = p->stream;
    const Bins bn = p->bins();
    const Basis B = p->basis();
    // FP16 hi/lo: T on FP16 matrix cores, as in the fused pass (the same bits)
    const bool h16 = p->prec == GINT_FP16_SPLIT && force_h16_fits(p->geo.P, p->nbmax, p->mno);
    STCHK(timed_on(p, st, GINT_K_PACK, [&] {
        return h16 ? launch_pack_S2_h16(st, p->geo, bn, B, (int)p->npair, D, p->norb, p->S2pk.p)
                   : launch_pack_S2(st, p->f32(), p->geo, bn, B, (int)p->npair, D, p->norb, p->S2pk.p);
    }));
    STCHK(timed_on(p, st, rho ? GINT_K_RHO_FORCE : GINT_K_FORCE, [&] {
        return launch_force_batch(st, p->f32(), p->geo, bn, B, p->nbmax, p->mno, p->S2pk.p, W, wscale,
                                  p->Fent.as<double>(), rho, h16);
    }));
    STCHK(timed_on(p, st, GINT_K_F_REDUCE, [&] {
        return launch_force_reduce(st, p->natom, p->aptr.as<int>(), p->aent.as<int>(), p->perm.as<int>(),
                                   p->Fent.as<double>(), dEdR);
    }));
    return GINT_OK;
}

gint_status gint_force(gint_plan p, const double *W_dev, const double *D_dev, double *dEdR_dev)
{
    STCHK(check_plan(p));
    return force_impl(p, W_dev, p->dV, D_dev, dEdR_dev);
}

gint_status gint_force_weighted(gint_plan p, const double *w_dev, const double *D_dev, double *dEdR_dev)
{
    return force_impl(p, w_dev, 1.0, D_dev, dEdR_dev);
}

gint_status gint_rho_force(gint_plan p, const double *W_dev, const double *D_dev, double *rho_dev, double *dEdR_dev)
{
    STCHK(check_plan(p));
    if (!rho_dev)
        return fail(GINT_EINVAL, "rho must be a non-NULL device pointer");
    return force_impl(p, W_dev, p->dV, D_dev, dEdR_dev, rho_dev);
}

}  // extern "C"

namespace {
// H, rho and the force of one cell: the fused pass when a batch fits it;
// otherwise H and the rho + force pass on a second stream of the plan
// (two_streams) or one after the other on the plan's stream.
gint_status H_rho_force_impl(gint_plan p, const double *V_dev, const double *D_dev, double *H_dev, double *rho_dev,
                             double *dEdR_dev, bool two_streams)
{
    if (H_rho_force_fits((int)p->prec, p->geo.P, p->nbmax, p->mno)) {
        // one pass per H slab evaluates each batch's orbital tiles once for
        // the H blocks, rho and the force partials
        const Bins bn = p->bins();
        const Basis B = p->basis();
        const hipStream_t st = p->stream;
        STCHK(timed(p, GINT_K_H_FILL,
                    [&] { return launch_fill_f64(st, H_dev, (long long)p->norb * p->norb, 0.0); }));
        // FP16 hi/lo: the fused pass's T runs on FP16 matrix cores as well
        STCHK(timed(p, GINT_K_PACK, [&] {
            return p->prec == GINT_FP16_SPLIT
                       ? launch_pack_S2_h16(st, p->geo, bn, B, (int)p->npair, D_dev, p->norb, p->S2pk.p)
                       : launch_pack_S2(st, p->f32(), p->geo, bn, B, (int)p->npair, D_dev, p->norb, p->S2pk.p);
        }));
        for (size_t i = 0; i + 1 < p->slab.size(); ++i) {
            const int b0 = p->slab[i], b1 = p->slab[i + 1];
            STCHK(timed(p, GINT_K_H_RHO_FORCE, [&] {
                return launch_H_rho_force(st, (int)p->prec, p->geo, bn, B, p->nbmax, p->mno, p->S2pk.p, V_dev, p->dV,
                                          p->Fent.as<double>(), rho_dev, b0, b1, p->boff.as<int>(), p->hpart());
            }));
            STCHK(timed(p, GINT_K_H_REDUCE, [&] {
                return launch_H_pairreduce(st, p->f32(), p->npair_owned, p->porder(), p->pown.as<int>(),
                                           p->plist.as<int>(), p->lsl.as<int>(), (int)p->slab.size() - 1, (int)i,
                                           p->blist.as<int>(), B, p->mno, p->norb, p->hpart(), p->slab_q[i],
                                           i > 0 ? 1 : 0, H_dev);
            }));
        }
        STCHK(timed(p, GINT_K_F_REDUCE, [&] {
            return launch_force_reduce(st, p->natom, p->aptr.as<int>(), p->aent.as<int>(), p->perm.as<int>(),
                                       p->Fent.as<double>(), dEdR_dev);
        }));
        return GINT_OK;
    }
    if (!two_streams) {
        STCHK(build_H_impl(p, V_dev, p->dV, H_dev));
        return force_impl(p, V_dev, p->dV, D_dev, dEdR_dev, rho_dev);
    }
    // batches too large for the fused pass: H beside the rho + force pass on
    // a second stream
    if (!p->aux) {
        // default priority, like every stream of the library
        HIPCHK(hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
    }
    // fork: rho and the force on the second stream, H on the plan's stream;
    // join: the plan's stream waits for both
    HIPCHK(hipEventRecord(p->ev_fork, p->stream));
    HIPCHK(hipStreamWaitEvent(p->aux, p->ev_fork, 0));
    STCHK(force_impl(p, V_dev, p->dV, D_dev, dEdR_dev, rho_dev, p->aux));
    STCHK(build_H_impl(p, V_dev, p->dV, H_dev));
    HIPCHK(hipEventRecord(p->ev_join, p->aux));
    HIPCHK(hipStreamWaitEvent(p->stream, p->ev_join, 0));
    return GINT_OK;
}
}  // namespace

extern "C" {

gint_status gint_H_rho_force(gint_plan p, const double *V_dev, const double *D_dev, double *H_dev, double *rho_dev,
                             double *dEdR_dev)
{
    STCHK(check_plan(p));
    if (!V_dev || !D_dev || !H_dev || !rho_dev || !dEdR_dev)
        return fail(GINT_EINVAL, "V, D, H, rho and dEdR must be non-NULL device pointers");
    HIPCHK(hipSetDevice(p->device));
    return H_rho_force_impl(p, V_dev, D_dev, H_dev, rho_dev, dEdR_dev, true);
}

}  // extern "C"

namespace {
constexpr int kMaxHRExt = kHRBox;  // |n_k| of the lattice vectors of the H(R) / rho(R) calls

// per-image atoms, wrap shifts and the most images in one batch, once per
// list generation
gint_status hr_images(gint_plan p)
{
    if (p->hr_gen == p->gen)
        return GINT_OK;
    const hipStream_t st = p->stream;
    const long long nb = p->geo.nbatch;
    STCHK(p->img_atom.ensure(sizeof(int) * (size_t)(p->nimg + 1)));
    STCHK(p->wsh.ensure(sizeof(int) * 3 * (size_t)p->natom));
    HIPCHK(launch_HR_prep(st, p->geo, p->nent, p->ent_atom.as<int>(), p->ent_img.as<int>(), p->img_atom.as<int>(),
                          p->perm.as<int>(), p->pos_in.as<double>(), p->xw.as<double>(), p->wsh.as<int>()));
    STCHK(p->maxv.ensure(2 * sizeof(int)));
    HIPCHK(launch_max_i32(st, p->cnt_i.as<int>(), nb, p->maxv.as<int>()));
    int most = 0;
    STCHK(read_scalar(p, p->maxv.as<int>(), &most));
    p->nbmax_img = most;
    p->hr_gen = p->gen;
    return GINT_OK;
}

// when the block partials of the unfolded images fit the partial-buffer
// budget, the sorted canonical triples of the fixed-order H(R) reduction,
// once per list generation
// per-batch block offsets of the unfolded images (once per geometry)
gint_status hr_blocks(gint_plan p)
{
    STCHK(hr_images(p));
    if (p->hblk_gen == p->gen)
        return GINT_OK;
    const hipStream_t st = p->stream;
    const long long nb = p->geo.nbatch;
    STCHK(p->img_id.ensure(sizeof(int) * (size_t)(p->nimg + 1)));
    HIPCHK(launch_iota(st, p->nimg + 1, p->img_id.as<int>()));
    STCHK(p->cnt_u.ensure(sizeof(int) * nb));
    STCHK(p->boff_u.ensure(sizeof(int) * (nb + 1)));
    HIPCHK(launch_block_count(st, (int)nb, p->iptr.as<int>(), p->cnt_u.as<int>()));
    STCHK(scan_i32(p, st, p->cnt_u.as<int>(), nb, p->boff_u.as<int>()));
    int nbu = 0;
    STCHK(read_scalar(p, p->boff_u.as<int>() + nb, &nbu));
    if (nbu < 0)
        return fail(GINT_EUNSUPPORTED, "H(R) block lists exceed 2^31 entries");
    p->nblock_u = nbu;
    p->hblk_gen = p->gen;
    return GINT_OK;
}

// canonical (I, J, R) triple of every unfolded block, sorted, and the runs
// of equal triples (once per geometry); GINT_EUNSUPPORTED when an image
// pair spans more than kHRBox cells along an axis
gint_status hr_triples(gint_plan p)
{
    STCHK(hr_blocks(p));
    if (p->htri_gen == p->gen) {
        if (p->htri_bad)
            return fail(GINT_EUNSUPPORTED, "an atom-image pair spans more than %d cells along an axis", kHRBox);
        return GINT_OK;
    }
    const hipStream_t st = p->stream;
    const long long nb = p->geo.nbatch;
    const int nbu = (int)p->nblock_u;
    p->ntri = 0;
    p->htri_bad = false;
    if (nbu > 0) {
        const size_t n = (size_t)nbu;
        STCHK(p->hkey.ensure(sizeof(unsigned long long) * n));
        STCHK(p->hkey2.ensure(sizeof(unsigned long long) * n));
        STCHK(p->hcode.ensure(sizeof(int) * n));
        STCHK(p->hcode2.ensure(sizeof(int) * n));
        STCHK(p->hbad.ensure(sizeof(int)));
        HIPCHK(launch_fill_i32(st, p->hbad.as<int>(), 1, 0));
        HIPCHK(launch_HR_keys(st, (int)nb, p->iptr.as<int>(), p->boff_u.as<int>(), p->img_atom.as<int>(),
                              p->img.as<int>(), p->perm.as<int>(), p->wsh.as<int>(), p->natom,
                              p->hkey.as<unsigned long long>(), p->hcode.as<int>(), p->hbad.as<int>()));
        int bad = 0;
        STCHK(read_scalar(p, p->hbad.as<int>(), &bad));
        if (bad) {
            p->htri_bad = true;
            p->htri_gen = p->gen;
            return fail(GINT_EUNSUPPORTED, "an atom-image pair spans more than %d cells along an axis", kHRBox);
        }
        int end_bit = 18;
        while (end_bit < 64 && ((unsigned long long)p->natom * p->natom) >> (end_bit - 18))
            ++end_bit;
        size_t tb = 0;
        HIPCHK(sort_HR_keys(st, nullptr, tb, p->hkey.as<unsigned long long>(), p->hkey2.as<unsigned long long>(),
                            p->hcode.as<int>(), p->hcode2.as<int>(), nbu, end_bit));
        STCHK(p->sort_tmp.ensure(tb));
        HIPCHK(sort_HR_keys(st, p->sort_tmp.p, tb, p->hkey.as<unsigned long long>(),
                            p->hkey2.as<unsigned long long>(), p->hcode.as<int>(), p->hcode2.as<int>(), nbu,
                            end_bit));
        STCHK(p->hflag.ensure(sizeof(int) * n));
        STCHK(p->hfscan.ensure(sizeof(int) * (n + 1)));
        HIPCHK(launch_seg(st, nbu, p->hkey2.as<unsigned long long>(), p->hflag.as<int>(), nullptr, nullptr, nullptr,
                          false));
        STCHK(scan_i32(p, st, p->hflag.as<int>(), nbu, p->hfscan.as<int>()));
        int ntri = 0;
        STCHK(read_scalar(p, p->hfscan.as<int>() + nbu, &ntri));
        STCHK(p->tstart.ensure(sizeof(int) * ((size_t)ntri + 1)));
        STCHK(p->tkey.ensure(sizeof(unsigned long long) * ((size_t)ntri + 1)));
        HIPCHK(launch_seg(st, nbu, p->hkey2.as<unsigned long long>(), nullptr, p->hfscan.as<int>(),
                          p->tstart.as<int>(), p->tkey.as<unsigned long long>(), true));
        p->ntri = ntri;
        // the triples' reductions heaviest first (block count)
        STCHK(p->tcost.ensure(sizeof(int) * 2 * ((size_t)ntri + 1)));
        STCHK(p->tord.ensure(sizeof(int) * 2 * ((size_t)ntri + 1)));
        size_t tb2 = 0;
        HIPCHK(launch_item_order(st, nullptr, tb2, ntri, 1, 1, nullptr, nullptr, nullptr, nullptr, nullptr));
        STCHK(p->tsort_tmp.ensure(tb2));
        HIPCHK(launch_item_order(st, p->tsort_tmp.p, tb2, ntri, 1, 1, p->tstart.as<int>(), p->tcost.as<int>(),
                                 p->tcost.as<int>() + ntri + 1, p->tord.as<int>(), p->tord.as<int>() + ntri + 1));
    }
    p->htri_gen = p->gen;
    return GINT_OK;
}

gint_status hr_prepare(gint_plan p)
{
    STCHK(hr_images(p));
    if (p->hrfix_gen == p->gen)
        return GINT_OK;
    STCHK(hr_blocks(p));
    const long long nbu = p->nblock_u;
    const size_t esz = p->f32() ? sizeof(float) : sizeof(double);
    const size_t blk_bytes = esz * (size_t)block_pitch(p->mno, (int)esz);
    p->hr_fixed = !p->ext_hpart &&
                  blk_bytes * (size_t)std::max(nbu, 1LL) <= std::max(p->hbudget_eff, p->Hpart.bytes);
    if (p->hr_fixed && nbu > 0) {
        STCHK(hr_triples(p));
        STCHK(p->Hpart.ensure(blk_bytes * (size_t)nbu));
    }
    p->hrfix_gen = p->gen;
    return GINT_OK;
}

// D(R) blocks of the rho / force contractions packed per triple (the
// triples and the triple of every block entry once per geometry, the blocks
// per call).  *ps stays NULL, and the kernels gather D(R) elements instead,
// when the triples are unavailable or gathering is forced.
gint_status hr_pack(gint_plan p, const HRMap &m, const double *DR, PackedS *buf, const PackedS **ps)
{
    *ps = nullptr;
    if (g_dr_gather)
        return GINT_OK;
    const gint_status tst = hr_triples(p);
    if (tst == GINT_EUNSUPPORTED) {
        g_last_error.clear();
        return GINT_OK;
    }
    STCHK(tst);
    if (p->ntri == 0)
        return GINT_OK;
    const hipStream_t st = p->stream;
    if (p->etri_gen != p->gen) {
        STCHK(p->etri.ensure(sizeof(int) * (size_t)p->nblock_u));
        HIPCHK(launch_entry_tri(st, p->nblock_u, p->hcode2.as<int>(), p->hfscan.as<int>(), p->etri.as<int>()));
        p->etri_gen = p->gen;
    }
    STCHK(p->spk.ensure(sizeof(double) * 512 * (size_t)p->ntri));
    STCHK(p->snz.ensure(sizeof(int) * (size_t)p->ntri));
    const Basis B = p->basis();
    STCHK(timed(p, GINT_K_PACK, [&] {
        return launch_S_pack(st, p->ntri, p->tkey.as<unsigned long long>(), p->natom, B.orb0, m, p->norb, DR,
                             p->spk.as<double>(), p->snz.as<int>());
    }));
    *buf = PackedS{p->etri.as<int>(), p->boff_u.as<int>(), p->snz.as<int>(), p->spk.as<double>()};
    *ps = buf;
    return GINT_OK;
}

// Validate a caller's list of lattice vectors and upload its box map (kept
// while the list is unchanged); also checks that the unfolded images of a
// batch fit the LDS of the per-batch kernels.
gint_status hr_map(gint_plan p, int nR, const int *R, HRMap *m)
{
    int ext[3] = {0, 0, 0};
    for (int q = 0; q < nR; ++q)
        for (int k = 0; k < 3; ++k) {
            if (R[3 * q + k] < -kMaxHRExt || R[3 * q + k] > kMaxHRExt)
                return fail(GINT_EINVAL, "R[%d] has a component %d outside [-%d, %d]", q, R[3 * q + k], kMaxHRExt,
                            kMaxHRExt);
            ext[k] = std::max(ext[k], std::abs(R[3 * q + k]));
        }
    const size_t nbox = (size_t)(2 * ext[0] + 1) * (2 * ext[1] + 1) * (2 * ext[2] + 1);
    std::vector<int> map(nbox, -1);
    for (int q = 0; q < nR; ++q) {
        const size_t i = ((size_t)(R[3 * q] + ext[0]) * (2 * ext[1] + 1) + R[3 * q + 1] + ext[1]) * (2 * ext[2] + 1) +
                         R[3 * q + 2] + ext[2];
        if (map[i] >= 0)
            return fail(GINT_EINVAL, "R[%d] repeats R[%d]", q, map[i]);
        map[i] = q;
    }
    HIPCHK(hipSetDevice(p->device));
    STCHK(hr_images(p));
    const size_t esz = p->f32() ? sizeof(float) : sizeof(double);
    if (p->nbmax_img > kMaxBatchAtoms || esz * (size_t)p->nbmax_img * p->geo.P * kRow + 16384 > 163840)
        return fail(GINT_EUNSUPPORTED, "%d atom images reach one %d-point batch; use a smaller batch", p->nbmax_img,
                    p->geo.P);
    std::vector<int> key(map);
    key.insert(key.end(), ext, ext + 3);
    if (key != p->hr_key) {
        STCHK(p->rmap.ensure(sizeof(int) * nbox));
        HIPCHK(hipMemcpyAsync(p->rmap.p, map.data(), sizeof(int) * nbox, hipMemcpyHostToDevice, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));  // map (host) outlives the copy
        p->hr_key.swap(key);
    }
    m->rmap = p->rmap.as<int>();
    for (int k = 0; k < 3; ++k)
        m->ext[k] = ext[k];
    return GINT_OK;
}
}  // namespace

extern "C" {

gint_status gint_HR_lattice(gint_plan p, int cap, int *nR, int *R)
{
    STCHK(check_plan(p));
    if (!nR || cap < 0 || (cap > 0 && !R))
        return fail(GINT_EINVAL, "nR must be non-NULL, cap >= 0, and R non-NULL when cap > 0");
    HIPCHK(hipSetDevice(p->device));
    STCHK(hr_images(p));
    const int M = kMaxHRExt, w = 2 * M + 1;
    const size_t nbox = (size_t)w * w * w;
    STCHK(p->rmap.ensure(sizeof(int) * nbox));
    p->hr_key.clear();  // the R map buffer is reused here
    HIPCHK(launch_fill_i32(p->stream, p->rmap.as<int>(), (long long)nbox, 0));
    HIPCHK(launch_HR_mark(p->stream, p->geo, p->iptr.as<int>(), p->img_atom.as<int>(), p->img.as<int>(),
                          p->wsh.as<int>(), M, p->rmap.as<int>()));
    std::vector<int> mark(nbox);
    HIPCHK(hipMemcpyAsync(mark.data(), p->rmap.p, sizeof(int) * nbox, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    int n = 0;
    for (size_t i = 0; i < nbox; ++i)
        if (mark[i]) {
            if (n < cap) {
                R[3 * n] = (int)(i / ((size_t)w * w)) - M;
                R[3 * n + 1] = (int)((i / w) % w) - M;
                R[3 * n + 2] = (int)(i % w) - M;
            }
            ++n;
        }
    *nR = n;
    if (n > cap)
        return fail(GINT_EINVAL, "%d lattice vectors, room for %d (nR holds the count)", n, cap);
    return GINT_OK;
}

gint_status gint_build_HR(gint_plan p, const double *V_dev, int nR, const int *R, double *HR_dev)
{
    STCHK(check_plan(p));
    if (!V_dev || !HR_dev || !R)
        return fail(GINT_EINVAL, "V and HR must be non-NULL device pointers and R a non-NULL host array");
    if (nR < 1)
        return fail(GINT_EINVAL, "nR = %d must be >= 1", nR);
    HRMap m;
    STCHK(hr_map(p, nR, R, &m));
    STCHK(hr_prepare(p));
    const hipStream_t st = p->stream;
    STCHK(timed(p, GINT_K_H_FILL,
                [&] { return launch_fill_f64(st, HR_dev, (long long)nR * p->norb * p->norb, 0.0); }));
    const Basis B = p->basis();
    if (p->hr_fixed) {
        // the Gamma-point H block kernel over the unfolded images (one image
        // per entry), then the fixed-order sums per canonical triple
        Bins bu = p->bins();
        bu.bptr = p->iptr.as<int>();
        bu.ent_atom = p->img_atom.as<int>();
        bu.ent_img = p->img_id.as<int>();
        STCHK(timed(p, GINT_K_H, [&] {
            return launch_H_batch(st, (int)p->prec, p->geo, bu, B, p->nbmax_img, 0, p->geo.nbatch, V_dev, p->dV,
                                  p->boff_u.as<int>(), p->mno, p->Hpart.p);
        }));
        STCHK(timed(p, GINT_K_HR, [&] {
            return launch_HR_reduce(st, p->f32(), p->ntri, p->ntri > 0 ? p->tord.as<int>() + p->ntri + 1 : nullptr,
                                    p->tkey.as<unsigned long long>(), p->tstart.as<int>(),
                                    p->hcode2.as<int>(), p->natom, m, B, p->mno, p->norb, p->Hpart.p, HR_dev);
        }));
        return GINT_OK;
    }
    STCHK(timed(p, GINT_K_HR, [&] {
        return launch_HR_batch(st, p->f32(), p->geo, p->nbmax_img, p->iptr.as<int>(), p->img_atom.as<int>(),
                               p->img.as<int>(), B, p->wsh.as<int>(), V_dev, p->dV, m, p->norb, HR_dev);
    }));
    return GINT_OK;
}

gint_status gint_build_rhoR(gint_plan p, int nR, const int *R, const double *DR_dev, double *rho_dev)
{
    STCHK(check_plan(p));
    if (!DR_dev || !rho_dev || !R)
        return fail(GINT_EINVAL, "DR and rho must be non-NULL device pointers and R a non-NULL host array");
    if (nR < 1)
        return fail(GINT_EINVAL, "nR = %d must be >= 1", nR);
    HRMap m;
    STCHK(hr_map(p, nR, R, &m));
    PackedS buf;
    const PackedS *ps = nullptr;
    STCHK(hr_pack(p, m, DR_dev, &buf, &ps));
    const Basis B = p->basis();
    STCHK(timed(p, GINT_K_RHO, [&] {
        return launch_rhoR_batch(p->stream, p->f32(), p->geo, p->nbmax_img, p->iptr.as<int>(), p->img_atom.as<int>(),
                                 p->img.as<int>(), B, p->wsh.as<int>(), m, p->norb, DR_dev, ps, rho_dev);
    }));
    return GINT_OK;
}

gint_status gint_HR_to_Hk(gint_plan p, int nR, const int *R, const double *HR_dev, int nk, const double *kfrac,
                          double *Hk_dev)
{
    STCHK(check_plan(p));
    if (!R || !kfrac || !HR_dev || !Hk_dev)
        return fail(GINT_EINVAL, "R and kfrac must be non-NULL host arrays, HR and Hk non-NULL device pointers");
    if (nR < 1 || nk < 1)
        return fail(GINT_EINVAL, "nR = %d and nk = %d must be >= 1", nR, nk);
    for (int i = 0; i < 3 * nk; ++i)
        if (!std::isfinite(kfrac[i]))
            return fail(GINT_EINVAL, "kfrac has non-finite entries");
    HIPCHK(hipSetDevice(p->device));
    // phases in FP64 on the host: 2 pi kappa . n reduced to [0, 1) turns first
    std::vector<double> ph((size_t)2 * nk * nR);
    for (int k = 0; k < nk; ++k)
        for (int q = 0; q < nR; ++q) {
            double t = 0.0;
            for (int d = 0; d < 3; ++d)
                t += kfrac[3 * k + d] * (double)R[3 * q + d];
            t -= std::floor(t);
            const double a = 2.0 * M_PI * t;
            ph[2 * ((size_t)k * nR + q)] = std::cos(a);
            ph[2 * ((size_t)k * nR + q) + 1] = std::sin(a);
        }
    STCHK(p->hk_phase.ensure(sizeof(double) * ph.size()));
    HIPCHK(hipMemcpyAsync(p->hk_phase.p, ph.data(), sizeof(double) * ph.size(), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));  // ph (host) outlives the copy on every path
    const long long nel = (long long)p->norb * p->norb;
    STCHK(timed(p, GINT_K_HR, [&] {
        return launch_Hk(p->stream, nel, nR, nk, p->hk_phase.as<double>(), HR_dev, Hk_dev);
    }));
    return GINT_OK;
}

gint_status gint_HR_to_Hk_noalloc(gint_plan p, int nR, const int *R, const double *HR_dev, int nk,
                                  const double *kfrac, double *Hk_dev)
{
    STCHK(check_plan(p));
    if (!R || !kfrac || !HR_dev || !Hk_dev)
        return fail(GINT_EINVAL, "R and kfrac must be non-NULL host arrays, HR and Hk non-NULL device pointers");
    if (nR < 1 || nk < 1)
        return fail(GINT_EINVAL, "nR = %d and nk = %d must be >= 1", nR, nk);
    if (nR > kHkNaMaxR || nk > kHkNaMaxK || (long long)nR * nk > kHkNaMaxPhase)
        return fail(GINT_EINVAL,
                    "gint_HR_to_Hk_noalloc: nR = %d, nk = %d exceed its fixed workspace (nR <= %d, nk <= %d, "
                    "nR * nk <= %d); use gint_HR_to_Hk",
                    nR, nk, kHkNaMaxR, kHkNaMaxK, kHkNaMaxPhase);
    for (int i = 0; i < 3 * nk; ++i)
        if (!std::isfinite(kfrac[i]))
            return fail(GINT_EINVAL, "kfrac has non-finite entries");
    HIPCHK(hipSetDevice(p->device));
    HIPCHK(Hk_noalloc(p->stream, p->device, (long long)p->norb * p->norb, nR, R, nk, kfrac, HR_dev, Hk_dev));
    return GINT_OK;
}

gint_status gint_forceR(gint_plan p, const double *V_dev, int nR, const int *R, const double *DR_dev,
                        double *dEdR_dev)
{
    STCHK(check_plan(p));
    if (!V_dev || !DR_dev || !dEdR_dev || !R)
        return fail(GINT_EINVAL, "V, DR and dEdR must be non-NULL device pointers and R a non-NULL host array");
    if (nR < 1)
        return fail(GINT_EINVAL, "nR = %d must be >= 1", nR);
    HRMap m;
    STCHK(hr_map(p, nR, R, &m));
    STCHK(p->Fimg.ensure(sizeof(double) * 3 * (size_t)(p->nimg + 1)));
    PackedS buf;
    const PackedS *ps = nullptr;
    STCHK(hr_pack(p, m, DR_dev, &buf, &ps));
    const Basis B = p->basis();
    STCHK(timed(p, GINT_K_FORCE, [&] {
        return launch_forceR_batch(p->stream, p->f32(), p->geo, p->nbmax_img, p->iptr.as<int>(),
                                   p->img_atom.as<int>(), p->img.as<int>(), B, p->wsh.as<int>(), m, p->norb, DR_dev,
                                   ps, V_dev, p->dV, p->Fimg.as<double>());
    }));
    STCHK(timed(p, GINT_K_F_REDUCE, [&] {
        return launch_forceR_reduce(p->stream, p->natom, p->aptr.as<int>(), p->aent.as<int>(), p->ent_img.as<int>(),
                                    p->perm.as<int>(), p->Fimg.as<double>(), dEdR_dev);
    }));
    return GINT_OK;
}

gint_status gint_plan_sync(gint_plan p)
{
    STCHK(check_plan(p));
    HIPCHK(hipSetDevice(p->device));
    HIPCHK(hipStreamSynchronize(p->stream));
    HIPCHK(hipGetLastError());
    return GINT_OK;
}

gint_status gint_plan_work(gint_plan p, gint_work *out)
{
    STCHK(check_plan(p));
    if (!out)
        return fail(GINT_EINVAL, "out is NULL");
    HIPCHK(hipSetDevice(p->device));
    const int nblk = 2048;
    STCHK(p->sums.ensure(sizeof(double) * 2 * nblk));
    HIPCHK(launch_support_count(p->stream, p->geo, p->bins(), p->basis(), p->sums.as<double>(), nblk));
    std::vector<double> h(2 * nblk);
    HIPCHK(hipMemcpyAsync(h.data(), p->sums.p, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < nblk; ++i) {
        s1 += h[2 * i];
        s2 += h[2 * i + 1];
    }
    out->ngrid = (long long)p->geo.N[0] * p->geo.N[1] * p->geo.N[2];
    out->nbatch = p->geo.nbatch;
    out->nentry = p->nent;
    out->npair = p->npair;
    out->sum_ng = s1;
    out->sum_ng2 = s2;
    for (int k = 0; k < 3; ++k)
        out->batch[k] = p->geo.bs[k];
    out->nslab = (int)p->slab.size() - 1;
    out->nblock = p->nblock;
    out->mno = p->mno;
    out->partial_bytes = p->f32() ? 4 : 8;
    out->nblock_hr = p->hrfix_gen == p->gen ? p->nblock_u : -1;
    return GINT_OK;
}

gint_status gint_plan_set_timing(gint_plan p, int enable)
{
    STCHK(check_plan(p));
    HIPCHK(hipSetDevice(p->device));
    STCHK(drain_marks(p));
    p->timing = enable != 0;
    for (int k = 0; k < GINT_NKERNEL; ++k) {
        p->timed_ms[k] = 0.0;
        p->timed_n[k] = 0;
    }
    return GINT_OK;
}

gint_status gint_plan_timing(gint_plan p, double *ms, int *launches)
{
    STCHK(check_plan(p));
    if (!ms || !launches)
        return fail(GINT_EINVAL, "ms and launches must be non-NULL");
    HIPCHK(hipSetDevice(p->device));
    STCHK(drain_marks(p));
    for (int k = 0; k < GINT_NKERNEL; ++k) {
        ms[k] = p->timed_ms[k];
        launches[k] = p->timed_n[k];
    }
    return GINT_OK;
}

gint_status gint_plan_atom_order(gint_plan p, int *order)
{
    STCHK(check_plan(p));
    if (!order)
        return fail(GINT_EINVAL, "order is NULL");
    HIPCHK(hipSetDevice(p->device));
    HIPCHK(hipMemcpyAsync(order, p->perm.p, sizeof(int) * p->natom, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return GINT_OK;
}

gint_status gint_test_fail_rebuilds(int n)
{
    if (n < 0)
        return fail(GINT_EINVAL, "n = %d must be >= 0", n);
    g_fail_rebuilds = n;
    return GINT_OK;
}

gint_status gint_test_DR_gather(int on)
{
    g_dr_gather = on ? 1 : 0;
    return GINT_OK;
}

int gint_norb(gint_plan p) { return (p && p->magic == kMagic) ? p->norb : -1; }
int gint_natom(gint_plan p) { return (p && p->magic == kMagic) ? p->natom : -1; }
double gint_dV(gint_plan p) { return (p && p->magic == kMagic) ? p->dV : -1.0; }

void gint_plan_destroy(gint_plan p)
{
    if (!p || p->magic != kMagic)
        return;
    (void)hipSetDevice(p->device);
    (void)hipStreamSynchronize(p->stream);
    p->magic = 0;
    delete p;
}

}  // extern "C"


// ===========================================================================
// Spherical-grid projector overlaps (Sec. 3.3.2): per-plan projector tables,
// quadrature rules and per-geometry neighbour lists; the kernels are in
// gint_sphere.hip.

namespace {
constexpr unsigned kPBMagic = 0x47505342u;  // "GPSB"
}  // namespace

struct gint_psibeta_s {
    unsigned magic = kPBMagic;
    gint_plan plan = nullptr;
    long long gen = -1;  // list generation of the plan the neighbour lists were built for
    int nprad = 0, npa = 0, nproj = 0, nang = 0, nrq = 0;
    int nent = 0;  // neighbour entries over all projector atoms
    int nps = 0;   // most projectors of one species (row stride of the table)
    double rb_max = 0.0;
    std::vector<int> pin_h, prow_h;  // projector atoms (input order) and their first rows
    std::vector<double> prb_h;       // projector cutoff of each projector atom
    std::vector<int> sp_nproj;       // projectors per species
    DevBuf prad, psp, pknots, ps0, psn, pcoef, pscratch, ang, rq;
    DevBuf pint, pin, prow, prb, cnt, ioff, eptr, ent, img;
    DevBuf tab;  // W e^{-iA.r} beta_p at every grid point of every projector atom (per call)
};

namespace {

gint_status check_psibeta(gint_psibeta b)
{
    if (!b)
        return fail(GINT_EINVAL, "psibeta is NULL");
    if (b->magic != kPBMagic)
        return fail(GINT_ESTATE, "psibeta is destroyed or corrupted");
    return check_plan(b->plan);
}

// neighbour lists of the projector atoms for the plan's current positions
gint_status psibeta_lists(gint_psibeta b)
{
    gint_plan p = b->plan;
    if (b->gen == p->gen)
        return GINT_OK;
    const hipStream_t s = p->stream;
    const int natom = p->natom, npa = b->npa;
    if (npa == 0) {
        b->gen = p->gen;
        return GINT_OK;
    }
    std::vector<int> inv(natom);
    HIPCHK(hipMemcpyAsync(inv.data(), p->inv_perm.p, sizeof(int) * natom, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> pint(npa);
    for (int a = 0; a < npa; ++a)
        pint[a] = inv[b->pin_h[a]];
    const Geo &g = p->geo;
    int m[3];
    for (int i = 0; i < 3; ++i) {
        const double bn = std::sqrt(g.rec[3 * i] * g.rec[3 * i] + g.rec[3 * i + 1] * g.rec[3 * i + 1] +
                                    g.rec[3 * i + 2] * g.rec[3 * i + 2]);
        m[i] = (int)std::ceil((b->rb_max + p->rc_max) * bn) + 1;
        if (m[i] > 125)
            return fail(GINT_EUNSUPPORTED, "projector and orbital cutoffs span more than 125 cells");
    }
    const size_t nn = (size_t)npa * natom;
    STCHK(b->pint.ensure(sizeof(int) * npa));
    HIPCHK(hipMemcpyAsync(b->pint.p, pint.data(), sizeof(int) * npa, hipMemcpyHostToDevice, s));
    STCHK(b->cnt.ensure(sizeof(int) * nn));
    const Basis B = p->basis();
    HIPCHK(launch_pb_images(s, g, B, npa, b->pint.as<int>(), b->prb.as<double>(), m, b->cnt.as<int>(), nullptr,
                            nullptr));
    std::vector<int> cnt(nn);
    HIPCHK(hipMemcpyAsync(cnt.data(), b->cnt.p, sizeof(int) * nn, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // image offsets of every (projector atom, atom) pair; entries of the
    // pairs with images, per projector atom in atom (internal) order
    std::vector<int> ioff(nn), ent, eptr(npa + 1);
    long long tot = 0;
    for (int a = 0; a < npa; ++a) {
        eptr[a] = (int)(ent.size() / 4);
        for (int J = 0; J < natom; ++J) {
            const size_t t = (size_t)a * natom + J;
            ioff[t] = (int)tot;
            if (cnt[t] > 0) {
                ent.push_back(J);
                ent.push_back((int)tot);
                ent.push_back(cnt[t]);
                ent.push_back(a);
            }
            tot += cnt[t];
            if (tot >= 0x7fffffffLL)
                return fail(GINT_EUNSUPPORTED, "projector neighbour lists exceed 2^31 images");
        }
    }
    eptr[npa] = (int)(ent.size() / 4);
    b->nent = eptr[npa];
    STCHK(b->ioff.ensure(sizeof(int) * nn));
    STCHK(b->img.ensure(sizeof(int) * (size_t)std::max(tot, 1LL)));
    STCHK(b->ent.ensure(sizeof(int) * std::max(ent.size(), (size_t)4)));
    STCHK(b->eptr.ensure(sizeof(int) * (npa + 1)));
    HIPCHK(hipMemcpyAsync(b->ioff.p, ioff.data(), sizeof(int) * nn, hipMemcpyHostToDevice, s));
    if (!ent.empty())
        HIPCHK(hipMemcpyAsync(b->ent.p, ent.data(), sizeof(int) * ent.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(b->eptr.p, eptr.data(), sizeof(int) * (npa + 1), hipMemcpyHostToDevice, s));
    HIPCHK(launch_pb_images(s, g, B, npa, b->pint.as<int>(), b->prb.as<double>(), m, b->cnt.as<int>(),
                            b->ioff.as<int>(), b->img.as<int>()));
    HIPCHK(hipStreamSynchronize(s));  // the host tables outlive the copies
    b->gen = p->gen;
    return GINT_OK;
}

}  // namespace

extern "C" {

gint_status gint_psibeta_create(gint_plan p, int nspecies, const gint_species *proj, int nang, const double *ang,
                                int nrq, const double *rq, gint_psibeta *out)
{
    STCHK(check_plan(p));
    if (!out)
        return fail(GINT_EINVAL, "out is NULL");
    if (nspecies != p->nspecies || !proj)
        return fail(GINT_EINVAL, "projectors must be given for each of the plan's %d species", p->nspecies);
    if (nang < 1 || nang > 65536 || !ang || nrq < 1 || nrq > 65536 || !rq)
        return fail(GINT_EINVAL, "need 1..65536 angular and radial quadrature nodes (non-NULL)");
    if ((long long)nang * nrq >= 0x7fffffffLL)
        return fail(GINT_EINVAL, "quadrature grid of %lld points is too large", (long long)nang * nrq);
    if (!finite3(ang, 4LL * nang) || !finite3(rq, 2LL * nrq))
        return fail(GINT_EINVAL, "quadrature rules have non-finite entries");
    for (int i = 0; i < nrq; ++i)
        if (rq[2 * i] < 0.0 || rq[2 * i] > 1.0)
            return fail(GINT_EINVAL, "radial node %d = %g is outside [0, 1]", i, rq[2 * i]);
    int nrad_total = 0;
    for (int s = 0; s < nspecies; ++s) {
        const gint_species &S = proj[s];
        if (S.nradial < 0 || (S.nradial > 0 && !S.radial))
            return fail(GINT_EINVAL, "projector species %d: bad radial list", s);
        nrad_total += S.nradial;
        int np = 0;
        for (int k = 0; k < S.nradial; ++k) {
            const gint_radial &R = S.radial[k];
            if (R.l < 0 || R.l > 2)
                return fail(R.l < 0 ? GINT_EINVAL : GINT_EUNSUPPORTED, "projector %d of species %d: l = %d", k, s,
                            R.l);
            if (R.nr < 4 || !(R.dr > 0.0) || !std::isfinite(R.dr) || !R.f)
                return fail(GINT_EINVAL, "projector %d of species %d: bad table", k, s);
            if (!finite3(R.f, R.nr) || !std::isfinite(R.dfdr_0) || !std::isfinite(R.dfdr_rc))
                return fail(GINT_EINVAL, "projector %d of species %d: non-finite table", k, s);
            np += 2 * R.l + 1;
        }
        if (np > kMaxOrb)
            return fail(GINT_EUNSUPPORTED, "species %d has %d projectors (max %d)", s, np, kMaxOrb);
    }
    if (nrad_total > kMaxRadTotal)
        return fail(GINT_EUNSUPPORTED, "%d projector radials (max %d)", nrad_total, kMaxRadTotal);
    HIPCHK(hipSetDevice(p->device));
    gint_psibeta b = new (std::nothrow) gint_psibeta_s;
    if (!b)
        return fail(GINT_ENOMEM, "host allocation failed");
    b->plan = p;
    b->nang = nang;
    b->nrq = nrq;
    // projector tables, ordered like the orbitals (l ascending, stable; m)
    std::vector<DevRadial> rad;
    std::vector<DevSpecies> sp(nspecies);
    std::vector<double> knots, s0, sn;
    int coef_off = 0;
    b->sp_nproj.assign(nspecies, 0);
    for (int s = 0; s < nspecies; ++s) {
        const gint_species &S = proj[s];
        sp[s].rad0 = (int)rad.size();
        sp[s].nrad = S.nradial;
        sp[s].rc = 0.0;
        for (int o = 0; o < kMaxOrb; ++o)
            sp[s].orb_rad[o] = sp[s].orb_m[o] = 0;
        int orb = 0;
        for (int l = 0; l <= 2; ++l)
            for (int k = 0; k < S.nradial; ++k) {
                const gint_radial &R = S.radial[k];
                if (R.l != l)
                    continue;
                DevRadial d;
                for (int m = 0; m < 2 * l + 1; ++m) {
                    sp[s].orb_rad[orb + m] = (signed char)rad.size();
                    sp[s].orb_m[orb + m] = (signed char)(m - l);
                }
                d.dr = R.dr;
                d.inv_dr = 1.0 / R.dr;
                d.rc = (R.nr - 1) * R.dr;
                d.l = R.l;
                d.nr = R.nr;
                d.orb0 = orb;
                d.coef_off = coef_off;
                d.knot_off = (int)knots.size();
                coef_off += 4 * (R.nr - 1);
                knots.insert(knots.end(), R.f, R.f + R.nr);
                s0.push_back(R.dfdr_0);
                sn.push_back(R.dfdr_rc);
                rad.push_back(d);
                orb += 2 * l + 1;
                sp[s].rc = std::max(sp[s].rc, d.rc);
            }
        sp[s].norb = orb;
        b->sp_nproj[s] = orb;
        b->nps = std::max(b->nps, orb);
        b->rb_max = std::max(b->rb_max, sp[s].rc);
    }
    b->nprad = (int)rad.size();
    // projector atoms (input order) and their rows
    std::vector<int> spc_h(p->natom);
    gint_status st = GINT_OK;
    do {
        hipError_t e = hipMemcpyAsync(spc_h.data(), p->spc_in.p, sizeof(int) * p->natom, hipMemcpyDeviceToHost,
                                      p->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) {
            st = fail(GINT_EDEVICE, "reading the species failed: %s", hipGetErrorString(e));
            break;
        }
        int row = 0;
        for (int i = 0; i < p->natom; ++i) {
            const int np = b->sp_nproj[spc_h[i]];
            if (np == 0)
                continue;
            b->pin_h.push_back(i);
            b->prow_h.push_back(row);
            b->prb_h.push_back(sp[spc_h[i]].rc);
            row += np;
        }
        b->npa = (int)b->pin_h.size();
        b->nproj = row;
        auto upload = [&](DevBuf &d, const void *h, size_t bytes) -> gint_status {
            STCHK(d.ensure(bytes));
            if (bytes)
                HIPCHK(hipMemcpyAsync(d.p, h, bytes, hipMemcpyHostToDevice, p->stream));
            return GINT_OK;
        };
        if ((st = upload(b->psp, sp.data(), sizeof(DevSpecies) * sp.size())) != GINT_OK) break;
        if ((st = upload(b->ang, ang, sizeof(double) * 4 * nang)) != GINT_OK) break;
        if ((st = upload(b->rq, rq, sizeof(double) * 2 * nrq)) != GINT_OK) break;
        if ((st = upload(b->pin, b->pin_h.data(), sizeof(int) * b->npa)) != GINT_OK) break;
        if ((st = upload(b->prow, b->prow_h.data(), sizeof(int) * b->npa)) != GINT_OK) break;
        if ((st = upload(b->prb, b->prb_h.data(), sizeof(double) * b->npa)) != GINT_OK) break;
        if ((st = b->tab.ensure(2 * sizeof(double) * (size_t)b->npa * nang * nrq * (size_t)std::max(b->nps, 1))) !=
            GINT_OK)
            break;
        if (b->nprad > 0) {
            if ((st = upload(b->prad, rad.data(), sizeof(DevRadial) * rad.size())) != GINT_OK) break;
            if ((st = upload(b->pknots, knots.data(), sizeof(double) * knots.size())) != GINT_OK) break;
            if ((st = upload(b->ps0, s0.data(), sizeof(double) * s0.size())) != GINT_OK) break;
            if ((st = upload(b->psn, sn.data(), sizeof(double) * sn.size())) != GINT_OK) break;
            if ((st = b->pcoef.ensure(sizeof(double) * coef_off)) != GINT_OK) break;
            if ((st = b->pscratch.ensure(sizeof(double) * 3 * knots.size())) != GINT_OK) break;
            e = launch_spline(p->stream, b->nprad, b->prad.as<DevRadial>(), b->pknots.as<double>(),
                              b->ps0.as<double>(), b->psn.as<double>(), b->pcoef.as<double>(),
                              b->pscratch.as<double>());
            if (e != hipSuccess) {
                st = fail(GINT_EDEVICE, "projector spline launch failed: %s", hipGetErrorString(e));
                break;
            }
        }
        e = hipStreamSynchronize(p->stream);  // the host tables outlive the copies
        if (e != hipSuccess) {
            st = fail(GINT_EDEVICE, "projector setup failed on the device: %s", hipGetErrorString(e));
            break;
        }
        st = psibeta_lists(b);
    } while (0);
    if (st != GINT_OK) {
        b->magic = 0;
        delete b;
        return st;
    }
    *out = b;
    return GINT_OK;
}

int gint_psibeta_nproj(gint_psibeta b) { return (b && b->magic == kPBMagic) ? b->nproj : -1; }

gint_status gint_psibeta_overlap(gint_psibeta b, const double A[3], double *Q_dev)
{
    STCHK(check_psibeta(b));
    if (!A || !Q_dev)
        return fail(GINT_EINVAL, "A (host) and Q (device) must be non-NULL");
    if (!finite3(A, 3))
        return fail(GINT_EINVAL, "A has non-finite entries");
    gint_plan p = b->plan;
    HIPCHK(hipSetDevice(p->device));
    STCHK(psibeta_lists(b));
    STCHK(timed(p, GINT_K_H_FILL,
                [&] { return launch_fill_f64(p->stream, Q_dev, 2LL * b->nproj * p->norb, 0.0); }));
    STCHK(timed(p, GINT_K_PSIBETA, [&] {
        return launch_psibeta(p->stream, p->geo, p->basis(), b->prad.as<DevRadial>(), b->psp.as<DevSpecies>(),
                              b->pcoef.as<double>(), b->nprad, b->npa, b->pint.as<int>(), b->pin.as<int>(),
                              b->prow.as<int>(), b->ent.as<int4>(), b->nent, b->img.as<int>(),
                              p->pos_in.as<double>(), b->nang, b->ang.as<double>(), b->nrq, b->rq.as<double>(), A,
                              b->nps, b->tab.p, p->norb, Q_dev);
    }));
    return GINT_OK;
}

void gint_psibeta_destroy(gint_psibeta b)
{
    if (!b || b->magic != kPBMagic)
        return;
    if (b->plan && b->plan->magic == kMagic) {
        (void)hipSetDevice(b->plan->device);
        (void)hipStreamSynchronize(b->plan->stream);
    }
    b->magic = 0;
    delete b;
}

}  // extern "C"

// ===========================================================================
// Batched cells: one plan per cell; every call on the batch is captured once
// into a hipGraph made of kChains concurrent chains (cells assigned longest
// first to the least loaded chain, each chain with its own H partial buffer)
// and replayed with a single hipGraphLaunch while the geometry and the
// caller's pointers stay the same.

namespace {
constexpr unsigned kBatchMagic = 0x47424154u;  // "GBAT"
constexpr int kChains = 4;                     // one per hardware queue of the process

struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> sig;
    std::vector<long long> gens;
};
}  // namespace

struct gint_batch_s {
    unsigned magic = kBatchMagic;
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<gint_plan> plans;
    std::vector<int> chain_of;
    std::vector<int> order;  // cells by decreasing cost
    hipStream_t cap = nullptr;  // private origin stream of the captures
    hipStream_t chains[kChains] = {};
    hipEvent_t fork = nullptr, join[kChains] = {};
    DevBuf hpart[kChains];
    GraphSlot gH, gR, gF, gHRF;

    ~gint_batch_s()
    {
        for (GraphSlot *g : {&gH, &gR, &gF, &gHRF})
            if (g->exec)
                (void)hipGraphExecDestroy(g->exec);
        for (auto p : plans)
            gint_plan_destroy(p);
        for (int c = 0; c < kChains; ++c) {
            if (join[c])
                (void)hipEventDestroy(join[c]);
            if (chains[c])
                (void)hipStreamDestroy(chains[c]);
        }
        if (fork)
            (void)hipEventDestroy(fork);
        if (cap)
            (void)hipStreamDestroy(cap);
    }
};

namespace {

gint_status check_batch(gint_batch b)
{
    if (!b)
        return fail(GINT_EINVAL, "batch is NULL");
    if (b->magic != kBatchMagic)
        return fail(GINT_ESTATE, "batch is destroyed or corrupted");
    return GINT_OK;
}

// Capture `body` (which enqueues every cell's work on its chain stream) into
// the slot's graph unless the pointers and geometries are unchanged, then
// launch the graph on the batch stream.
template <typename F>
gint_status run_graph(gint_batch b, GraphSlot &slot, const std::vector<const void *> &sig, F body)
{
    std::vector<long long> gens;
    for (auto p : b->plans)
        gens.push_back(p->gen);
    if (!slot.exec || slot.sig != sig || slot.gens != gens) {
        if (slot.exec) {
            (void)hipGraphExecDestroy(slot.exec);
            slot.exec = nullptr;
        }
        for (auto p : b->plans)
            if (p->timing)
                return fail(GINT_ESTATE, "disable per-kernel timing on the cells before batched calls");
        // during the capture every cell runs on its chain's stream
        std::vector<hipStream_t> own(b->plans.size());
        for (size_t i = 0; i < b->plans.size(); ++i) {
            own[i] = b->plans[i]->stream;
            b->plans[i]->stream = b->chains[b->chain_of[i]];
        }
        struct Restore {
            gint_batch b;
            std::vector<hipStream_t> &own;
            ~Restore()
            {
                for (size_t i = 0; i < b->plans.size(); ++i)
                    b->plans[i]->stream = own[i];
            }
        } restore{b, own};
        HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        gint_status st = GINT_OK;
        hipError_t e = hipEventRecord(b->fork, b->cap);
        for (int c = 0; c < kChains && e == hipSuccess; ++c)
            e = hipStreamWaitEvent(b->chains[c], b->fork, 0);
        if (e == hipSuccess)
            st = body();
        for (int c = 0; c < kChains && e == hipSuccess; ++c) {
            e = hipEventRecord(b->join[c], b->chains[c]);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(b->cap, b->join[c], 0);
        }
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
        if (st != GINT_OK) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return fail(GINT_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&slot.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            slot.exec = nullptr;
            return fail(GINT_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
        }
        slot.sig = sig;
        slot.gens = gens;
    }
    HIPCHK(hipGraphLaunch(slot.exec, b->stream));
    return GINT_OK;
}

}  // namespace

extern "C" {

gint_status gint_batch_create(int ncell, const gint_cell *cells, int nspecies, const gint_species *species,
                              gint_precision prec, void *hip_stream, gint_batch *out)
{
    if (!out)
        return fail(GINT_EINVAL, "out is NULL");
    if (ncell < 1 || !cells)
        return fail(GINT_EINVAL, "ncell must be >= 1 and cells non-NULL");
    double rc_max = 0.0;
    STCHK(validate_species(nspecies, species, &rc_max));
    for (int i = 0; i < ncell; ++i) {
        Geo g{};
        STCHK(validate_geometry(cells[i].lattice, cells[i].grid, g));
        if (cells[i].natom < 1 || cells[i].natom > kMaxAtoms || !cells[i].species_of_atom || !cells[i].positions)
            return fail(GINT_EINVAL, "cell %d: invalid atoms", i);
    }
    int dev = 0;
    STCHK(device_ok(&dev));
    gint_batch b = new (std::nothrow) gint_batch_s();
    if (!b)
        return fail(GINT_ENOMEM, "host allocation failed");
    b->device = dev;
    b->stream = (hipStream_t)hip_stream;
    gint_status st = GINT_OK;
    auto bail = [&](gint_status s2) {
        if (b->stream)
            (void)hipStreamSynchronize(b->stream);
        b->magic = 0;
        delete b;
        return s2;
    };
    for (int c = 0; c < kChains; ++c) {
        if (hipStreamCreateWithFlags(&b->chains[c], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->join[c], hipEventDisableTiming) != hipSuccess)
            return bail(fail(GINT_EDEVICE, "stream/event creation failed"));
    }
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        return bail(fail(GINT_EDEVICE, "event creation failed"));
    // per-chain H partial buffers (a chain runs its cells one after the
    // other): at most 8 GiB each and a third of free memory overall
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess)
        return bail(fail(GINT_EDEVICE, "hipMemGetInfo failed"));
    size_t per_chain = std::min((size_t)8 << 30, fr / (3 * kChains));
    for (int c = 0; c < kChains; ++c)
        if ((st = b->hpart[c].ensure(per_chain)) != GINT_OK)
            return bail(st);
    // plans, cost, longest-first assignment to the least loaded chain
    std::vector<double> cost(ncell);
    for (int i = 0; i < ncell; ++i) {
        gint_plan p = nullptr;
        st = plan_create(cells[i].lattice, cells[i].grid, nspecies, species, cells[i].natom, cells[i].species_of_atom,
                         cells[i].positions, prec, b->chains[0], b->hpart[0].p, per_chain, &p);
        if (st != GINT_OK)
            return bail(st);
        b->plans.push_back(p);
        cost[i] = (double)p->nent * p->geo.P * p->nbmax;
    }
    b->order.resize(ncell);
    for (int i = 0; i < ncell; ++i)
        b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    b->chain_of.assign(ncell, 0);
    double load[kChains] = {0};
    for (int i : b->order) {
        int c = 0;
        for (int k = 1; k < kChains; ++k)
            if (load[k] < load[c])
                c = k;
        load[c] += cost[i];
        b->chain_of[i] = c;
        b->plans[i]->stream = b->stream;  // single-cell calls run on the batch's stream
        b->plans[i]->ext_hpart = b->hpart[c].p;
    }
    if (hipDeviceSynchronize() != hipSuccess)
        return bail(fail(GINT_EDEVICE, "batch construction failed on the device"));
    *out = b;
    return GINT_OK;
}

int gint_batch_ncell(gint_batch b) { return check_batch(b) == GINT_OK ? (int)b->plans.size() : -1; }

gint_plan gint_batch_cell(gint_batch b, int i)
{
    if (check_batch(b) != GINT_OK || i < 0 || i >= (int)b->plans.size())
        return nullptr;
    return b->plans[i];
}

gint_status gint_batch_build_H(gint_batch b, const double *const *V_dev, double *const *H_dev)
{
    STCHK(check_batch(b));
    if (!V_dev || !H_dev)
        return fail(GINT_EINVAL, "pointer arrays must be non-NULL");
    const int n = (int)b->plans.size();
    std::vector<const void *> sig;
    for (int i = 0; i < n; ++i) {
        if (!V_dev[i] || !H_dev[i])
            return fail(GINT_EINVAL, "cell %d: NULL device pointer", i);
        sig.push_back(V_dev[i]);
        sig.push_back(H_dev[i]);
    }
    HIPCHK(hipSetDevice(b->device));
    return run_graph(b, b->gH, sig, [&]() -> gint_status {
        for (int i : b->order)
            STCHK(build_H_impl(b->plans[i], V_dev[i], b->plans[i]->dV, H_dev[i]));
        return GINT_OK;
    });
}

gint_status gint_batch_build_rho(gint_batch b, const double *const *D_dev, double *const *rho_dev)
{
    STCHK(check_batch(b));
    if (!D_dev || !rho_dev)
        return fail(GINT_EINVAL, "pointer arrays must be non-NULL");
    const int n = (int)b->plans.size();
    std::vector<const void *> sig;
    for (int i = 0; i < n; ++i) {
        if (!D_dev[i] || !rho_dev[i])
            return fail(GINT_EINVAL, "cell %d: NULL device pointer", i);
        sig.push_back(D_dev[i]);
        sig.push_back(rho_dev[i]);
    }
    HIPCHK(hipSetDevice(b->device));
    return run_graph(b, b->gR, sig, [&]() -> gint_status {
        for (int i : b->order)
            STCHK(gint_build_rho(b->plans[i], D_dev[i], rho_dev[i]));
        return GINT_OK;
    });
}

gint_status gint_batch_force(gint_batch b, const double *const *W_dev, const double *const *D_dev,
                             double *const *dEdR_dev)
{
    STCHK(check_batch(b));
    if (!W_dev || !D_dev || !dEdR_dev)
        return fail(GINT_EINVAL, "pointer arrays must be non-NULL");
    const int n = (int)b->plans.size();
    std::vector<const void *> sig;
    for (int i = 0; i < n; ++i) {
        if (!W_dev[i] || !D_dev[i] || !dEdR_dev[i])
            return fail(GINT_EINVAL, "cell %d: NULL device pointer", i);
        sig.push_back(W_dev[i]);
        sig.push_back(D_dev[i]);
        sig.push_back(dEdR_dev[i]);
    }
    HIPCHK(hipSetDevice(b->device));
    return run_graph(b, b->gF, sig, [&]() -> gint_status {
        for (int i : b->order)
            STCHK(force_impl(b->plans[i], W_dev[i], b->plans[i]->dV, D_dev[i], dEdR_dev[i]));
        return GINT_OK;
    });
}

gint_status gint_batch_H_rho_force(gint_batch b, const double *const *V_dev, const double *const *D_dev,
                                   double *const *H_dev, double *const *rho_dev, double *const *dEdR_dev)
{
    STCHK(check_batch(b));
    if (!V_dev || !D_dev || !H_dev || !rho_dev || !dEdR_dev)
        return fail(GINT_EINVAL, "pointer arrays must be non-NULL");
    const int n = (int)b->plans.size();
    std::vector<const void *> sig;
    for (int i = 0; i < n; ++i) {
        if (!V_dev[i] || !D_dev[i] || !H_dev[i] || !rho_dev[i] || !dEdR_dev[i])
            return fail(GINT_EINVAL, "cell %d: NULL device pointer", i);
        for (const void *q : {(const void *)V_dev[i], (const void *)D_dev[i], (const void *)H_dev[i],
                              (const void *)rho_dev[i], (const void *)dEdR_dev[i]})
            sig.push_back(q);
    }
    HIPCHK(hipSetDevice(b->device));
    return run_graph(b, b->gHRF, sig, [&]() -> gint_status {
        for (int i : b->order)
            STCHK(H_rho_force_impl(b->plans[i], V_dev[i], D_dev[i], H_dev[i], rho_dev[i], dEdR_dev[i], false));
        return GINT_OK;
    });
}

gint_status gint_batch_autotune(gint_batch b, const double *const *V_dev, const double *const *D_dev,
                                double *const *H_dev, double *const *rho_dev, double *const *dEdR_dev, int reps,
                                int *chosen)
{
    STCHK(check_batch(b));
    if (!V_dev || !D_dev || !H_dev || !rho_dev || !dEdR_dev)
        return fail(GINT_EINVAL, "pointer arrays must be non-NULL");
    if (reps < 1)
        return fail(GINT_EINVAL, "reps must be >= 1");
    const int n = (int)b->plans.size();
    for (int i = 0; i < n; ++i)
        if (!V_dev[i] || !D_dev[i] || !H_dev[i] || !rho_dev[i] || !dEdR_dev[i])
            return fail(GINT_EINVAL, "cell %d: NULL device pointer", i);
    HIPCHK(hipSetDevice(b->device));
    // candidate batch shapes: 32-point boxes first, then 16-point ones
    static const int cand[][3] = {{4, 4, 2}, {4, 2, 4}, {2, 4, 4}, {8, 2, 2}, {2, 2, 8}, {2, 2, 4}, {4, 2, 2}};
    const int ncand = (int)(sizeof(cand) / sizeof(cand[0]));
    hipEvent_t ev[2];
    HIPCHK(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return fail(GINT_EDEVICE, "event creation failed");
    }
    gint_status st = GINT_OK;
    std::vector<int> done(n, 0);
    for (int i0 = 0; i0 < n && st == GINT_OK; ++i0) {
        if (done[i0])
            continue;
        gint_plan p = b->plans[i0];
        // every cell with the same mesh and atom count takes i0's choice
        std::vector<int> cls;
        for (int i = i0; i < n; ++i) {
            gint_plan q = b->plans[i];
            if (!done[i] && q->natom == p->natom && q->geo.N[0] == p->geo.N[0] && q->geo.N[1] == p->geo.N[1] &&
                q->geo.N[2] == p->geo.N[2])
                cls.push_back(i);
        }
        const hipStream_t own = p->stream;
        p->stream = b->stream;
        float best = 0.0f;
        int bi = -1;
        for (int c = 0; c < ncand && st == GINT_OK; ++c) {
            const int P = cand[c][0] * cand[c][1] * cand[c][2];
            if (P != 32 && p->prec != GINT_FP64 && p->prec != GINT_FP32)
                continue;
            if (gint_plan_tune(p, cand[c], 0) != GINT_OK)
                continue;  // e.g. too many atoms reach one batch of this shape
            auto run = [&]() -> gint_status {
                STCHK(build_H_impl(p, V_dev[i0], p->dV, H_dev[i0]));
                STCHK(gint_build_rho(p, D_dev[i0], rho_dev[i0]));
                return force_impl(p, V_dev[i0], p->dV, D_dev[i0], dEdR_dev[i0]);
            };
            if ((st = run()) != GINT_OK)
                break;
            float ms = 0.0f;
            if (hipEventRecord(ev[0], b->stream) != hipSuccess) {
                st = fail(GINT_EDEVICE, "hipEventRecord failed");
                break;
            }
            for (int r = 0; r < reps && st == GINT_OK; ++r)
                st = run();
            if (st != GINT_OK)
                break;
            if (hipEventRecord(ev[1], b->stream) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
                st = fail(GINT_EDEVICE, "event timing failed");
                break;
            }
            if (bi < 0 || ms < best) {
                best = ms;
                bi = c;
            }
        }
        p->stream = own;
        if (st == GINT_OK && bi < 0)
            st = fail(GINT_EUNSUPPORTED, "cell %d: no candidate batch shape fits", i0);
        for (int i : cls) {
            if (st != GINT_OK)
                break;
            st = gint_plan_tune(b->plans[i], cand[bi], 0);
            done[i] = 1;
            if (chosen)
                for (int k = 0; k < 3; ++k)
                    chosen[3 * i + k] = cand[bi][k];
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return st;
}

gint_status gint_batch_sync(gint_batch b)
{
    STCHK(check_batch(b));
    HIPCHK(hipSetDevice(b->device));
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipGetLastError());
    return GINT_OK;
}

void gint_batch_destroy(gint_batch b)
{
    if (!b || b->magic != kBatchMagic)
        return;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    (void)hipDeviceSynchronize();
    b->magic = 0;
    delete b;
}

}  // extern "C"
