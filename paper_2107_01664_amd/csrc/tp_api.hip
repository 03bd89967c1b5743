// C-ABI of libtpsurf: validation, resident problem state and the host orchestration of
// the hot path (energy, differential, fractional apply, preconditioner, descent step).
#include "tp_solver.h"
#include "tp_sobolev.h"
#include "tp_obstacle.h"
#include "tp_tree.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

namespace tp {

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

static tp_status fail(tp_status st, const std::string& msg)
{
    set_error(msg);
    return st;
}

// ------------------------------------------------------------------ device info

const DeviceInfo& device_info()
{
    static std::mutex mu;
    static DeviceInfo info[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    std::lock_guard<std::mutex> lk(mu);
    DeviceInfo& d = info[dev];
    if (d.device < 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            d.num_cu = prop.multiProcessorCount;
            d.max_threads_per_cu = prop.maxThreadsPerMultiProcessor;
        } else {
            d.num_cu = 256;
            d.max_threads_per_cu = 2048;
        }
        d.device = dev;
    }
    return d;
}

// ------------------------------------------------------------------ kernel timing

// Per-launch durations of the all-pairs kernels, from HIP events recorded on the launch
// stream.  A launch's pair of events is kept pending and resolved only when the figures are
// read or reset, so that measuring never makes the host wait for the GPU.
struct Profiler {
    struct Pending {
        hipEvent_t a, b;
        int device, kind;
        double pairs, cols;
    };
    struct Spare {
        hipEvent_t a, b;
        int device;
    };
    std::mutex mu;
    bool on = false;
    tp_kernel_stats st[4];
    std::vector<Pending> pending;
    std::vector<Spare> spare;   // resolved pairs of events, for reuse on their device

    // Adds the finished launches to the figures (all of them, waiting, when wait is set)
    // and keeps their events for reuse.  Called with mu held.
    void resolve(bool wait)
    {
        size_t keep = 0;
        for (size_t i = 0; i < pending.size(); ++i) {
            Pending& p = pending[i];
            const hipError_t q = wait ? hipEventSynchronize(p.b) : hipEventQuery(p.b);
            if (q == hipErrorNotReady) {
                pending[keep++] = p;
                continue;
            }
            float ms = 0.f;
            if (q == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                st[p.kind].ms_total += ms;
                st[p.kind].pairs_total += p.pairs;
                st[p.kind].cols_total += p.cols;
                st[p.kind].launches += 1;
            }
            if (spare.size() < 1024) {
                spare.push_back({p.a, p.b, p.device});
            } else {
                (void)hipEventDestroy(p.a);
                (void)hipEventDestroy(p.b);
            }
        }
        pending.resize(keep);
        (void)hipGetLastError();
    }
};
constexpr int kKindSobolev = 3;   // profile slot of the inner-product operator's pair kernel
static Profiler g_prof;

struct PairTimer {
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false, stopped = false;
    int device = 0, kind = 0;
    double pairs = 0, cols = 0;
    hipStream_t s = nullptr;
    PairTimer(int kind_, double pairs_, double cols_, hipStream_t s_) : kind(kind_), pairs(pairs_), cols(cols_), s(s_)
    {
        {
            std::lock_guard<std::mutex> lk(g_prof.mu);
            on = g_prof.on && hipGetDevice(&device) == hipSuccess;
            for (size_t i = g_prof.spare.size(); on && i-- > 0;)
                if (g_prof.spare[i].device == device) {
                    a = g_prof.spare[i].a;
                    b = g_prof.spare[i].b;
                    g_prof.spare[i] = g_prof.spare.back();
                    g_prof.spare.pop_back();
                    break;
                }
        }
        if (on) {
            if (!a && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)) on = false;
            else (void)hipEventRecord(a, s);
        }
    }
    void stop()
    {
        if (!on) return;
        stopped = hipEventRecord(b, s) == hipSuccess;
    }
    ~PairTimer()
    {
        if (on && stopped) {
            std::lock_guard<std::mutex> lk(g_prof.mu);
            g_prof.pending.push_back({a, b, device, kind, pairs, cols});
            if (g_prof.pending.size() >= 256) g_prof.resolve(false);
            return;
        }
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// ------------------------------------------------------------------ device buffers
//
// Device memory comes from the allocator registered with tp_set_allocator (for example
// the caller's caching allocator) or, when none is registered, from hipMalloc.  Each
// buffer keeps the free function that matches its allocation.

struct AllocatorState {
    std::mutex mu;
    tp_alloc_fn alloc = nullptr;
    tp_free_fn free_ = nullptr;
    void* user = nullptr;
    int64_t live = 0;     // buffers allocated through the registered allocator and not freed
};
static AllocatorState g_alloc;

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    tp_free_fn fr = nullptr;     // free function of the registered allocator (null: hipFree)
    void* fr_user = nullptr;
    hipStream_t fr_stream = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) {
            if (fr) {
                fr(p, n * sizeof(T), fr_stream, fr_user);
                std::lock_guard<std::mutex> lk(g_alloc.mu);
                --g_alloc.live;
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        n = 0;
        fr = nullptr;
        fr_user = nullptr;
    }
    size_t bytes() const { return n * sizeof(T); }
    void swap(DevBuf& o)
    {
        std::swap(p, o.p);
        std::swap(n, o.n);
        std::swap(fr, o.fr);
        std::swap(fr_user, o.fr_user);
        std::swap(fr_stream, o.fr_stream);
    }
    // Grow to at least cnt elements (contents are not preserved).
    tp_status ensure(size_t cnt, hipStream_t s)
    {
        if (cnt <= n && p) return TP_OK;
        if (p) {
            if (hipStreamSynchronize(s) != hipSuccess) return fail(TP_E_DEVICE, "stream sync failed");
            release();
        }
        const size_t want = std::max<size_t>(cnt, 1);
        const size_t bytes = want * sizeof(T);
        tp_alloc_fn a = nullptr;
        tp_free_fn f = nullptr;
        void* u = nullptr;
        {
            // the registered functions are called without the lock held: they may run
            // arbitrary caller code (which may free other buffers of the library)
            std::lock_guard<std::mutex> lk(g_alloc.mu);
            a = g_alloc.alloc;
            f = g_alloc.free_;
            u = g_alloc.user;
            if (a) ++g_alloc.live;
        }
        if (a) {
            void* q = a(bytes, s, u);
            if (!q) {
                std::lock_guard<std::mutex> lk(g_alloc.mu);
                --g_alloc.live;
                return fail(TP_E_OUT_OF_MEMORY, "the registered allocator returned NULL for " + std::to_string(bytes) + " bytes");
            }
            p = static_cast<T*>(q);
            fr = f;
            fr_user = u;
            fr_stream = s;
        } else if (hipMalloc((void**)&p, bytes) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(TP_E_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        n = want;
        return TP_OK;
    }
};

// Pinned host memory (hipHostMalloc), for scalars read back after a stream sync.
template <class T>
struct HostBuf {
    T* p = nullptr;
    size_t n = 0;
    HostBuf() = default;
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
    ~HostBuf() { release(); }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    // Grow to at least cnt elements (zeroed); the caller makes sure no copy still uses it.
    tp_status ensure(size_t cnt)
    {
        if (cnt <= n && p) return TP_OK;
        release();
        const size_t want = std::max<size_t>(cnt, 1);
        if (hipHostMalloc((void**)&p, want * sizeof(T), hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(TP_E_OUT_OF_MEMORY, "hipHostMalloc of " + std::to_string(want * sizeof(T)) + " bytes failed");
        }
        std::memset((void*)p, 0, want * sizeof(T));
        n = want;
        return TP_OK;
    }
};

// Slots of the per-problem device scalars (P->scal) and their pinned mirror (P->hs).
enum ScalarSlot {
    kSlotE = 0,       // energy (twice the energy after a gradient)
    kSlotArea = 1,
    kSlotVol6 = 2,    // six times the signed volume
    kSlotMax = 3,     // largest vertex displacement of the direction
    kSlotGG = 4,      // g.g per coordinate (3)
    kSlotGX = 7,      // g.x per coordinate (3)
    kSlotS = 10,      // J Y, 2 x 2 entries of 3 coordinates each (12)
    kSlotR = 22,      // J y_g, 2 entries of 3 (6)
    kSlotObs = 28,    // obstacle potential (unweighted)
    kSlotImp = 29,    // implicit obstacles and attractors (weighted)
    kNumSlots = 30
};

// Ring of device tables for the multi-problem CG launches and their pinned staging.
constexpr int kTabSlots = 4;
struct TabRing {
    DevBuf<char> dev;
    HostBuf<char> host;
    size_t slot_bytes = 0;
    hipEvent_t ev[kTabSlots] = {nullptr, nullptr, nullptr, nullptr};
    bool used[kTabSlots] = {false, false, false, false};
    int next = 0;
    TabRing() = default;
    TabRing(const TabRing&) = delete;
    TabRing& operator=(const TabRing&) = delete;
    ~TabRing()
    {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Barnes-Hut tree over a static obstacle's faces (built once, when the obstacle is set).
struct ObsTree {
    DevBuf<double> flo, fhi, fr2, box, na, nsx, nX, nlo, nhi, nr2;
    DevBuf<uint64_t> kin, kout;
    DevBuf<char> tmp;
    DevBuf<int32_t> order, pos;
    DevBuf<unsigned long long> counts;
    BhBuffers view;
    bool built = false;
    size_t bytes() const
    {
        return flo.bytes() + fhi.bytes() + fr2.bytes() + box.bytes() + na.bytes() + nsx.bytes() + nX.bytes() +
               nlo.bytes() + nhi.bytes() + nr2.bytes() + kin.bytes() + kout.bytes() + tmp.bytes() + order.bytes() +
               pos.bytes() + counts.bytes();
    }
    tp_status ensure(int64_t nFo, int leaf, hipStream_t s)
    {
        const int64_t M = (int64_t)bh_node_count(nFo, leaf, nullptr);
        TP_TRY(flo.ensure(3 * nFo, s));
        TP_TRY(fhi.ensure(3 * nFo, s));
        TP_TRY(fr2.ensure(nFo, s));
        TP_TRY(box.ensure(6, s));
        TP_TRY(kin.ensure(nFo, s));
        TP_TRY(kout.ensure(nFo, s));
        const size_t tb = bh_sort_temp_bytes(nFo);
        TP_TRY(tmp.ensure(tb, s));
        TP_TRY(order.ensure(nFo, s));
        TP_TRY(pos.ensure(nFo, s));
        TP_TRY(na.ensure(M, s));
        TP_TRY(nsx.ensure(3 * M, s));
        TP_TRY(nX.ensure(3 * M, s));
        TP_TRY(nlo.ensure(3 * M, s));
        TP_TRY(nhi.ensure(3 * M, s));
        TP_TRY(nr2.ensure(M, s));
        TP_TRY(counts.ensure(2, s));
        BhBuffers& b = view;
        b = BhBuffers();
        b.flo = flo.p; b.fhi = fhi.p; b.fr2 = fr2.p; b.box = box.p; b.keys_in = kin.p; b.keys_out = kout.p;
        b.sort_tmp = tmp.p; b.sort_bytes = tb; b.order = order.p; b.pos = pos.p; b.na = na.p; b.nsx = nsx.p;
        b.nX = nX.p; b.nlo = nlo.p; b.nhi = nhi.p; b.nr2 = nr2.p; b.counts = counts.p;
        return TP_OK;
    }
};

}  // namespace tp

using namespace tp;

// ------------------------------------------------------------------ problem state

struct tp_problem {
    int device = 0;
    hipStream_t stream = nullptr;
    tp_params prm;
    double sigma = 1.0 / 3.0;
    int64_t nV = 0, nF = 0, cap = 0;

    DevBuf<double> V;
    DevBuf<int32_t> F;              // faces in the Morton order of the first mesh's barycenters
    DevBuf<int32_t> face_orig;      // caller's number of each stored face
    FaceData fd;
    DevBuf<float4> fx, fl, fn, tbox;
    DevBuf<double4> dx, dn;
    DevBuf<int> flags;
    bool geom_valid = false;     // fd describes V
    bool cotan_valid = false;    // lap_val describes V (or will, once aux_join is reached)

    // The cotan values, the solvers' matrix and the preconditioner's set-up for new vertex
    // positions can run on a second stream beside the all-pairs work, which does not read
    // them (start_cotan); until the problem's stream has waited for aux_join (join_aux)
    // aux_pending is set, and only calls that leave V and those buffers alone may run.
    hipStream_t aux = nullptr;
    hipEvent_t aux_fork = nullptr, aux_join = nullptr;
    bool aux_pending = false;
    bool setup_used = false;     // a solve needed the set-up since the positions last changed

    // topology (built on first use)
    bool have_vf = false, have_lap = false;
    DevBuf<int32_t> vf_off, vf_idx, tmp_i, tmp_j;
    DevBuf<int32_t> lap_off, lap_col, comp;
    DevBuf<double> lap_val, inv_count;
    // vertex pins: mask, the solver's cotan values with the pinned rows and columns replaced
    // by the identity, and the component weights of the mean-zero projection with the
    // pinned components left out
    DevBuf<int8_t> pin_mask;
    DevBuf<double> lap_pin, inv_count_pin;
    int64_t npins = 0;
    std::vector<int32_t> comp_host;
    DevBuf<int32_t> ell_col;
    DevBuf<double> ell_val;
    int ell_w = 0;

    // two-level Schwarz preconditioner (block order, dense block inverses, coarse inverse)
    bool have_pcg = false;
    PcgSetup pcg;
    DevBuf<int32_t> pcg_perm, pcg_pcol, pcg_bstart, pcg_whole, pcg_blk, pcg_astart, pcg_aob, pcg_acomp,
        pcg_abl_off, pcg_abl;
    DevBuf<int8_t> pcg_rslot, pcg_eslot;
    DevBuf<float> pcg_Binv;
    DevBuf<double> pcg_pval, pcg_phi, pcg_rw, pcg_esum, pcg_C0inv, pcg_Vb, pcg_rho, pcg_red, pcg_bp, pcg_xp;
    // more blocks than one co-resident workgroup each: the multi-launch solve and its work
    bool pcg_ml = false;
    DevBuf<double> ml_r, ml_p, ml_s, ml_m, ml_an, ml_v, ml_shares, ml_g, ml_part;
    DevBuf<char> ml_state;
    HostBuf<char> ml_state_host;
    int64_t nnz = 0;
    int ncomp = 0;
    int last_iters = 0;              // iterations of the problem's last solve (launch grouping)
    int warm_cols = 0;               // > 0: W2 and Y hold the solutions of the last step's two
                                     // Poisson solves with this many columns (warm start)
    bool warm_now = false;           // this step's solves start from them

    double area0 = 0, vol0 = 0, mean_edge = 0;

    // work
    DevBuf<double> part, gface, zbuf, scal, red, vol6, edge;
    // GMRES on A = B + B0: Krylov blocks V, Z, work vectors, small device arrays
    DevBuf<double> gm_V, gm_Z, gm_w, gm_b, gm_r, gm_x, gm_small, gm_red, gm_Q, gm_Qn, gm_AQ, gm_one, gm_dinv,
        gm_sv, gm_sw, gm_smw;
    DevBuf<int32_t> gm_lab0;
    // static obstacle (Sec. 7.3.2): face data of the obstacle mesh, per-face work arrays
    DevBuf<double4> obs_x;
    DevBuf<double> obs_e, obs_g, bm_area, bm_t, imp_e, imp_g;
    ImplicitSet imp;
    int64_t obs_n = 0, obs_cap = 0;
    double obs_p = 6.0, obs_w = 0.0;
    ObsTree obs_tree;               // Barnes-Hut tree of the obstacle (theta > 0)
    DevBuf<char> ub;
    DevBuf<float> symp;             // partial sums of the symmetric fractional apply
    DevBuf<double> cg_Z, cg_p, cg_red, cg_relres;
    DevBuf<unsigned> cg_bar;
    DevBuf<int> cg_iters;
    DevBuf<double> R, Y, W1, W2, gbuf, dir, Vt, Vsave;

    // Barnes-Hut tree and work arrays (params.theta > 0)
    DevBuf<double> bh_nm;   // node moments of the Barnes-Hut fractional apply [2P][kp]
    // block cluster tree (chi > 0): device CSR lists, far-field values [2P][k + 1], the
    // geometry version they describe and their block counts
    DevBuf<int32_t> bct_far_off, bct_far_col, bct_near_off, bct_near_col;
    DevBuf<uint64_t> bct_fr0, bct_fr1, bct_fkeys, bct_nkeys, bct_sorted, bct_grow;
    DevBuf<double> bct_rec;
    DevBuf<char> bct_tmp;
    DevBuf<unsigned long long> bct_cnt;
    HostBuf<unsigned long long> bct_hcnt;
    DevBuf<double> bct_yt;
    int64_t bct_ver = -1, bct_nadm = 0, bct_ninad = 0;
    DevBuf<double> bh_flo, bh_fhi, bh_fr2, bh_box, bh_na, bh_nsx, bh_nX, bh_nlo, bh_nhi, bh_nr2, bh_gS, bh_eS,
        bh_accF, bh_accN;
    DevBuf<uint64_t> bh_kin, bh_kout;
    DevBuf<char> bh_tmp;
    DevBuf<int32_t> bh_order, bh_pos;
    DevBuf<unsigned long long> bh_counts;
    BhBuffers bh;
    const double* fd_V = nullptr;    // vertices the face data currently describe
    uint64_t geom_ver = 0;           // incremented by every face-geometry launch
    uint64_t bh_ver = ~0ull;         // geometry version the tree was built for
    double rho2 = 0.0;               // FP64 near-field radius^2: (2 x mean edge of the first mesh)^2

    // FP64 near-field grid (TP_PREC_FP32_NEAR64), rebuilt per geometry
    DevBuf<uint32_t> ng_kin, ng_kout;
    DevBuf<int32_t> ng_vin, ng_vout;
    DevBuf<float4> ng_sfx, ng_sfl;
    DevBuf<int2> ng_cell;
    DevBuf<char> ng_tmp;
    DevBuf<NearGridParams> ng_prm;
    NearGrid ng;
    uint64_t ng_ver = ~0ull;         // geometry version the grid was built for

    // pinned host mirrors of device scalars, flags and CG results; multi-problem CG tables
    HostBuf<double> hs, hrelres;
    HostBuf<int> hflags, hiters;
    TabRing tab;

    // device memory held by the problem
    size_t device_bytes() const
    {
        size_t b = V.bytes() + F.bytes() + fx.bytes() + fl.bytes() + fn.bytes() + dx.bytes() + dn.bytes() +
                   flags.bytes();
        b += vf_off.bytes() + vf_idx.bytes() + tmp_i.bytes() + tmp_j.bytes() + lap_off.bytes() +
             lap_col.bytes() + comp.bytes() + lap_val.bytes() + inv_count.bytes() + pin_mask.bytes() +
             lap_pin.bytes() + inv_count_pin.bytes() + ell_col.bytes() +
             ell_val.bytes();
        b += pcg_perm.bytes() + pcg_pcol.bytes() + pcg_bstart.bytes() + pcg_whole.bytes() + pcg_blk.bytes() +
             pcg_astart.bytes() + pcg_aob.bytes() + pcg_acomp.bytes() + pcg_abl_off.bytes() + pcg_abl.bytes() +
             pcg_rslot.bytes() + pcg_eslot.bytes() + pcg_phi.bytes() + pcg_rw.bytes() + pcg_esum.bytes() +
             pcg_Binv.bytes() + pcg_pval.bytes() + pcg_C0inv.bytes() + pcg_Vb.bytes() +
             pcg_rho.bytes() + pcg_red.bytes() + pcg_bp.bytes() + pcg_xp.bytes();
        b += gm_V.bytes() + gm_Z.bytes() + gm_w.bytes() + gm_b.bytes() + gm_r.bytes() + gm_x.bytes() +
             gm_small.bytes() + gm_red.bytes() + gm_Q.bytes() + gm_Qn.bytes() + gm_AQ.bytes() + gm_one.bytes() +
             gm_lab0.bytes() + gm_dinv.bytes() + gm_sv.bytes() + gm_sw.bytes() + gm_smw.bytes() + obs_x.bytes() + obs_tree.bytes() +
             obs_e.bytes() + obs_g.bytes() + bm_area.bytes() + bm_t.bytes() + imp_e.bytes() + imp_g.bytes();
        b += ml_r.bytes() + ml_p.bytes() + ml_s.bytes() + ml_m.bytes() + ml_an.bytes() + ml_v.bytes() +
             ml_shares.bytes() + ml_g.bytes() + ml_part.bytes() + ml_state.bytes();
        b += part.bytes() + gface.bytes() + zbuf.bytes() + scal.bytes() + red.bytes() + vol6.bytes() +
             edge.bytes() + ub.bytes() + symp.bytes();
        b += cg_Z.bytes() + cg_p.bytes() + cg_red.bytes() + cg_relres.bytes() + cg_bar.bytes() +
             cg_iters.bytes();
        b += R.bytes() + Y.bytes() + W1.bytes() + W2.bytes() + gbuf.bytes() + dir.bytes() + Vt.bytes() +
             Vsave.bytes() + tab.dev.bytes();
        b += bh_flo.bytes() + bh_fhi.bytes() + bh_fr2.bytes() + bh_box.bytes() + bh_na.bytes() + bh_nsx.bytes() +
             bh_nX.bytes() + bh_nlo.bytes() + bh_nhi.bytes() + bh_nr2.bytes() + bh_gS.bytes() + bh_eS.bytes() +
             bh_accF.bytes() + bh_accN.bytes() + bh_kin.bytes() + bh_kout.bytes() + bh_tmp.bytes() +
             bh_order.bytes() + bh_pos.bytes() + bh_counts.bytes() + bh_nm.bytes() + bct_far_off.bytes() +
             bct_far_col.bytes() + bct_near_off.bytes() + bct_near_col.bytes() + bct_yt.bytes() +
             bct_fr0.bytes() + bct_fr1.bytes() + bct_fkeys.bytes() + bct_nkeys.bytes() + bct_sorted.bytes() +
             bct_grow.bytes() + bct_tmp.bytes() + bct_cnt.bytes() + bct_rec.bytes();
        b += ng_kin.bytes() + ng_kout.bytes() + ng_vin.bytes() + ng_vout.bytes() + ng_sfx.bytes() + ng_sfl.bytes() +
             ng_cell.bytes() + ng_tmp.bytes() + ng_prm.bytes();
        return b;
    }
};

namespace {

// Faces reordered: Fnew[p] = Fold[order[p]], orig[p] = order[p].
__global__ void k_permute_faces(const int32_t* __restrict__ Fold, const int32_t* __restrict__ order, int64_t nF,
                                int32_t* __restrict__ Fnew, int32_t* __restrict__ orig)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nF) return;
    const int32_t s = order[p];
    for (int c = 0; c < 3; ++c) Fnew[3 * p + c] = Fold[3 * (int64_t)s + c];
    orig[p] = s;
}

// Per-face edge-length sums (for the mean edge length of the initial mesh).
__global__ void k_face_edges(const double* __restrict__ V, const int32_t* __restrict__ F, int64_t nF,
                             double* __restrict__ out)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double* a = V + 3 * (int64_t)F[3 * f + c];
        const double* b = V + 3 * (int64_t)F[3 * f + (c + 1) % 3];
        const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
        s += sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
    out[f] = s;
}

tp_status validate_params(const tp_params* in, tp_params& out, double& sigma)
{
    tp_params_default(&out);
    if (in) out = *in;
    if (!(out.alpha > 1.0) || !std::isfinite(out.alpha))
        return fail(TP_E_INVALID_ARGUMENT, "alpha must be a finite number > 1");
    if (!(out.beta > 0.0) || !std::isfinite(out.beta))
        return fail(TP_E_INVALID_ARGUMENT, "beta must be a finite number > 0");
    if (out.precision < 0 || out.precision > 5) return fail(TP_E_INVALID_ARGUMENT, "unknown precision");
    if (!(out.cg_rtol > 0.0)) return fail(TP_E_INVALID_ARGUMENT, "cg_rtol must be > 0");
    if (out.cg_maxiter < 1) return fail(TP_E_INVALID_ARGUMENT, "cg_maxiter must be >= 1");
    if (out.cg_precond != 0 && out.cg_precond != 1) return fail(TP_E_INVALID_ARGUMENT, "cg_precond must be 0 or 1");
    if (!(out.theta >= 0.0) || !std::isfinite(out.theta)) return fail(TP_E_INVALID_ARGUMENT, "theta must be finite and >= 0");
    if (out.leaf_size < 1 || out.leaf_size > 64) return fail(TP_E_INVALID_ARGUMENT, "leaf_size must lie in [1, 64]");
    if (!(out.chi >= 0.0) || !std::isfinite(out.chi)) return fail(TP_E_INVALID_ARGUMENT, "chi must be finite and >= 0");
    if (out.sym_pairs < -1 || out.sym_pairs > 1) return fail(TP_E_INVALID_ARGUMENT, "sym_pairs must be -1, 0 or 1");
    if (out.sym_band < 0) return fail(TP_E_INVALID_ARGUMENT, "sym_band must be >= 0");
    sigma = out.sigma;
    if (sigma < 0.0) {
        const double s = (out.beta - 2.0) / out.alpha;   // s = 2 - 2/p when beta = 2 alpha
        sigma = 2.0 - s;
    }
    if (!(sigma > 0.0 && sigma < 1.0))
        return fail(TP_E_INVALID_ARGUMENT, "sigma must lie in (0, 1) (fractional order 2 sigma in (0, 2))");
    return TP_OK;
}

tp_status check_flags(tp_problem* P)
{
    int h[kNumFlags] = {0, 0, 0, 0};
    TP_HIP(hipMemcpyAsync(h, P->flags.p, sizeof(h), hipMemcpyDeviceToHost, P->stream));
    TP_HIP(hipStreamSynchronize(P->stream));
    if (h[0] | h[1] | h[2] | h[3]) TP_HIP(hipMemsetAsync(P->flags.p, 0, sizeof(h), P->stream));
    if (h[kFlagBadIndex]) return fail(TP_E_BAD_INDEX, "a face refers to a vertex index outside [0, nV)");
    if (h[kFlagNonFinite]) return fail(TP_E_NONFINITE, "non-finite vertex coordinates or face quantities");
    if (h[kFlagDegenerate]) return fail(TP_E_DEGENERATE_FACE, "a face has zero area (its normal is undefined)");
    if (h[kFlagCgAbort]) return fail(TP_E_DEVICE, "CG workgroup barrier timed out");
    return TP_OK;
}

// Read one device double (synchronous).
tp_status read_scalars(tp_problem* P, const double* dev, double* host, int n)
{
    TP_HIP(hipMemcpyAsync(host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, P->stream));
    TP_HIP(hipStreamSynchronize(P->stream));
    return TP_OK;
}

tp_status alloc_faces(tp_problem* P)
{
    P->cap = face_capacity(P->nF, 4);
    TP_TRY(P->fx.ensure(P->cap, P->stream));
    TP_TRY(P->fl.ensure(P->cap, P->stream));
    TP_TRY(P->fn.ensure(P->cap, P->stream));
    TP_TRY(P->dx.ensure(P->cap, P->stream));
    TP_TRY(P->dn.ensure(P->cap, P->stream));
    TP_TRY(P->tbox.ensure(2 * (P->cap / kTileJ), P->stream));
    P->fd.nF = P->nF;
    P->fd.cap = P->cap;
    P->fd.fx = P->fx.p;
    P->fd.fl = P->fl.p;
    P->fd.fn = P->fn.p;
    P->fd.dx = P->dx.p;
    P->fd.dn = P->dn.p;
    P->fd.tbox = P->tbox.p;
    TP_TRY(P->flags.ensure(kNumFlags, P->stream));
    TP_HIP(hipMemsetAsync(P->flags.p, 0, sizeof(int) * kNumFlags, P->stream));
    TP_TRY(P->scal.ensure(256, P->stream));
    TP_TRY(P->red.ensure(reduce_scratch_doubles(16), P->stream));
    TP_TRY(P->hs.ensure(256));
    TP_TRY(P->hflags.ensure(kNumFlags));
    TP_TRY(P->hiters.ensure(2 * kMaxCols));
    TP_TRY(P->hrelres.ensure(2 * kMaxCols));
    return TP_OK;
}

// Face quantities at vertices Vsrc (defaults to the problem's vertices).
tp_status geometry(tp_problem* P, const double* Vsrc = nullptr)
{
    const double* src = Vsrc ? Vsrc : P->V.p;
    TP_HIP(launch_face_geom(src, P->nV, P->F.p, P->nF, P->fd, P->flags.p, P->stream));
    TP_TRY(check_flags(P));
    P->geom_valid = (Vsrc == nullptr);
    P->fd_V = src;
    ++P->geom_ver;
    return TP_OK;
}

tp_status ensure_geometry(tp_problem* P)
{
    if (!P->geom_valid) TP_TRY(geometry(P));
    return TP_OK;
}

tp_status ensure_vf(tp_problem* P)
{
    if (P->have_vf) return TP_OK;
    hipStream_t s = P->stream;
    TP_TRY(P->vf_off.ensure(P->nV + 1, s));
    TP_TRY(P->vf_idx.ensure(3 * P->nF, s));
    TP_TRY(P->tmp_i.ensure(P->nV + 1, s));
    TP_HIP(hipMemsetAsync(P->tmp_i.p, 0, sizeof(int32_t) * (P->nV + 1), s));
    TP_HIP(launch_vf_count(P->F.p, P->nF, P->nV, P->tmp_i.p, s));
    TP_HIP(launch_scan(P->tmp_i.p, P->nV, P->vf_off.p, s));
    TP_HIP(hipMemsetAsync(P->tmp_i.p, 0, sizeof(int32_t) * (P->nV + 1), s));
    TP_HIP(launch_vf_fill(P->F.p, P->nF, P->nV, P->vf_off.p, P->tmp_i.p, P->vf_idx.p, s));
    TP_HIP(launch_sort_rows(P->vf_off.p, P->nV, P->vf_idx.p, s));
    P->have_vf = true;
    return TP_OK;
}

// Block partition for the preconditioner: vertices ordered by (component, Morton code
// of the position in the component's bounding cube), each component cut into equal blocks
// of at most pcg_block_size() consecutive vertices.  Builds the permuted ELL pattern, the
// neighbouring-block lists and the per-block / per-component tables.
tp_status build_pcg(tp_problem* P, const std::vector<int32_t>& label, int ncomp,
                    const std::vector<int32_t>& hoff, const std::vector<int32_t>& hcol)
{
    hipStream_t s = P->stream;
    const int64_t n = P->nV;
    const int BS = pcg_block_size();
    std::vector<double> hV(3 * n);
    TP_HIP(hipMemcpyAsync(hV.data(), P->V.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    std::vector<double> lo(3 * ncomp, 1e300), hi(3 * ncomp, -1e300);
    for (int64_t v = 0; v < n; ++v)
        for (int d = 0; d < 3; ++d) {
            lo[3 * label[v] + d] = std::min(lo[3 * label[v] + d], hV[3 * v + d]);
            hi[3 * label[v] + d] = std::max(hi[3 * label[v] + d], hV[3 * v + d]);
        }
    auto spread = [](uint64_t x) {   // 21 bits -> every third bit
        x &= 0x1fffff;
        x = (x | x << 32) & 0x1f00000000ffffull;
        x = (x | x << 16) & 0x1f0000ff0000ffull;
        x = (x | x << 8) & 0x100f00f00f00f00full;
        x = (x | x << 4) & 0x10c30c30c30c30c3ull;
        x = (x | x << 2) & 0x1249249249249249ull;
        return x;
    };
    // one scale for the three axes (the cube around the component's box), so the Morton
    // cells are cubes and the blocks compact in space: per-axis scaling stretches the cells
    // of flat components (a torus lying in a plane) and costs a third more CG iterations
    std::vector<double> ext(ncomp, 0.0);
    for (int c = 0; c < ncomp; ++c)
        for (int d = 0; d < 3; ++d) ext[c] = std::max(ext[c], hi[3 * c + d] - lo[3 * c + d]);
    std::vector<uint64_t> key(n);
    for (int64_t v = 0; v < n; ++v) {
        uint64_t code = 0;
        for (int d = 0; d < 3; ++d) {
            const double l = lo[3 * label[v] + d], e = ext[label[v]];
            const double t = e > 0.0 ? (hV[3 * v + d] - l) / e : 0.0;
            const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097151.0));
            code |= spread(q) << d;
        }
        key[v] = code;
    }
    std::vector<int32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
        if (label[a] != label[b]) return label[a] < label[b];
        return key[a] < key[b];
    });
    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) iperm[perm[i]] = (int32_t)i;
    // blocks: each component [c0, c1) in the new order cut into ceil(m / BS) equal parts
    std::vector<int32_t> bstart, bcomp, whole;
    int64_t pos = 0;
    while (pos < n) {
        const int c = label[perm[pos]];
        int64_t end = pos;
        while (end < n && label[perm[end]] == c) ++end;
        const int64_t m = end - pos;
        const int64_t nbc = (m + BS - 1) / BS;
        for (int64_t q = 0; q < nbc; ++q) {
            bstart.push_back((int32_t)(pos + q * m / nbc));
            bcomp.push_back(c);
            whole.push_back(nbc == 1 ? 1 : 0);
        }
        pos = end;
    }
    const int nb = (int)bstart.size();
    bstart.push_back((int32_t)n);
    P->have_pcg = false;
    if (nb < 1 || nb > pcg_max_blocks_multi()) return TP_OK;  // too many blocks: plain CG
    P->pcg_ml = nb > pcg_max_blocks();                        // multi-launch solve
    std::vector<int32_t> blk(n);
    for (int b = 0; b < nb; ++b)
        for (int32_t i = bstart[b]; i < bstart[b + 1]; ++i) blk[i] = b;
    // aggregates: runs of `agg` consecutive blocks of one component, so that the coarse
    // space (4 functions per aggregate) has at most pcg_max_coarse() functions
    const int agg = std::max(1, (4 * nb + pcg_max_coarse() - 1) / pcg_max_coarse());
    std::vector<int32_t> astart, aob(nb), acomp;
    for (int b = 0; b < nb;) {
        int e = b;
        while (e < nb && e - b < agg && bcomp[e] == bcomp[b]) ++e;
        for (int q = b; q < e; ++q) aob[q] = (int32_t)astart.size();
        astart.push_back(b);
        acomp.push_back(bcomp[b]);
        b = e;
    }
    const int na = (int)astart.size();
    astart.push_back(nb);
    if (4 * na > pcg_max_coarse()) return TP_OK;                // too many components: plain CG
    // aggregates touching each block (through its rows' entries), and each row's slots
    std::vector<int32_t> abl_off(1, 0), abl;
    for (int b = 0; b < nb; ++b) {
        std::vector<int32_t> lst;
        for (int32_t i = bstart[b]; i < bstart[b + 1]; ++i) {
            const int32_t old = perm[i];
            for (int32_t q = hoff[old]; q < hoff[old + 1]; ++q) lst.push_back(aob[blk[iperm[hcol[q]]]]);
        }
        lst.push_back(aob[b]);
        std::sort(lst.begin(), lst.end());
        lst.erase(std::unique(lst.begin(), lst.end()), lst.end());
        if ((int)lst.size() > pcg_max_block_aggregates()) return TP_OK;   // plain CG
        abl.insert(abl.end(), lst.begin(), lst.end());
        abl_off.push_back((int32_t)abl.size());
    }
    const int w = P->ell_w;
    std::vector<int32_t> pcol((size_t)w * n);
    std::vector<int8_t> rslot((size_t)kPcgRowSlots * n, (int8_t)-1), eslot((size_t)w * n);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t old = perm[i];
        const int32_t b = hoff[old], len = hoff[old + 1] - b;
        const int bi = blk[i];
        int nq = 0;
        int sl_of_q[kPcgRowSlots];
        for (int e = 0; e < w; ++e) {
            const int32_t j = e < len ? iperm[hcol[b + e]] : (int32_t)i;   // padding: the row itself, value 0
            pcol[(size_t)e * n + i] = j;
            const int32_t ag = aob[blk[j]];
            int sl = -1;
            for (int q = abl_off[bi]; q < abl_off[bi + 1]; ++q)
                if (abl[q] == ag) sl = q - abl_off[bi];
            int q = 0;
            while (q < nq && sl_of_q[q] != sl) ++q;
            if (q == nq) {
                if (nq == kPcgRowSlots) return TP_OK;             // plain CG
                sl_of_q[nq++] = sl;
                rslot[(size_t)q * n + i] = (int8_t)sl;
            }
            eslot[(size_t)e * n + i] = (int8_t)q;
        }
    }
    auto up = [&](auto& buf, const auto& host) -> tp_status {
        TP_TRY(buf.ensure(std::max<size_t>(host.size(), 1), s));
        TP_HIP(hipMemcpyAsync(buf.p, host.data(), sizeof(host[0]) * host.size(), hipMemcpyHostToDevice, s));
        return TP_OK;
    };
    TP_TRY(up(P->pcg_perm, perm));
    TP_TRY(up(P->pcg_pcol, pcol));
    TP_TRY(up(P->pcg_bstart, bstart));
    TP_TRY(up(P->pcg_whole, whole));
    TP_TRY(up(P->pcg_blk, blk));
    TP_TRY(up(P->pcg_astart, astart));
    TP_TRY(up(P->pcg_aob, aob));
    TP_TRY(up(P->pcg_acomp, acomp));
    TP_TRY(up(P->pcg_abl_off, abl_off));
    TP_TRY(up(P->pcg_abl, abl));
    TP_TRY(up(P->pcg_rslot, rslot));
    TP_TRY(up(P->pcg_eslot, eslot));
    const int nc = 4 * na;
    TP_TRY(P->pcg_pval.ensure((size_t)w * n, s));
    TP_TRY(P->pcg_phi.ensure((size_t)4 * n, s));
    TP_TRY(P->pcg_rw.ensure((size_t)kPcgRowSlots * 4 * n, s));
    TP_TRY(P->pcg_esum.ensure((size_t)nc, s));
    TP_TRY(P->pcg_Binv.ensure((size_t)nb * BS * BS, s));
    TP_TRY(P->pcg_C0inv.ensure((size_t)nc * nc, s));
    TP_HIP(hipStreamSynchronize(s));
    PcgSetup& ps = P->pcg;
    ps.n = n; ps.nb = nb; ps.na = na; ps.nc = nc; ps.ell_w = w;
    ps.perm = P->pcg_perm.p; ps.pcol = P->pcg_pcol.p; ps.pval = P->pcg_pval.p;
    ps.bstart = P->pcg_bstart.p; ps.whole = P->pcg_whole.p; ps.blk = P->pcg_blk.p;
    ps.astart = P->pcg_astart.p; ps.agg_of_block = P->pcg_aob.p; ps.acomp = P->pcg_acomp.p;
    ps.abl_off = P->pcg_abl_off.p; ps.abl = P->pcg_abl.p; ps.rslot = P->pcg_rslot.p; ps.eslot = P->pcg_eslot.p;
    ps.phi = P->pcg_phi.p; ps.rw = P->pcg_rw.p; ps.esum = P->pcg_esum.p;
    ps.Binv = P->pcg_Binv.p; ps.C0inv = P->pcg_C0inv.p;
    P->have_pcg = true;
    return TP_OK;
}

// Cotan sparsity pattern and connected components (host union-find on a copy of F).
tp_status ensure_lap(tp_problem* P)
{
    if (P->have_lap) return TP_OK;
    TP_TRY(ensure_vf(P));
    hipStream_t s = P->stream;
    TP_TRY(P->tmp_j.ensure(6 * P->nF + 1, s));
    TP_TRY(P->lap_off.ensure(P->nV + 1, s));
    TP_HIP(launch_lap_pattern_count(P->F.p, P->nV, P->vf_off.p, P->vf_idx.p, P->tmp_j.p, P->tmp_i.p, s));
    TP_HIP(launch_scan(P->tmp_i.p, P->nV, P->lap_off.p, s));
    int32_t nnz = 0;
    TP_HIP(hipMemcpyAsync(&nnz, P->lap_off.p + P->nV, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    P->nnz = nnz;
    TP_TRY(P->lap_col.ensure(std::max<int64_t>(nnz, 1), s));
    TP_TRY(P->lap_val.ensure(std::max<int64_t>(nnz, 1), s));
    TP_HIP(launch_lap_pattern_fill(P->nV, P->vf_off.p, P->tmp_j.p, P->lap_off.p, P->lap_col.p, s));
    std::vector<int32_t> hoff(P->nV + 1), hcol(std::max<int64_t>(nnz, 1));
    {
        TP_HIP(hipMemcpyAsync(hoff.data(), P->lap_off.p, sizeof(int32_t) * (P->nV + 1), hipMemcpyDeviceToHost, s));
        TP_HIP(hipMemcpyAsync(hcol.data(), P->lap_col.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        int w = 1;
        for (int64_t v = 0; v < P->nV; ++v) w = std::max(w, hoff[v + 1] - hoff[v]);
        P->ell_w = w;
        TP_TRY(P->ell_col.ensure((size_t)w * P->nV, s));
        TP_TRY(P->ell_val.ensure((size_t)w * P->nV, s));
    }

    // connected components over the face graph
    std::vector<int32_t> hF(3 * P->nF);
    TP_HIP(hipMemcpyAsync(hF.data(), P->F.p, sizeof(int32_t) * 3 * P->nF, hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> parent(P->nV);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int32_t a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    };
    for (int64_t f = 0; f < P->nF; ++f)
        for (int c = 1; c < 3; ++c) {
            int32_t a = find(hF[3 * f]), b = find(hF[3 * f + c]);
            if (a != b) parent[std::max(a, b)] = std::min(a, b);
        }
    std::vector<int32_t> label(P->nV), root_label(P->nV, -1);
    int nc = 0;
    for (int64_t v = 0; v < P->nV; ++v) {
        int32_t r = find((int32_t)v);
        if (root_label[r] < 0) root_label[r] = nc++;
        label[v] = root_label[r];
    }
    if (nc > kMaxComponents)
        return fail(TP_E_INVALID_ARGUMENT, "more than " + std::to_string(kMaxComponents) + " connected components");
    std::vector<double> cnt(nc, 0.0);
    for (int64_t v = 0; v < P->nV; ++v) cnt[label[v]] += 1.0;
    for (auto& c : cnt) c = 1.0 / c;
    P->ncomp = nc;
    TP_TRY(P->comp.ensure(P->nV, s));
    TP_TRY(P->inv_count.ensure(nc, s));
    TP_HIP(hipMemcpyAsync(P->comp.p, label.data(), sizeof(int32_t) * P->nV, hipMemcpyHostToDevice, s));
    TP_HIP(hipMemcpyAsync(P->inv_count.p, cnt.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
    TP_HIP(hipStreamSynchronize(s));
    P->comp_host = label;
    if (P->prm.cg_precond) TP_TRY(build_pcg(P, label, nc, hoff, hcol));
    P->have_lap = true;
    return TP_OK;
}

// The cotan values of V, the solvers' matrix and the preconditioner's set-up, on stream s
// (buffers allocated beforehand: this enqueues kernels only).
tp_status launch_cotan(tp_problem* P, hipStream_t s)
{
    TP_HIP(launch_cotan_values(P->V.p, P->F.p, P->nV, P->vf_off.p, P->vf_idx.p, P->lap_off.p, P->lap_col.p,
                               P->lap_val.p, s));
    // the solvers' matrix: the cotan values, with the pin rows appended (Sec. 7.2)
    const double* sv = P->lap_val.p;
    if (P->npins > 0) {
        TP_HIP(launch_pin_values(P->nV, P->lap_off.p, P->lap_col.p, P->lap_val.p, P->pin_mask.p, P->lap_pin.p, s));
        sv = P->lap_pin.p;
    }
    TP_HIP(launch_csr_to_ell(P->nV, P->lap_off.p, P->lap_col.p, sv, P->ell_w, P->ell_col.p, P->ell_val.p, s));
    if (P->have_pcg) TP_HIP(launch_pcg_setup(P->pcg, P->V.p, P->lap_off.p, sv, s));
    return TP_OK;
}

// The problem's second stream and its two events, made on first use; false if they cannot
// be made (then everything runs on the problem's stream).
bool ensure_aux(tp_problem* P)
{
    if (P->aux) return true;
    hipStream_t a = nullptr;
    hipEvent_t f = nullptr, j = nullptr;
    if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
        if (j) (void)hipEventDestroy(j);
        if (f) (void)hipEventDestroy(f);
        if (a) (void)hipStreamDestroy(a);
        (void)hipGetLastError();
        return false;
    }
    P->aux = a;
    P->aux_fork = f;
    P->aux_join = j;
    return true;
}

// Makes the problem's stream wait for the work started on the second stream.
tp_status join_aux(tp_problem* P)
{
    if (!P->aux_pending) return TP_OK;
    TP_HIP(hipStreamWaitEvent(P->stream, P->aux_join, 0));
    P->aux_pending = false;
    return TP_OK;
}

// Starts the set-up for the current V on the second stream, after everything enqueued so
// far on the problem's stream, so that it runs beside the energy, differential and
// fractional launches that follow; ensure_cotan joins it.  Does nothing before the
// topology exists, when the set-up is current, or when no second stream can be made.
tp_status start_cotan(tp_problem* P)
{
    if (!P->have_lap || P->cotan_valid) return TP_OK;
    TP_TRY(join_aux(P));
    if (P->npins > 0) TP_TRY(P->lap_pin.ensure(std::max<int64_t>(P->nnz, 1), P->stream));
    if (!ensure_aux(P)) return TP_OK;   // ensure_cotan does the set-up on the problem's stream
    TP_HIP(hipEventRecord(P->aux_fork, P->stream));
    TP_HIP(hipStreamWaitEvent(P->aux, P->aux_fork, 0));
    TP_TRY(launch_cotan(P, P->aux));
    TP_HIP(hipEventRecord(P->aux_join, P->aux));
    P->aux_pending = true;
    P->cotan_valid = true;
    return TP_OK;
}

tp_status ensure_cotan(tp_problem* P)
{
    TP_TRY(ensure_lap(P));
    TP_TRY(join_aux(P));
    P->setup_used = true;
    if (!P->cotan_valid) {
        if (P->npins > 0) TP_TRY(P->lap_pin.ensure(std::max<int64_t>(P->nnz, 1), P->stream));
        TP_TRY(launch_cotan(P, P->stream));
        P->cotan_valid = true;
    }
    return TP_OK;
}

// Sum of n doubles with stride ld (device), to the host.
tp_status device_sum(tp_problem* P, const double* x, int ld, int64_t n, double* out)
{
    TP_HIP(launch_dot_cols(x, ld, nullptr, 0, n, 1, P->red.p, P->scal.p, P->stream));
    return read_scalars(P, P->scal.p, out, 1);
}

// Total area (from the current face data, which must describe Vsrc) and signed volume.
tp_status total_area_volume(tp_problem* P, const double* Vsrc, double* area, double* vol)
{
    // areas are the .w lane of the FP64 barycenter array
    TP_TRY(device_sum(P, &P->dx.p[0].w, 4, P->nF, area));
    TP_TRY(P->vol6.ensure(P->nF, P->stream));
    TP_HIP(launch_face_volume(Vsrc, P->F.p, P->nF, P->vol6.p, P->stream));
    double v6 = 0;
    TP_TRY(device_sum(P, P->vol6.p, 1, P->nF, &v6));
    *vol = v6 / 6.0;
    return TP_OK;
}

// ------------------------------------------------------------------ batches
//
// A batch is a list of problems that share a device and a stream.  The all-pairs work of
// one phase of all its problems goes into shared launches (launch_pairs_*), and their CG
// solves into shared cooperative launches (launch_pcg_batch); the O(F) and O(V) passes are
// launched per problem back to back, and the host waits once per phase for the whole
// batch.  A problem's arithmetic does not depend on the other problems of its batch, so
// its results are the same alone and in any batch.

using Batch = std::vector<tp_problem*>;

bool finite(double x) { return std::isfinite(x); }

// Copy the device scalars and flags of every problem to its pinned host mirrors.
tp_status enqueue_fetch(const Batch& B)
{
    for (tp_problem* P : B) {
        TP_HIP(hipMemcpyAsync(P->hs.p, P->scal.p, sizeof(double) * kNumSlots, hipMemcpyDeviceToHost, P->stream));
        TP_HIP(hipMemcpyAsync(P->hflags.p, P->flags.p, sizeof(int) * kNumFlags, hipMemcpyDeviceToHost, P->stream));
    }
    return TP_OK;
}

tp_status sync_batch(const Batch& B)
{
    TP_HIP(hipStreamSynchronize(B[0]->stream));
    return TP_OK;
}

// Status from the fetched device flags of P (clears them on both sides).
tp_status flag_status(tp_problem* P)
{
    int* h = P->hflags.p;
    const int bad = h[kFlagBadIndex], nonfin = h[kFlagNonFinite], degen = h[kFlagDegenerate],
              abort_ = h[kFlagCgAbort];
    if (bad | nonfin | degen | abort_) {
        TP_HIP(hipMemsetAsync(P->flags.p, 0, sizeof(int) * kNumFlags, P->stream));
        for (int q = 0; q < kNumFlags; ++q) h[q] = 0;
    }
    if (bad) return fail(TP_E_BAD_INDEX, "a face refers to a vertex index outside [0, nV)");
    if (nonfin) return fail(TP_E_NONFINITE, "non-finite vertex coordinates or face quantities");
    if (degen) return fail(TP_E_DEGENERATE_FACE, "a face has zero area (its normal is undefined)");
    if (abort_) return fail(TP_E_DEVICE, "CG workgroup barrier timed out");
    return TP_OK;
}

// ------------------------------------------------------------------ Barnes-Hut

tp_status ensure_bh(tp_problem* P)
{
    hipStream_t s = P->stream;
    const int64_t nF = P->nF;
    const int64_t M = (int64_t)bh_node_count(nF, P->prm.leaf_size, nullptr);
    TP_TRY(P->bh_flo.ensure(3 * nF, s));
    TP_TRY(P->bh_fhi.ensure(3 * nF, s));
    TP_TRY(P->bh_fr2.ensure(nF, s));
    TP_TRY(P->bh_box.ensure(6, s));
    TP_TRY(P->bh_kin.ensure(nF, s));
    TP_TRY(P->bh_kout.ensure(nF, s));
    const size_t tb = bh_sort_temp_bytes(nF);
    TP_TRY(P->bh_tmp.ensure(tb, s));
    TP_TRY(P->bh_order.ensure(nF, s));
    TP_TRY(P->bh_pos.ensure(nF, s));
    TP_TRY(P->bh_na.ensure(M, s));
    TP_TRY(P->bh_nsx.ensure(3 * M, s));
    TP_TRY(P->bh_nX.ensure(3 * M, s));
    TP_TRY(P->bh_nlo.ensure(3 * M, s));
    TP_TRY(P->bh_nhi.ensure(3 * M, s));
    TP_TRY(P->bh_nr2.ensure(M, s));
    TP_TRY(P->bh_gS.ensure(7 * nF, s));
    TP_TRY(P->bh_eS.ensure(nF, s));
    TP_TRY(P->bh_accF.ensure(4 * nF, s));
    TP_TRY(P->bh_accN.ensure(4 * M, s));
    TP_TRY(P->bh_counts.ensure(2, s));
    TP_TRY(P->bh_nm.ensure((size_t)M * ((kMaxGroupCols + 3) / 4 * 4), s));
    BhBuffers& b = P->bh;
    b.flo = P->bh_flo.p; b.fhi = P->bh_fhi.p; b.fr2 = P->bh_fr2.p; b.box = P->bh_box.p;
    b.keys_in = P->bh_kin.p; b.keys_out = P->bh_kout.p; b.sort_tmp = P->bh_tmp.p; b.sort_bytes = tb;
    b.order = P->bh_order.p; b.pos = P->bh_pos.p; b.na = P->bh_na.p; b.nsx = P->bh_nsx.p; b.nX = P->bh_nX.p;
    b.nlo = P->bh_nlo.p; b.nhi = P->bh_nhi.p; b.nr2 = P->bh_nr2.p; b.gS = P->bh_gS.p; b.eS = P->bh_eS.p;
    b.accF = P->bh_accF.p; b.accN = P->bh_accN.p; b.counts = P->bh_counts.p;
    return TP_OK;
}

// The Morton tree of the current face data (built once per geometry).
tp_status ensure_tree(tp_problem* P)
{
    TP_TRY(ensure_bh(P));
    if (P->bh_ver != P->geom_ver) {
        TP_HIP(launch_bh_build(P->bh, P->fd_V, P->F.p, P->face_orig.p, P->nF, P->prm.leaf_size, P->fd, P->stream));
        P->bh_ver = P->geom_ver;
    }
    return TP_OK;
}

// Block lists of the block cluster tree (Sec. 5.1.4) for the current geometry, built on the
// host from the tree's node boxes, radii and areas: a breadth-first split of (root, root);
// a pair of clusters is admissible when max(r_I^2, r_J^2) < chi^2 dist^2 (dist between the
// boxes), otherwise it is split into its children's pairs until both are leaves (all
// leaves lie at the same depth); empty clusters (padding) are dropped.
// Grow buf to at least need elements, keeping its first used ones (tmp: spare buffer).
tp_status grow_keep(DevBuf<uint64_t>& buf, DevBuf<uint64_t>& tmp, size_t used, size_t need, hipStream_t s)
{
    if (need <= buf.n && buf.p) return TP_OK;
    TP_TRY(tmp.ensure(std::max(need, buf.n + buf.n / 2), s));
    if (used) TP_HIP(hipMemcpyAsync(tmp.p, buf.p, sizeof(uint64_t) * used, hipMemcpyDeviceToDevice, s));
    buf.swap(tmp);
    return TP_OK;
}

// Block lists of the block cluster tree of the current tree (once per geometry), built on
// the device level by level (the block counts of each level are read back to size the
// next), then sorted into CSR rows.
tp_status ensure_bct(tp_problem* P)
{
    TP_TRY(ensure_tree(P));
    if (P->bct_ver == P->geom_ver) return TP_OK;
    hipStream_t s = P->stream;
    int64_t Pl = 0;
    const int64_t M = (int64_t)bh_node_count(P->nF, P->prm.leaf_size, &Pl);
    TP_TRY(P->bct_cnt.ensure(3, s));
    TP_TRY(P->bct_hcnt.ensure(3));
    TP_TRY(P->bct_rec.ensure((size_t)8 * M, s));
    TP_HIP(launch_bct_nodes(P->bh, M, P->bct_rec.p, s));
    TP_TRY(P->bct_fr0.ensure(1024, s));
    const uint64_t root = (1ull << 32) | 1ull;
    TP_HIP(hipMemcpyAsync(P->bct_fr0.p, &root, sizeof(root), hipMemcpyHostToDevice, s));
    TP_HIP(hipStreamSynchronize(s));
    DevBuf<uint64_t>* cur = &P->bct_fr0;
    DevBuf<uint64_t>* nxt = &P->bct_fr1;
    int64_t n = 1, nfar = 0, nnear = 0;
    while (n > 0) {
        TP_TRY(nxt->ensure((size_t)4 * n, s));
        TP_TRY(grow_keep(P->bct_fkeys, P->bct_grow, (size_t)nfar, (size_t)(nfar + n), s));
        TP_TRY(grow_keep(P->bct_nkeys, P->bct_grow, (size_t)nnear, (size_t)(nnear + n), s));
        unsigned long long* h = P->bct_hcnt.p;
        h[0] = (unsigned long long)nfar;
        h[1] = (unsigned long long)nnear;
        h[2] = 0;
        TP_HIP(hipMemcpyAsync(P->bct_cnt.p, h, 3 * sizeof(unsigned long long), hipMemcpyHostToDevice, s));
        TP_HIP(launch_bct_expand(P->bct_rec.p, Pl, P->prm.chi, cur->p, n, P->bct_fkeys.p, P->bct_nkeys.p, nxt->p,
                                 P->bct_cnt.p, s));
        TP_HIP(hipMemcpyAsync(h, P->bct_cnt.p, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        nfar = (int64_t)h[0];
        nnear = (int64_t)h[1];
        n = (int64_t)h[2];
        std::swap(cur, nxt);
    }
    if (nfar > (int64_t)INT32_MAX || nnear > (int64_t)INT32_MAX)
        return fail(TP_E_OUT_OF_MEMORY, "block cluster tree: more than 2^31 blocks");
    const int64_t nmax = std::max<int64_t>(std::max(nfar, nnear), 1);
    TP_TRY(P->bct_sorted.ensure((size_t)nmax, s));
    const size_t tb = bct_sort_temp_bytes(nmax);
    TP_TRY(P->bct_tmp.ensure(tb, s));
    TP_TRY(P->bct_far_off.ensure((size_t)M + 1, s));
    TP_TRY(P->bct_far_col.ensure((size_t)std::max<int64_t>(nfar, 1), s));
    TP_TRY(P->bct_near_off.ensure((size_t)Pl + 1, s));
    TP_TRY(P->bct_near_col.ensure((size_t)std::max<int64_t>(nnear, 1), s));
    TP_TRY(P->bct_yt.ensure((size_t)M * ((kMaxGroupCols + 3) / 4 * 4 + 4), s));
    TP_HIP(launch_bct_sort_csr(P->bct_fkeys.p, P->bct_sorted.p, nfar, P->bct_tmp.p, tb, M, P->bct_far_off.p,
                               P->bct_far_col.p, s));
    TP_HIP(launch_bct_sort_csr(P->bct_nkeys.p, P->bct_sorted.p, nnear, P->bct_tmp.p, tb, Pl, P->bct_near_off.p,
                               P->bct_near_col.p, s));
    P->bct_nadm = nfar;
    P->bct_ninad = nnear;
    P->bct_ver = P->geom_ver;
    return TP_OK;
}

// E_BH -> scal[slot]; with dE, the differential of E_BH into dE (nV x 3).  The face data
// must describe P->fd_V (the tree is built from it).
tp_status enqueue_bh(tp_problem* P, double* dE, int slot)
{
    hipStream_t s = P->stream;
    TP_TRY(ensure_tree(P));
    const int leaf = P->prm.leaf_size;
    if (dE) {
        TP_TRY(ensure_vf(P));
        TP_TRY(P->gface.ensure((size_t)7 * P->nF, s));
    }
    TP_HIP(launch_bh_eval(P->bh, P->nF, leaf, P->prm.theta, P->prm.precision, P->prm.alpha, P->prm.beta, P->fd,
                          dE != nullptr, P->gface.p, P->nF, s));
    if (dE)
        TP_HIP(launch_grad_gather(P->fd_V, P->F.p, P->nV, P->nF, P->vf_off.p, P->vf_idx.p, P->gface.p, P->nF, dE, s));
    TP_HIP(launch_dot_cols(P->bh_eS.p, 1, nullptr, 0, P->nF, 1, P->red.p, P->scal.p + slot, s));
    return TP_OK;
}

// The energy from the scalar the gradient phase leaves in its slot: twice the energy for
// the direct sums (sum_S a_S dE/da_S), E_BH itself for Barnes-Hut.
double gradient_energy(const tp_problem* P, double v)
{
    return P->prm.theta > 0.0 ? v : 0.5 * v;
}

// ------------------------------------------------------------------ all-pairs phases

bool near_field(const tp_problem* P) { return P->prm.precision == TP_PREC_FP32_NEAR64; }

// Device bytes of the near-field grid of a problem of nF faces.
size_t near_grid_bytes(int64_t nF)
{
    const int64_t gm = near_grid_gmax(nF);
    return (size_t)nF * (4 + 4 + 4 + 4 + 16 + 16) + (size_t)(gm * gm * gm) * sizeof(int2) +
           near_grid_sort_temp_bytes(nF) + sizeof(NearGridParams);
}

// The near-field grid of the current face data (built once per geometry).
tp_status ensure_near_grid(tp_problem* P)
{
    hipStream_t s = P->stream;
    const size_t n = (size_t)P->nF;
    NearGrid& g = P->ng;
    if (!g.prm) {
        g.gmax = near_grid_gmax(P->nF);
        const size_t gm = (size_t)g.gmax;
        TP_TRY(P->ng_kin.ensure(n, s));
        TP_TRY(P->ng_kout.ensure(n, s));
        TP_TRY(P->ng_vin.ensure(n, s));
        TP_TRY(P->ng_vout.ensure(n, s));
        TP_TRY(P->ng_sfx.ensure(n, s));
        TP_TRY(P->ng_sfl.ensure(n, s));
        TP_TRY(P->ng_cell.ensure(gm * gm * gm, s));
        g.sort_bytes = near_grid_sort_temp_bytes(P->nF);
        TP_TRY(P->ng_tmp.ensure(g.sort_bytes, s));
        TP_TRY(P->ng_prm.ensure(1, s));
        g.kin = P->ng_kin.p; g.kout = P->ng_kout.p; g.vin = P->ng_vin.p; g.vout = P->ng_vout.p;
        g.sfx = P->ng_sfx.p; g.sfl = P->ng_sfl.p; g.cell = P->ng_cell.p; g.sort_tmp = P->ng_tmp.p;
        g.prm = P->ng_prm.p;
    }
    if (P->ng_ver != P->geom_ver) {
        TP_HIP(launch_near_grid_build(g, P->fd, P->nF, (float)P->rho2, s));
        P->ng_ver = P->geom_ver;
    }
    return TP_OK;
}

// The FP64 near-field slice (index n_split of the partial buffer, nacc accumulators) of
// every problem of the batch that uses it, in one launch.
tp_status enqueue_near(const Batch& B, const std::vector<PairPlan>& plans, int nacc, bool grad)
{
    std::vector<PairJob> jobs;
    for (size_t m = 0; m < B.size(); ++m) {
        tp_problem* P = B[m];
        if (!near_field(P)) continue;
        const PairPlan& pl = plans[m];
        TP_TRY(ensure_near_grid(P));
        PairJob J = make_pair_job(P->fd, pl, P->part.p + (size_t)pl.n_split * nacc * pl.irows);
        J.n_itiles = (int)((P->nF + near_block_faces() - 1) / near_block_faces());
        J.tiles_per_split = J.ntiles_j;
        J.rho2 = (float)P->rho2;
        J.nord = P->ng.vout;
        J.nfx = P->ng.sfx;
        J.nfl = P->ng.sfl;
        J.ncell = P->ng.cell;
        J.ngp = P->ng.prm;
        jobs.push_back(J);
    }
    if (jobs.empty()) return TP_OK;
    TP_HIP(launch_near64(jobs.data(), (int)jobs.size(), B[0]->prm.alpha, B[0]->prm.beta, grad, B[0]->stream));
    return TP_OK;
}

// The symmetric all-pairs kernels (launch_grad_sym, launch_frac_sym: each unordered pair
// evaluated once for both rows) are used for the direct FP32 sums, unless forced by
// tp_params.sym_pairs = 1, from kSymMinFaces faces on, below which they have too few pairs
// of blocks to fill the GPU.  Their partial buffer is kept within kSymPartBytes by running
// the rows in bands (one launch and one reduction per band; a single band up to about
// 68,000 faces for E + dE).
constexpr double kSymPartBytes = 512.0 * 1024.0 * 1024.0;
constexpr int64_t kSymMinFaces = 16384;
constexpr int kGradOutputs = 7;   // partial sums per face of the E + dE kernels

bool sym_size_ok(const tp_params& prm, int64_t nF, int nacc)
{
    (void)nacc;
    if (prm.sym_pairs == 0 || prm.theta > 0.0 || nF < 1) return false;
    return prm.sym_pairs == 1 || nF >= kSymMinFaces;
}

int sym_band_height(const tp_params& prm, int64_t nF, int kc)
{
    const int K = sym_band_blocks(nF, kc, kSymPartBytes);
    return prm.sym_band > 0 ? std::min(K, prm.sym_band) : K;
}

size_t sym_buffer_floats(const tp_params& prm, int64_t nF, int kc)
{
    return sym_part_floats(nF, kc, sym_band_height(prm, nF, kc));
}

// The bands of rows of a symmetric launch over nF faces with kc sums per face: fn(K, a0, a1,
// share of the unordered pairs) for each band in order.
template <class Fn>
tp_status for_each_sym_band(const tp_params& prm, int64_t nF, int kc, Fn&& fn)
{
    const int nB = (int)((nF + frac_sym_block_faces() - 1) / frac_sym_block_faces());
    const int K = sym_band_height(prm, nF, kc);
    const double total = (double)sym_band_units(nF, 0, nB);
    for (int a0 = 0; a0 < nB; a0 += K) {
        const int a1 = std::min(nB, a0 + K);
        TP_TRY(fn(K, a0, a1, (double)sym_band_units(nF, a0, a1) / total));
    }
    return TP_OK;
}

bool sym_frac_eligible(const tp_params& prm, int64_t nF, int kc)
{
    return prm.precision != TP_PREC_FP64 && !(prm.chi > 0.0) && kc >= 1 && kc <= kMaxGroupCols &&
           sym_size_ok(prm, nF, kc);
}

// The operator A = B + B0 (direct sums at any theta): the FP32 precisions.
bool sym_sobolev_eligible(const tp_params& prm, int64_t nF)
{
    if (prm.precision == TP_PREC_FP64 || prm.sym_pairs == 0 || nF < 1) return false;
    return prm.sym_pairs == 1 || nF >= kSymMinFaces;
}

// E + dE: the FP32 precisions with FP64 per-face sums (not the FP32-accumulator studies).
bool sym_grad_eligible(const tp_params& prm, int64_t nF)
{
    const int p = prm.precision;
    return (p == TP_PREC_FP32_HILO || p == TP_PREC_FP32 || p == TP_PREC_FP32_NEAR64) && sym_size_ok(prm, nF, kGradOutputs);
}

// E of every problem (face data must describe the point of evaluation) -> scal[slot].
tp_status enqueue_energy(const Batch& B, int slot)
{
    if (B.empty()) return TP_OK;
    if (B[0]->prm.theta > 0.0) {
        for (tp_problem* P : B) TP_TRY(enqueue_bh(P, nullptr, slot));
        return TP_OK;
    }
    hipStream_t s = B[0]->stream;
    const int prec = B[0]->prm.precision;
    std::vector<PairJob> jobs;
    std::vector<PairPlan> plans;
    std::vector<char> sym(B.size(), 0);
    double pairs = 0;
    for (size_t m = 0; m < B.size(); ++m) {
        tp_problem* P = B[m];
        PairPlan pl = plan_for(kKindEnergy, prec, 1, P->nF, P->cap);
        if (sym_grad_eligible(P->prm, P->nF)) {
            // symmetric kernel: part = [near field slice (irows)][pair-of-blocks partials]
            // [a_i near_i (nF)]; the near field goes to slice 0
            sym[m] = 1;
            pl.n_split = 0;
            TP_TRY(P->part.ensure((size_t)pl.irows + (size_t)sym_units(P->nF) + (size_t)P->nF, s));
            plans.push_back(pl);
            continue;
        }
        const int slices = pl.n_split + (near_field(P) ? 1 : 0);
        TP_TRY(P->part.ensure((size_t)slices * pl.irows, s));
        TP_TRY(P->gface.ensure((size_t)pl.irows, s));
        jobs.push_back(make_pair_job(P->fd, pl, P->part.p));
        jobs.back().rho2 = (float)P->rho2;
        plans.push_back(pl);
        pairs += (double)P->nF * (double)(P->nF - 1);
    }
    if (!jobs.empty()) {
        PairTimer t(kKindEnergy, pairs, 0.0, s);
        TP_HIP(launch_pairs_energy(jobs.data(), (int)jobs.size(), prec, B[0]->prm.alpha, B[0]->prm.beta, s));
        t.stop();
    }
    for (size_t m = 0; m < B.size(); ++m) {
        if (!sym[m]) continue;
        tp_problem* P = B[m];
        PairTimer t(kKindEnergy, (double)P->nF * (double)(P->nF - 1), 0.0, s);
        TP_HIP(launch_energy_sym(P->fd, P->part.p + plans[m].irows, prec, P->prm.alpha, P->prm.beta, (float)P->rho2,
                                 s));
        t.stop();
    }
    TP_TRY(enqueue_near(B, plans, 1, false));
    for (size_t m = 0; m < B.size(); ++m) {
        tp_problem* P = B[m];
        const PairPlan& pl = plans[m];
        if (sym[m]) {
            // E = the partials of the pairs of blocks, then sum_i a_i near_i, in that order
            const int64_t units = sym_units(P->nF);
            int64_t n = units;
            if (near_field(P)) {
                TP_HIP(launch_area_times(P->fd, P->part.p, P->nF, P->part.p + pl.irows + units, s));
                n += P->nF;
            }
            TP_HIP(launch_dot_cols(P->part.p + pl.irows, 1, nullptr, 0, n, 1, P->red.p, P->scal.p + slot, s));
            continue;
        }
        const int slices = pl.n_split + (near_field(P) ? 1 : 0);
        TP_HIP(launch_reduce_splits(P->part.p, slices, 1, pl.irows, P->nF, P->gface.p, pl.irows, s));
        // E = sum_S a_S sum_T a_T K(S,T)
        TP_HIP(launch_dot_cols(&P->dx.p[0].w, 4, P->gface.p, 1, P->nF, 1, P->red.p, P->scal.p + slot, s));
    }
    return TP_OK;
}

// dE of every problem into dE[m] (nV x 3) and 2E -> scal[slot].
tp_status enqueue_gradient(const Batch& B, double* const* dE, int slot)
{
    if (B.empty()) return TP_OK;
    if (B[0]->prm.theta > 0.0) {
        for (size_t m = 0; m < B.size(); ++m) TP_TRY(enqueue_bh(B[m], dE[m], slot));
        return TP_OK;
    }
    hipStream_t s = B[0]->stream;
    const int prec = B[0]->prm.precision;
    std::vector<PairJob> jobs;
    std::vector<PairPlan> plans;
    std::vector<char> sym(B.size(), 0);
    double pairs = 0;
    for (size_t m = 0; m < B.size(); ++m) {
        tp_problem* P = B[m];
        TP_TRY(ensure_vf(P));
        PairPlan pl = plan_for(kKindGrad, prec, 1, P->nF, P->cap);
        if (sym_grad_eligible(P->prm, P->nF)) {
            // symmetric kernel; the near field (if any) goes to slice 0 of part
            sym[m] = 1;
            pl.n_split = 0;
            TP_TRY(P->symp.ensure(sym_buffer_floats(P->prm, P->nF, kGradOutputs), s));
            TP_TRY(P->part.ensure((size_t)7 * pl.irows, s));
            TP_TRY(P->gface.ensure((size_t)7 * pl.irows, s));
            plans.push_back(pl);
            continue;
        }
        const int slices = pl.n_split + (near_field(P) ? 1 : 0);
        TP_TRY(P->part.ensure((size_t)slices * 7 * pl.irows, s));
        TP_TRY(P->gface.ensure((size_t)7 * pl.irows, s));
        jobs.push_back(make_pair_job(P->fd, pl, P->part.p));
        jobs.back().rho2 = (float)P->rho2;
        plans.push_back(pl);
        pairs += (double)P->nF * (double)(P->nF - 1);
    }
    if (!jobs.empty()) {
        PairTimer t(kKindGrad, pairs, 0.0, s);
        TP_HIP(launch_pairs_grad(jobs.data(), (int)jobs.size(), prec, B[0]->prm.alpha, B[0]->prm.beta, s));
        t.stop();
    }
    // the near field first: the reduction of a face's last band adds it
    TP_TRY(enqueue_near(B, plans, 7, true));
    for (size_t m = 0; m < B.size(); ++m) {
        if (!sym[m]) continue;
        tp_problem* P = B[m];
        const PairPlan& pl = plans[m];
        const double pp = (double)P->nF * (double)(P->nF - 1);
        TP_TRY(for_each_sym_band(P->prm, P->nF, 7, [&](int K, int a0, int a1, double share) -> tp_status {
            PairTimer t(kKindGrad, pp * share, 0.0, s);
            TP_HIP(launch_grad_sym(P->fd, P->symp.p, K, a0, a1, prec, P->prm.alpha, P->prm.beta, (float)P->rho2, s));
            t.stop();
            TP_HIP(launch_reduce_sym_band(P->symp.p, P->nF, 7, K, a0, a1, near_field(P) ? P->part.p : nullptr,
                                          P->gface.p, pl.irows, s));
            return TP_OK;
        }));
    }
    for (size_t m = 0; m < B.size(); ++m) {
        tp_problem* P = B[m];
        const PairPlan& pl = plans[m];
        const int slices = pl.n_split + (near_field(P) ? 1 : 0);
        if (!sym[m])
            TP_HIP(launch_reduce_splits(P->part.p, slices, 7, pl.irows, P->nF, P->gface.p, pl.irows, s));
        TP_HIP(launch_grad_gather(P->V.p, P->F.p, P->nV, P->nF, P->vf_off.p, P->vf_idx.p, P->gface.p,
                                  pl.irows, dE[m], s));
        // 2E = sum_S a_S dE/da_S, since dE/da_S = sum_T a_T (K(S,T) + K(T,S))
        TP_HIP(launch_dot_cols(&P->dx.p[0].w, 4, P->gface.p + 6 * pl.irows, 1, P->nF, 1, P->red.p,
                               P->scal.p + slot, s));
    }
    return TP_OK;
}

// Lu[m][:, c] = (L^sigma u[m])[:, c] for k columns (row strides ldu, ldl).
tp_status enqueue_fractional(const Batch& B, const double* const* u, int ldu, int k, double* const* Lu,
                             int ldl)
{
    if (B.empty()) return TP_OK;
    hipStream_t s = B[0]->stream;
    const int prec = B[0]->prm.precision;
    const size_t esz = prec == TP_PREC_FP64 ? sizeof(double) : sizeof(float);
    for (tp_problem* P : B) TP_TRY(ensure_vf(P));
    std::vector<PairJob> jobs(B.size());
    std::vector<PairPlan> plans(B.size());
    for (int c0 = 0; c0 < k; c0 += kMaxGroupCols) {
        const int kc = std::min(kMaxGroupCols, k - c0);
        const int kp = (kc + 3) / 4 * 4;
        double pairs = 0;
        std::vector<PairJob> direct;
        std::vector<char> sym(B.size(), 0);
        for (size_t m = 0; m < B.size(); ++m) {
            tp_problem* P = B[m];
            const PairPlan pl = plan_for(kKindFrac, prec, kc, P->nF, P->cap);
            TP_TRY(P->ub.ensure((size_t)P->cap * kp * esz, s));
            TP_TRY(P->zbuf.ensure((size_t)kc * std::max<int64_t>(pl.irows, P->nF), s));
            // face averages of columns [c0, c0 + kc): a shifted pointer with stride ldu
            TP_HIP(launch_face_avg(P->F.p, P->nF, P->cap, u[m] + c0, ldu, kc, kp, prec, P->ub.p, s));
            plans[m] = pl;
            if (P->prm.chi > 0.0) {
                // block cluster tree: hierarchical product, the row sums straight into zbuf
                TP_TRY(ensure_bct(P));
                TP_TRY(P->bh_nm.ensure((size_t)bh_node_count(P->nF, P->prm.leaf_size, nullptr) * kp, s));
                BctLists bl;
                bl.far_off = P->bct_far_off.p; bl.far_col = P->bct_far_col.p;
                bl.near_off = P->bct_near_off.p; bl.near_col = P->bct_near_col.p;
                TP_HIP(launch_bct_frac(P->bh, bl, P->nF, P->prm.leaf_size, prec, P->sigma, P->fd, P->ub.p, kp, kc,
                                       P->bh_nm.p, P->bct_yt.p, P->zbuf.p, pl.irows, s));
                continue;
            }
            if (P->prm.theta > 0.0) {
                // Barnes-Hut on the kernel matrix: the row sums straight into zbuf
                TP_TRY(ensure_tree(P));
                TP_TRY(P->bh_nm.ensure((size_t)bh_node_count(P->nF, P->prm.leaf_size, nullptr) * kp, s));
                TP_HIP(launch_bh_frac(P->bh, P->nF, P->prm.leaf_size, P->prm.theta, prec, P->sigma, P->fd, P->ub.p, kp,
                                      kc, P->bh_nm.p, P->zbuf.p, pl.irows, s));
                continue;
            }
            if (sym_frac_eligible(P->prm, P->nF, kc)) {
                TP_TRY(P->symp.ensure(sym_buffer_floats(P->prm, P->nF, kc), s));
                sym[m] = 1;
                continue;
            }
            TP_TRY(P->part.ensure((size_t)pl.n_split * kc * pl.irows, s));
            jobs[m] = make_pair_job(P->fd, pl, P->part.p, P->ub.p);
            direct.push_back(jobs[m]);
            pairs += (double)P->nF * (double)(P->nF - 1);
        }
        if (!direct.empty()) {
            PairTimer t(kKindFrac, pairs, pairs * kc, s);
            TP_HIP(launch_pairs_frac(direct.data(), (int)direct.size(), prec, B[0]->sigma, kc, s));
            t.stop();
        }
        for (size_t m = 0; m < B.size(); ++m) {
            if (!sym[m]) continue;
            tp_problem* P = B[m];
            const PairPlan& pl = plans[m];
            const double pp = (double)P->nF * (double)(P->nF - 1);
            TP_TRY(for_each_sym_band(P->prm, P->nF, kc, [&](int K, int a0, int a1, double share) -> tp_status {
                PairTimer t(kKindFrac, pp * share, pp * share * kc, s);
                TP_HIP(launch_frac_sym(P->fd, reinterpret_cast<const float*>(P->ub.p), P->symp.p, K, a0, a1, prec,
                                       P->sigma, kc, s));
                t.stop();
                TP_HIP(launch_reduce_sym_band(P->symp.p, P->nF, kc, K, a0, a1, nullptr, P->zbuf.p, pl.irows, s));
                return TP_OK;
            }));
        }
        for (size_t m = 0; m < B.size(); ++m) {
            tp_problem* P = B[m];
            const PairPlan& pl = plans[m];
            if (sym[m]) {
                // reduced band by band above
            } else if (!(P->prm.theta > 0.0) && !(P->prm.chi > 0.0))
                TP_HIP(launch_reduce_splits(P->part.p, pl.n_split, kc, pl.irows, P->nF, P->zbuf.p, pl.irows, s));
            TP_HIP(launch_ut_gather(P->F.p, P->nV, P->vf_off.p, P->vf_idx.p, P->fd, P->zbuf.p, pl.irows,
                                    kc, ldl, c0, Lu[m], s));
        }
    }
    return TP_OK;
}

// ------------------------------------------------------------------ Poisson solves

tp_status ensure_cg(tp_problem* P, int k)
{
    hipStream_t s = P->stream;
    TP_TRY(P->cg_Z.ensure(cg_state_doubles(P->nV, k), s));
    TP_TRY(P->cg_p.ensure((size_t)P->nV * k, s));
    TP_TRY(P->cg_red.ensure(cg_red_doubles(k), s));
    TP_TRY(P->cg_bar.ensure(cg_bar_words(k), s));
    TP_TRY(P->cg_iters.ensure(kMaxCols, s));
    TP_TRY(P->cg_relres.ensure(kMaxCols, s));
    TP_TRY(P->red.ensure(std::max(reduce_scratch_doubles(16), project_scratch_doubles(k, P->ncomp)), s));
    if (P->have_pcg) {
        const size_t n = (size_t)P->nV;
        const size_t kc = (size_t)std::min(k, kMaxGroupCols);
        TP_TRY(P->pcg_bp.ensure(n * kc, s));
        TP_TRY(P->pcg_xp.ensure(n * kc, s));
        if (!P->pcg_ml) {
            TP_TRY(P->pcg_Vb.ensure(2 * n * kc, s));
            TP_TRY(P->pcg_rho.ensure((size_t)2 * P->pcg.nb * 4 * kc, s));
            TP_TRY(P->pcg_red.ensure((size_t)2 * P->pcg.nb * 3 * kc, s));
        } else {
            for (DevBuf<double>* v : {&P->ml_r, &P->ml_p, &P->ml_s, &P->ml_m, &P->ml_an, &P->ml_v})
                TP_TRY(v->ensure(n * kc, s));
            TP_TRY(P->ml_shares.ensure((size_t)P->pcg.nb * 4 * kMaxGroupCols, s));
            TP_TRY(P->ml_g.ensure((size_t)P->pcg.nc * kMaxGroupCols, s));
            TP_TRY(P->ml_part.ensure(pcg_ml_part_doubles(P->nV), s));
            TP_TRY(P->ml_state.ensure(pcg_ml_state_bytes(), s));
            TP_TRY(P->ml_state_host.ensure(pcg_ml_state_bytes()));
        }
    }
    return TP_OK;
}

// A slot of the batch owner's ring of PCG tables (device + pinned host staging).  A slot
// is reused only after the copy that last read its staging has run.
tp_status pcg_table_slot(tp_problem* O, int n, void** dev, void** host, int* slot)
{
    TabRing& T = O->tab;
    const size_t need = (pcg_table_bytes(n) + 255) / 256 * 256;
    if (need > T.slot_bytes) {
        TP_HIP(hipStreamSynchronize(O->stream));
        TP_TRY(T.dev.ensure(need * kTabSlots, O->stream));
        TP_TRY(T.host.ensure(need * kTabSlots));
        T.slot_bytes = need;
        for (int q = 0; q < kTabSlots; ++q) T.used[q] = false;
    }
    for (int q = 0; q < kTabSlots; ++q)
        if (!T.ev[q]) TP_HIP(hipEventCreateWithFlags(&T.ev[q], hipEventDisableTiming));
    const int q = T.next;
    T.next = (q + 1) % kTabSlots;
    if (T.used[q]) TP_HIP(hipEventSynchronize(T.ev[q]));
    *dev = T.dev.p + (size_t)q * T.slot_bytes;
    *host = T.host.p + (size_t)q * T.slot_bytes;
    *slot = q;
    return TP_OK;
}

// x[m] = C^+ b[m] for k columns (row stride k) of every problem; b[m] is overwritten with
// its per-component mean-zero projection.  Iteration counts and final relative residuals
// go to the pinned mirrors at offset which * kMaxCols (read them after a sync).
tp_status enqueue_cg(const Batch& B, double* const* b, double* const* x, int k, int which, bool warm = false)
{
    if (B.empty()) return TP_OK;
    hipStream_t s = B[0]->stream;
    std::vector<size_t> pc, ml, plain;
    for (size_t m = 0; m < B.size(); ++m) {
        tp_problem* P = B[m];
        TP_TRY(ensure_cotan(P));
        TP_TRY(ensure_cg(P, k));
        TP_HIP(launch_project_mean(b[m], k, k, P->nV, P->comp.p, P->npins ? P->inv_count_pin.p : P->inv_count.p,
                                   P->ncomp, P->red.p, s));
        if (P->npins) TP_HIP(launch_zero_pinned(b[m], k, k, P->nV, P->pin_mask.p, s));
        if (P->have_pcg && P->pcg_ml) ml.push_back(m);
        else (P->have_pcg ? pc : plain).push_back(m);
    }
    // multi-launch solves (one problem at a time; each call returns after its solve)
    for (size_t m : ml) {
        tp_problem* P = B[m];
        PcgMlWork w;
        w.r = P->ml_r.p; w.p = P->ml_p.p; w.s = P->ml_s.p; w.m = P->ml_m.p; w.an = P->ml_an.p; w.v = P->ml_v.p;
        w.shares = P->ml_shares.p; w.g = P->ml_g.p; w.part = P->ml_part.p;
        w.state = P->ml_state.p; w.state_host = P->ml_state_host.p;
        for (int c0 = 0; c0 < k; c0 += kMaxGroupCols) {
            const int kc = std::min(kMaxGroupCols, k - c0);
            TP_HIP(launch_permute_rows(P->nV, kc, P->pcg.perm, k, c0, b[m], P->pcg_bp.p, true, s));
            TP_HIP(launch_pcg_ml(P->pcg, P->pcg_bp.p, P->pcg_xp.p, kc, P->prm.cg_rtol, P->prm.cg_maxiter, w,
                                 P->cg_iters.p + c0, P->cg_relres.p + c0, s));
            TP_HIP(launch_permute_rows(P->nV, kc, P->pcg.perm, k, c0, P->pcg_xp.p, x[m], false, s));
        }
    }
    if (!pc.empty()) {
        // the problems are grouped into cooperative launches in this order and each launch
        // lasts as long as its slowest problem: order them by their last solve's iteration
        // count (then by size), so that problems of like length share a launch
        std::stable_sort(pc.begin(), pc.end(), [&](size_t a, size_t b) {
            const tp_problem* A = B[a];
            const tp_problem* Q = B[b];
            if (A->last_iters != Q->last_iters) return A->last_iters > Q->last_iters;
            return A->pcg.nb > Q->pcg.nb;
        });
        std::vector<PcgItem> items(pc.size());
        for (int c0 = 0; c0 < k; c0 += kMaxGroupCols) {
            const int kc = std::min(kMaxGroupCols, k - c0);
            for (size_t q = 0; q < pc.size(); ++q) {
                tp_problem* P = B[pc[q]];
                TP_HIP(launch_permute_rows(P->nV, kc, P->pcg.perm, k, c0, b[pc[q]], P->pcg_bp.p, true, s));
                PcgItem& it = items[q];
                it.ps = &P->pcg;
                it.b = P->pcg_bp.p;
                it.x = P->pcg_xp.p;
                // warm start: x[m] still holds this solve's solution of the last step
                it.warm = warm && P->warm_now ? 1 : 0;
                if (it.warm)
                    TP_HIP(launch_permute_rows(P->nV, kc, P->pcg.perm, k, c0, x[pc[q]], P->pcg_xp.p, true, s));
                it.w.Vb = P->pcg_Vb.p; it.w.rho = P->pcg_rho.p; it.w.red = P->pcg_red.p;
                it.w.bar = P->cg_bar.p; it.w.flags = P->flags.p;
                it.w.iters = P->cg_iters.p + c0;
                it.w.relres = P->cg_relres.p + c0;
                it.rtol = P->prm.cg_rtol;
                it.maxiter = P->prm.cg_maxiter;
            }
            void *tdev = nullptr, *thost = nullptr;
            int slot = 0;
            TP_TRY(pcg_table_slot(B[0], (int)items.size(), &tdev, &thost, &slot));
            TP_HIP(launch_pcg_batch(items.data(), (int)items.size(), kc, tdev, thost, s));
            TP_HIP(hipEventRecord(B[0]->tab.ev[slot], s));
            B[0]->tab.used[slot] = true;
            for (size_t q = 0; q < pc.size(); ++q) {
                tp_problem* P = B[pc[q]];
                TP_HIP(launch_permute_rows(P->nV, kc, P->pcg.perm, k, c0, P->pcg_xp.p, x[pc[q]], false, s));
            }
        }
    }
    for (size_t m : plain) {
        tp_problem* P = B[m];
        CgWork w;
        w.Z = P->cg_Z.p; w.p = P->cg_p.p; w.red = P->cg_red.p; w.bar = P->cg_bar.p;
        w.iters = P->cg_iters.p; w.relres = P->cg_relres.p; w.flags = P->flags.p;
        TP_HIP(launch_cg(P->nV, P->ell_col.p, P->ell_val.p, P->ell_w, b[m], x[m], k, P->prm.cg_rtol,
                         P->prm.cg_maxiter, w, s));
    }
    for (size_t m = 0; m < B.size(); ++m) {
        tp_problem* P = B[m];
        TP_HIP(launch_project_mean(x[m], k, k, P->nV, P->comp.p, P->npins ? P->inv_count_pin.p : P->inv_count.p,
                                   P->ncomp, P->red.p, s));
        // the pinned rows are exactly zero (the coarse correction of the preconditioner
        // leaves rounding-level values there)
        if (P->npins) TP_HIP(launch_zero_pinned(x[m], k, k, P->nV, P->pin_mask.p, s));
        TP_HIP(hipMemcpyAsync(P->hiters.p + which * kMaxCols, P->cg_iters.p, sizeof(int) * k,
                              hipMemcpyDeviceToHost, s));
        TP_HIP(hipMemcpyAsync(P->hrelres.p + which * kMaxCols, P->cg_relres.p, sizeof(double) * k,
                              hipMemcpyDeviceToHost, s));
    }
    return TP_OK;
}

// Largest iteration count and relative residual of solve `which` (after a sync).
tp_status cg_result(tp_problem* P, int k, int which, int* it_max, double* res_max)
{
    int im = 0;
    double rm = 0;
    for (int c = 0; c < k; ++c) {
        im = std::max(im, P->hiters.p[which * kMaxCols + c]);
        const double r = P->hrelres.p[which * kMaxCols + c];
        rm = (r > rm || std::isnan(r)) ? r : rm;
    }
    *it_max = im;
    *res_max = rm;
    P->last_iters = im;
    // the solvers test |r|^2 <= rtol^2 |b|^2; the reported sqrt may round one ulp above rtol
    if (!(rm <= P->prm.cg_rtol * (1.0 + 1e-12)))
        return fail(TP_E_NOT_CONVERGED, "CG did not reach cg_rtol within cg_maxiter (relres " + std::to_string(rm) + ")");
    return TP_OK;
}

struct EventTimer {
    hipEvent_t e[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipStream_t s;
    explicit EventTimer(hipStream_t s_) : s(s_)
    {
        for (auto& x : e) (void)hipEventCreate(&x);
    }
    void mark(int i) { (void)hipEventRecord(e[i], s); }
    double ms(int i, int j)
    {
        float v = 0.f;
        (void)hipEventSynchronize(e[j]);
        (void)hipEventElapsedTime(&v, e[i], e[j]);
        return v;
    }
    ~EventTimer()
    {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// Y[m] = A~^{-1} R[m] = C^+ L^sigma C^+ R[m] columnwise (k columns, row stride k); R is
// not modified.  Uses W1, W2 of every problem.
tp_status enqueue_precond(const Batch& B, const double* const* R, int k, double* const* Y,
                          EventTimer* tm, int mark0, bool warm = false)
{
    if (B.empty()) return TP_OK;
    hipStream_t s = B[0]->stream;
    const size_t nb = B.size();
    std::vector<double*> w1(nb), w2(nb);
    std::vector<const double*> w2c(nb);
    for (size_t m = 0; m < nb; ++m) {
        tp_problem* P = B[m];
        const size_t nk = (size_t)P->nV * k;
        TP_TRY(P->W1.ensure(nk, s));
        TP_TRY(P->W2.ensure(nk, s));
        TP_HIP(hipMemcpyAsync(P->W1.p, R[m], nk * sizeof(double), hipMemcpyDeviceToDevice, s));
        w1[m] = P->W1.p;
        w2[m] = P->W2.p;
        w2c[m] = P->W2.p;
    }
    TP_TRY(enqueue_cg(B, w1.data(), w2.data(), k, 0, warm));      // W2 = C^+ P R
    if (tm) tm->mark(mark0);
    TP_TRY(enqueue_fractional(B, w2c.data(), k, k, w1.data(), k));   // W1 = L W2
    if (tm) tm->mark(mark0 + 1);
    TP_TRY(enqueue_cg(B, w1.data(), Y, k, 1, warm));               // Y = C^+ P W1
    // W2 now holds this call's first solution: a later step may start from it only when
    // it came from a step (which then sets warm_cols again)
    for (tp_problem* P : B) P->warm_cols = 0;
    if (tm) tm->mark(mark0 + 2);
    return TP_OK;
}

// ------------------------------------------------------------------ single-problem forms

tp_status run_energy(tp_problem* P, double* E)
{
    const Batch B{P};
    TP_TRY(enqueue_energy(B, kSlotE));
    TP_TRY(enqueue_fetch(B));
    TP_TRY(sync_batch(B));
    TP_TRY(flag_status(P));
    *E = P->hs.p[kSlotE];
    if (!finite(*E)) return fail(TP_E_NONFINITE, "non-finite energy (coincident face barycenters?)");
    return TP_OK;
}

tp_status run_gradient(tp_problem* P, double* E, double* dE)
{
    const Batch B{P};
    TP_TRY(enqueue_gradient(B, &dE, kSlotE));
    TP_TRY(enqueue_fetch(B));
    TP_TRY(sync_batch(B));
    TP_TRY(flag_status(P));
    *E = gradient_energy(P, P->hs.p[kSlotE]);
    if (!finite(*E)) return fail(TP_E_NONFINITE, "non-finite energy (coincident face barycenters?)");
    return TP_OK;
}

// Lu[:, c] for columns of u (row stride ldu) into Lu (row stride ldl), k columns.
tp_status run_fractional(tp_problem* P, const double* u, int ldu, int k, double* Lu, int ldl)
{
    const Batch B{P};
    return enqueue_fractional(B, &u, ldu, k, &Lu, ldl);
}

// Au = (B + B0) u for columns of u (row stride ldu) into Au (row stride ldo), in groups of
// kSobCols columns (one pair launch per group).
tp_status run_sobolev(tp_problem* P, const double* u, int ldu, int k, double* Au, int ldo)
{
    hipStream_t s = P->stream;
    const int prec = P->prm.precision;
    TP_TRY(ensure_vf(P));
    // order of the operator: 2s with s = (beta - 2) / alpha, the order of the energy's differential
    const double sexp = (P->prm.beta - 2.0) / P->prm.alpha;
    for (int c0 = 0; c0 < k; c0 += kSobCols) {
        const int kc = std::min(kSobCols, k - c0);
        SobolevCall c;
        c.fd = &P->fd;
        c.plan = sobolev_plan(prec, kc, P->nF, P->cap);
        c.precision = prec;
        c.s = sexp;
        c.V = P->V.p;
        c.F = P->F.p;
        c.nV = P->nV;
        c.nF = P->nF;
        c.vf_off = P->vf_off.p;
        c.vf_idx = P->vf_idx.p;
        TP_TRY(P->ub.ensure(sobolev_face_bytes(prec, kc, P->cap), s));
        TP_TRY(P->zbuf.ensure((size_t)4 * kc * c.plan.irows, s));
        if (sym_sobolev_eligible(P->prm, P->nF)) {
            // symmetric pair kernel, 4 kc sums per face and slice, in bands of rows
            c.sym_band = sym_band_height(P->prm, P->nF, 4 * kc);
            TP_TRY(P->symp.ensure(sym_part_floats(P->nF, 4 * kc, c.sym_band), s));
            c.symp = P->symp.p;
        } else {
            TP_TRY(P->part.ensure((size_t)c.plan.n_split * 4 * kc * c.plan.irows, s));
            c.part = P->part.p;
        }
        c.fu = P->ub.p;
        c.z = P->zbuf.p;
        const double pairs = (double)P->nF * (double)(P->nF - 1);
        PairTimer t(kKindSobolev, pairs, pairs * kc, s);
        TP_HIP(launch_sobolev(c, u, ldu, kc, Au, ldo, c0, t.on ? t.a : nullptr, t.on ? t.b : nullptr, s));
        t.stopped = t.on;   // launch_sobolev recorded both events around the pair kernel
    }
    return TP_OK;
}

// x = A^+ P b columnwise by right-preconditioned GMRES(m) on A = B + B0 with the
// preconditioner A~^{-1} of Sec. 5.2 and a zero initial guess (Sec. 5.4).  The
// preconditioner is applied through CG solves, so the directions it returns are kept (Z)
// and the solution is formed from them (the flexible form of GMRES).  The k columns run in
// lockstep, each with its own Krylov space, Hessenberg matrix and stopping test; classical
// Gram-Schmidt with one re-orthogonalization pass.  A cycle ends after m iterations or when
// every column's residual estimate is below rtol; the true residual P b - A x is then
// formed, and a new cycle starts from it unless it is below rtol or maxiter iterations have
// been spent.
//
// A annihilates the constants, and with several connected components only the global ones:
// the low-order term B0 couples the components (ubar(S) - ubar(T) = 1 across two of them),
// while the preconditioner annihilates each component's constants.  So P here subtracts the
// global mean, and with 2..kGmCoarseMax components the preconditioner gains the coarse term
// Q G^+ Q^T on the component indicators Q (G = Q^T A Q, inverted on the complement of the
// global constant as G + tr(G)/nc e e^T): the relative translations of the components are
// then solved for exactly.  With more components than that, P subtracts every component's
// mean and the solve is the Galerkin one on that subspace (no relative translations).
//
// precond = 1 adds omega diag(A)^{-1} to the preconditioner.  A~^{-1} alone under-weights
// the highest frequencies, where the face averages of L^sigma lose them (the spread of the
// eigenvalues of A~^{-1} A grows about fourfold per halving of the edge length), while the
// diagonal of A is accurate exactly there; omega matches the two on smooth functions:
// omega = w^T A~^{-1} w / w^T v with w = A v, v the coordinate functions (averaged over
// the three).  The diagonal is taken without the pairs of faces that share the vertex.
constexpr int kGmCoarseMax = 16;
//
// The preconditioner's Poisson solves run to kGmInnerRtol (or the problem's cg_rtol if
// looser): the flexible form forms the residual with the directions the preconditioner
// actually returned, so their accuracy changes the rate of convergence, not the solution's
// (on torus40k to 1e-6: 18 iterations with inner tolerances from 1e-10 to 1e-3, and 37 %
// less time at 1e-3).
constexpr double kGmInnerRtol = 1e-3;

struct CgRtolGuard {   // the CG tolerance of a problem, restored on every exit path
    tp_problem* P;
    double saved;
    CgRtolGuard(tp_problem* P_, double r) : P(P_), saved(P_->prm.cg_rtol) { P->prm.cg_rtol = std::max(saved, r); }
    ~CgRtolGuard() { P->prm.cg_rtol = saved; }
};

tp_status run_precond(tp_problem* P, const double* b, int k, double* x, tp_solve_report* rep);

tp_status run_sobolev_solve(tp_problem* P, const double* b, int k, double rtol, int m, int maxiter, int precond,
                            double* x, tp_gmres_report* rep)
{
    hipStream_t s = P->stream;
    TP_TRY(ensure_geometry(P));
    TP_TRY(ensure_lap(P));
    TP_TRY(ensure_vf(P));
    const int64_t n = P->nV;
    const size_t nk = (size_t)n * k;
    const int64_t vs = (int64_t)nk;
    TP_TRY(P->gm_V.ensure((size_t)(m + 1) * nk, s));
    TP_TRY(P->gm_Z.ensure((size_t)m * nk, s));
    TP_TRY(P->gm_w.ensure(nk, s));
    TP_TRY(P->gm_b.ensure(nk, s));
    TP_TRY(P->gm_r.ensure(nk, s));
    TP_TRY(P->gm_x.ensure(nk, s));
    // h1 [(m+1) k], h2 [(m+1) k], norms [k], scale [k], y [m k]
    const size_t o_h1 = 0, o_h2 = (size_t)(m + 1) * k, o_nrm = 2 * (size_t)(m + 1) * k, o_sc = o_nrm + k,
                 o_y = o_sc + k;
    const int nc = P->ncomp;
    const bool coarse = nc > 1 && nc <= kGmCoarseMax;
    const size_t o_cq = o_y + (size_t)m * k, o_cy = o_cq + (size_t)nc * k, o_om = o_cy + (size_t)nc * k;
    TP_TRY(P->gm_small.ensure(o_om + 6, s));
    TP_TRY(P->gm_red.ensure(std::max(krylov_scratch_doubles((m + 1) * k),
                                     project_scratch_doubles(k, P->ncomp)), s));
    double* sm = P->gm_small.p;
    EventTimer tm(s);
    tm.mark(0);
    CgRtolGuard inner(P, kGmInnerRtol);
    std::vector<double> Gchol;   // Cholesky factor (lower, row-major) of G + tr(G)/nc e e^T
    if (coarse) {
        TP_TRY(P->gm_lab0.ensure((size_t)n, s));
        TP_TRY(P->gm_one.ensure(1, s));
        TP_HIP(hipMemsetAsync(P->gm_lab0.p, 0, sizeof(int32_t) * (size_t)n, s));
        const double invn = 1.0 / (double)n;
        TP_HIP(hipMemcpyAsync(P->gm_one.p, &invn, sizeof(double), hipMemcpyHostToDevice, s));
        TP_TRY(P->gm_Q.ensure((size_t)nc * nk, s));
        TP_TRY(P->gm_Qn.ensure((size_t)n * nc, s));
        TP_TRY(P->gm_AQ.ensure((size_t)n * nc, s));
        // gm_Q: nc blocks of n x k, block l the indicator of component l in every column;
        // gm_Qn: one n x nc matrix whose column l is the indicator of component l
        TP_HIP(krylov_indicators(P->comp.p, n, nc, k, P->gm_Q.p, s));
        std::vector<int32_t> lab((size_t)n);
        TP_HIP(hipMemcpyAsync(lab.data(), P->comp.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        std::vector<double> qn((size_t)n * nc, 0.0), aq((size_t)n * nc);
        for (int64_t v = 0; v < n; ++v)
            if (lab[v] >= 0 && lab[v] < nc) qn[(size_t)v * nc + lab[v]] = 1.0;
        TP_HIP(hipMemcpyAsync(P->gm_Qn.p, qn.data(), sizeof(double) * qn.size(), hipMemcpyHostToDevice, s));
        TP_TRY(run_sobolev(P, P->gm_Qn.p, nc, nc, P->gm_AQ.p, nc));
        TP_HIP(hipMemcpyAsync(aq.data(), P->gm_AQ.p, sizeof(double) * aq.size(), hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        std::vector<double> G((size_t)nc * nc, 0.0);   // G[i][l] = q_i^T A q_l, rows in vertex order
        for (int64_t v = 0; v < n; ++v)
            if (lab[v] >= 0 && lab[v] < nc)
                for (int l = 0; l < nc; ++l) G[(size_t)lab[v] * nc + l] += aq[(size_t)v * nc + l];
        double tr = 0.0;
        for (int i = 0; i < nc; ++i) tr += G[(size_t)i * nc + i];
        if (!(tr > 0.0)) return fail(TP_E_NONFINITE, "component coupling matrix is not positive");
        std::vector<double> Gs((size_t)nc * nc);
        for (int i = 0; i < nc; ++i)
            for (int l = 0; l < nc; ++l)
                Gs[(size_t)i * nc + l] = 0.5 * (G[(size_t)i * nc + l] + G[(size_t)l * nc + i]) + tr / nc;
        Gchol.assign((size_t)nc * nc, 0.0);
        for (int i = 0; i < nc; ++i)
            for (int l = 0; l <= i; ++l) {
                double acc = Gs[(size_t)i * nc + l];
                for (int q = 0; q < l; ++q) acc -= Gchol[(size_t)i * nc + q] * Gchol[(size_t)l * nc + q];
                if (i == l) {
                    if (!(acc > 0.0)) return fail(TP_E_NONFINITE, "component coupling matrix is singular");
                    Gchol[(size_t)i * nc + i] = std::sqrt(acc);
                } else {
                    Gchol[(size_t)i * nc + l] = acc / Gchol[(size_t)l * nc + l];
                }
            }
        TP_TRY(P->gm_red.ensure(std::max({krylov_scratch_doubles((m + 1) * k), krylov_scratch_doubles(nc * k),
                                          project_scratch_doubles(k, P->ncomp)}), s));
    }
    double omega = 0.0;
    if (precond == 1) {
        // approximate diagonal: row sums of the two kernel matrices, then the vertex sums
        SobolevCall c;
        c.fd = &P->fd;
        c.plan = sobolev_plan(TP_PREC_FP32_HILO, 1, P->nF, P->cap);
        c.precision = TP_PREC_FP32_HILO;
        c.s = (P->prm.beta - 2.0) / P->prm.alpha;
        c.V = P->V.p;
        c.F = P->F.p;
        c.nV = P->nV;
        c.nF = P->nF;
        c.vf_off = P->vf_off.p;
        c.vf_idx = P->vf_idx.p;
        TP_TRY(P->part.ensure((size_t)c.plan.n_split * 4 * c.plan.irows, s));
        TP_TRY(P->zbuf.ensure((size_t)4 * c.plan.irows, s));
        TP_TRY(P->gm_dinv.ensure((size_t)n, s));
        c.part = P->part.p;
        c.z = P->zbuf.p;
        TP_HIP(launch_sobolev_diag(c, P->gm_dinv.p, s));
        // omega from the coordinate functions
        const size_t n3 = (size_t)n * 3;
        TP_TRY(P->gm_sv.ensure(n3, s));
        TP_TRY(P->gm_sw.ensure(n3, s));
        TP_TRY(P->gm_smw.ensure(n3, s));
        TP_TRY(P->red.ensure(std::max(reduce_scratch_doubles(16), project_scratch_doubles(3, P->ncomp)), s));
        TP_HIP(hipMemcpyAsync(P->gm_sv.p, P->V.p, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        TP_HIP(launch_project_mean(P->gm_sv.p, 3, 3, n, P->comp.p, P->inv_count.p, P->ncomp, P->red.p, s));
        TP_TRY(run_sobolev(P, P->gm_sv.p, 3, 3, P->gm_sw.p, 3));
        tp_solve_report prep;
        TP_TRY(run_precond(P, P->gm_sw.p, 3, P->gm_smw.p, &prep));
        TP_HIP(launch_dot_cols(P->gm_sw.p, 3, P->gm_smw.p, 3, n, 3, P->red.p, sm + o_om, s));
        TP_HIP(launch_dot_cols(P->gm_sw.p, 3, P->gm_sv.p, 3, n, 3, P->red.p, sm + o_om + 3, s));
        double nd[6];
        TP_HIP(hipMemcpyAsync(nd, sm + o_om, sizeof(nd), hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        int cnt = 0;
        for (int q = 0; q < 3; ++q)
            if (nd[3 + q] > 0.0 && nd[q] > 0.0) {
                omega += nd[q] / nd[3 + q];
                ++cnt;
            }
        if (cnt == 0) return fail(TP_E_NONFINITE, "no positive Rayleigh quotient for the diagonal weight");
        omega /= cnt;
    }
    const int32_t* plab = coarse ? P->gm_lab0.p : P->comp.p;
    const double* pinv = coarse ? P->gm_one.p : P->inv_count.p;
    const int pnc = coarse ? 1 : nc;
    auto project = [&](double* v) -> tp_status {
        TP_HIP(launch_project_mean(v, k, k, n, plab, pinv, pnc, P->gm_red.p, s));
        return TP_OK;
    };
    // Z += Q G^+ Q^T V (the coarse term), columnwise
    std::vector<double> qtv((size_t)nc * k), ycoef((size_t)nc * k), tv(nc);
    auto coarse_add = [&](const double* Vj, double* Zj) -> tp_status {
        TP_HIP(krylov_dots(P->gm_Q.p, vs, nc, Vj, n, k, P->gm_red.p, sm + o_cq, s));
        TP_HIP(hipMemcpyAsync(qtv.data(), sm + o_cq, sizeof(double) * nc * k, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        for (int c = 0; c < k; ++c) {
            for (int i = 0; i < nc; ++i) {   // forward substitution
                double acc = qtv[(size_t)i * k + c];
                for (int q = 0; q < i; ++q) acc -= Gchol[(size_t)i * nc + q] * tv[q];
                tv[i] = acc / Gchol[(size_t)i * nc + i];
            }
            for (int i = nc - 1; i >= 0; --i) {   // back substitution with the transpose
                double acc = tv[i];
                for (int q = i + 1; q < nc; ++q) acc -= Gchol[(size_t)q * nc + i] * ycoef[(size_t)q * k + c];
                ycoef[(size_t)i * k + c] = acc / Gchol[(size_t)i * nc + i];
            }
        }
        TP_HIP(hipMemcpyAsync(sm + o_cy, ycoef.data(), sizeof(double) * nc * k, hipMemcpyHostToDevice, s));
        TP_HIP(krylov_combine(Zj, P->gm_Q.p, vs, nc, sm + o_cy, n, k, true, s));
        return TP_OK;
    };
    auto col_norms = [&](const double* v, std::vector<double>& out) -> tp_status {
        TP_HIP(krylov_dots(v, vs, 1, v, n, k, P->gm_red.p, sm + o_nrm, s));
        out.assign(k, 0.0);
        TP_HIP(hipMemcpyAsync(out.data(), sm + o_nrm, sizeof(double) * k, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        for (double& v2 : out) v2 = std::sqrt(std::max(v2, 0.0));
        return TP_OK;
    };
    // P b, its norms, x = 0, r = P b
    TP_HIP(hipMemcpyAsync(P->gm_b.p, b, nk * sizeof(double), hipMemcpyDeviceToDevice, s));
    TP_TRY(project(P->gm_b.p));
    std::vector<double> bnorm, beta, relres(k, 0.0);
    TP_TRY(col_norms(P->gm_b.p, bnorm));
    TP_HIP(hipMemsetAsync(P->gm_x.p, 0, nk * sizeof(double), s));
    TP_HIP(hipMemcpyAsync(P->gm_r.p, P->gm_b.p, nk * sizeof(double), hipMemcpyDeviceToDevice, s));
    beta = bnorm;
    int total = 0, cycles = 0, pc_iters = 0;
    bool converged = false;
    std::vector<double> h1((size_t)(m + 1) * k), h2((size_t)(m + 1) * k), nrm2(k), scale(k), Y((size_t)m * k);
    for (;;) {
        // stopping test on the true residual
        bool all_done = true;
        for (int c = 0; c < k; ++c) {
            relres[c] = bnorm[c] > 0.0 ? beta[c] / bnorm[c] : 0.0;
            if (relres[c] > rtol) all_done = false;
        }
        if (all_done) {
            converged = true;
            break;
        }
        if (total >= maxiter) break;
        ++cycles;
        // V0 = r / beta for the columns still above the tolerance, 0 for the others
        std::vector<char> live(k, 0);
        for (int c = 0; c < k; ++c) {
            live[c] = relres[c] > rtol;
            scale[c] = live[c] ? 1.0 / beta[c] : 0.0;
        }
        TP_HIP(hipMemcpyAsync(sm + o_sc, scale.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        TP_HIP(krylov_scale(P->gm_V.p, P->gm_r.p, sm + o_sc, n, k, s));
        std::vector<std::vector<double>> H(k, std::vector<double>((size_t)(m + 1) * m, 0.0));
        std::vector<std::vector<double>> g(k, std::vector<double>(m + 1, 0.0)), cs(k, std::vector<double>(m, 0.0)),
            sn(k, std::vector<double>(m, 0.0));
        std::vector<int> used(k, 0);
        for (int c = 0; c < k; ++c) g[c][0] = live[c] ? beta[c] : 0.0;
        int j = 0;
        for (; j < m && total < maxiter; ++j) {
            bool any = false;
            for (int c = 0; c < k; ++c) any = any || live[c];
            if (!any) break;
            double* Vj = P->gm_V.p + (size_t)j * nk;
            double* Zj = P->gm_Z.p + (size_t)j * nk;
            tp_solve_report prep;
            TP_TRY(run_precond(P, Vj, k, Zj, &prep));
            pc_iters += prep.cg_iters[0] + prep.cg_iters[1];
            if (precond == 1) {
                TP_HIP(krylov_diag_add(Zj, Vj, P->gm_dinv.p, omega, n, k, s));
                // keep the directions in the solution space (mean zero, per component when
                // the component translations are left out)
                if (!coarse) TP_TRY(project(Zj));
            }
            if (coarse) TP_TRY(coarse_add(Vj, Zj));
            TP_TRY(run_sobolev(P, Zj, k, k, P->gm_w.p, k));
            TP_TRY(project(P->gm_w.p));
            TP_HIP(krylov_dots(P->gm_V.p, vs, j + 1, P->gm_w.p, n, k, P->gm_red.p, sm + o_h1, s));
            TP_HIP(krylov_subtract(P->gm_w.p, P->gm_V.p, vs, j + 1, sm + o_h1, n, k, s));
            TP_HIP(krylov_dots(P->gm_V.p, vs, j + 1, P->gm_w.p, n, k, P->gm_red.p, sm + o_h2, s));
            TP_HIP(krylov_subtract(P->gm_w.p, P->gm_V.p, vs, j + 1, sm + o_h2, n, k, s));
            TP_HIP(krylov_dots(P->gm_w.p, vs, 1, P->gm_w.p, n, k, P->gm_red.p, sm + o_nrm, s));
            TP_HIP(hipMemcpyAsync(h1.data(), sm + o_h1, sizeof(double) * (j + 1) * k, hipMemcpyDeviceToHost, s));
            TP_HIP(hipMemcpyAsync(h2.data(), sm + o_h2, sizeof(double) * (j + 1) * k, hipMemcpyDeviceToHost, s));
            TP_HIP(hipMemcpyAsync(nrm2.data(), sm + o_nrm, sizeof(double) * k, hipMemcpyDeviceToHost, s));
            TP_HIP(hipStreamSynchronize(s));
            ++total;
            for (int c = 0; c < k; ++c) {
                scale[c] = 0.0;
                if (!live[c]) continue;
                double* Hc = H[c].data() + (size_t)j * (m + 1);   // column j, rows 0..j+1
                for (int i = 0; i <= j; ++i) Hc[i] = h1[(size_t)i * k + c] + h2[(size_t)i * k + c];
                const double hn = std::sqrt(std::max(nrm2[c], 0.0));
                Hc[j + 1] = hn;
                for (int i = 0; i < j; ++i) {   // earlier rotations
                    const double a = Hc[i], bb = Hc[i + 1];
                    Hc[i] = cs[c][i] * a + sn[c][i] * bb;
                    Hc[i + 1] = -sn[c][i] * a + cs[c][i] * bb;
                }
                const double den = std::hypot(Hc[j], Hc[j + 1]);
                cs[c][j] = den > 0.0 ? Hc[j] / den : 1.0;
                sn[c][j] = den > 0.0 ? Hc[j + 1] / den : 0.0;
                Hc[j] = den;
                Hc[j + 1] = 0.0;
                g[c][j + 1] = -sn[c][j] * g[c][j];
                g[c][j] = cs[c][j] * g[c][j];
                used[c] = j + 1;
                const double est = std::fabs(g[c][j + 1]);
                if (est <= rtol * bnorm[c] || hn <= 0.0) live[c] = 0;
                else scale[c] = 1.0 / hn;
            }
            TP_HIP(hipMemcpyAsync(sm + o_sc, scale.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
            TP_HIP(krylov_scale(P->gm_V.p + (size_t)(j + 1) * nk, P->gm_w.p, sm + o_sc, n, k, s));
        }
        // y = R^{-1} g per column, x += Z y
        int nv = 0;
        std::fill(Y.begin(), Y.end(), 0.0);
        for (int c = 0; c < k; ++c) {
            const int u = used[c];
            nv = std::max(nv, u);
            for (int i = u - 1; i >= 0; --i) {
                double acc = g[c][i];
                for (int q = i + 1; q < u; ++q) acc -= H[c][(size_t)q * (m + 1) + i] * Y[(size_t)q * k + c];
                const double d = H[c][(size_t)i * (m + 1) + i];
                Y[(size_t)i * k + c] = d != 0.0 ? acc / d : 0.0;
            }
        }
        if (nv > 0) {
            TP_HIP(hipMemcpyAsync(sm + o_y, Y.data(), sizeof(double) * (size_t)nv * k, hipMemcpyHostToDevice, s));
            TP_HIP(krylov_combine(P->gm_x.p, P->gm_Z.p, vs, nv, sm + o_y, n, k, true, s));
        }
        // true residual r = P b - A x
        TP_TRY(run_sobolev(P, P->gm_x.p, k, k, P->gm_w.p, k));
        TP_TRY(project(P->gm_w.p));
        for (int c = 0; c < k; ++c) scale[c] = 1.0;
        TP_HIP(hipMemcpyAsync(sm + o_sc, scale.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        TP_HIP(hipMemcpyAsync(P->gm_r.p, P->gm_b.p, nk * sizeof(double), hipMemcpyDeviceToDevice, s));
        TP_HIP(krylov_subtract(P->gm_r.p, P->gm_w.p, vs, 1, sm + o_sc, n, k, s));
        TP_TRY(col_norms(P->gm_r.p, beta));
        if (nv == 0) {   // no progress possible (every column stopped on a breakdown)
            for (int c = 0; c < k; ++c) relres[c] = bnorm[c] > 0.0 ? beta[c] / bnorm[c] : 0.0;
            break;
        }
    }
    TP_TRY(project(P->gm_x.p));   // the representative with mean zero
    TP_HIP(hipMemcpyAsync(x, P->gm_x.p, nk * sizeof(double), hipMemcpyDeviceToDevice, s));
    tm.mark(1);
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->iters = total;
        rep->cycles = cycles;
        rep->relres = *std::max_element(relres.begin(), relres.end());
        rep->precond_cg_iters = pc_iters;
        rep->t_ms = tm.ms(0, 1);
        rep->omega = omega;
    }
    TP_HIP(hipStreamSynchronize(s));
    if (!converged) return fail(TP_E_NOT_CONVERGED, "GMRES did not reach the tolerance within maxiter iterations");
    return TP_OK;
}

// x = C^+ b for k columns (row stride k); b is overwritten with its projection.
tp_status run_cg(tp_problem* P, double* b, double* x, int k, int* it_max, double* res_max)
{
    const Batch B{P};
    TP_TRY(enqueue_cg(B, &b, &x, k, 0));
    TP_TRY(enqueue_fetch(B));
    TP_TRY(sync_batch(B));
    TP_TRY(flag_status(P));
    return cg_result(P, k, 0, it_max, res_max);
}

// x = A~^{-1} b columnwise, k columns, row stride k.  b is not modified.
tp_status run_precond(tp_problem* P, const double* b, int k, double* x, tp_solve_report* rep)
{
    TP_TRY(ensure_geometry(P));
    TP_TRY(ensure_lap(P));
    const Batch B{P};
    EventTimer tm(P->stream);
    tm.mark(0);
    TP_TRY(enqueue_precond(B, &b, k, &x, &tm, 1));
    TP_TRY(enqueue_fetch(B));
    TP_TRY(sync_batch(B));
    TP_TRY(flag_status(P));
    int it1 = 0, it2 = 0;
    double r1 = 0, r2 = 0;
    const tp_status st1 = cg_result(P, k, 0, &it1, &r1);
    const tp_status st2 = cg_result(P, k, 1, &it2, &r2);
    if (rep) {
        rep->cg_iters[0] = it1;
        rep->cg_iters[1] = it2;
        rep->cg_relres[0] = r1;
        rep->cg_relres[1] = r2;
        rep->t_ms[0] = tm.ms(0, 1);
        rep->t_ms[1] = tm.ms(1, 2);
        rep->t_ms[2] = tm.ms(2, 3);
        rep->t_ms[3] = tm.ms(0, 3);
    }
    if (st1 != TP_OK) return st1;
    return st2;
}

tp_status create_problem(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                         const tp_params* params, hipStream_t stream, tp_problem** out)
{
    if (!out) return fail(TP_E_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (!V || !F) return fail(TP_E_INVALID_ARGUMENT, "V and F must be non-NULL device pointers");
    if (nV < 3 || nF < 2) return fail(TP_E_INVALID_ARGUMENT, "need nV >= 3 and nF >= 2");
    if (nF > (int64_t)(INT32_MAX / 8) || nV > (int64_t)(INT32_MAX / 8))
        return fail(TP_E_INVALID_ARGUMENT, "mesh too large for 32-bit indices");
    auto* P = new tp_problem();
    tp_status st = validate_params(params, P->prm, P->sigma);
    if (st != TP_OK) {
        delete P;
        return st;
    }
    (void)hipGetDevice(&P->device);
    P->stream = stream;
    P->nV = nV;
    P->nF = nF;
    auto bail = [&](tp_status s) {
        (void)hipStreamSynchronize(P->stream);
        delete P;
        return s;
    };
    if ((st = P->V.ensure(3 * nV, stream)) != TP_OK) return bail(st);
    if ((st = P->F.ensure(3 * nF, stream)) != TP_OK) return bail(st);
    if ((st = alloc_faces(P)) != TP_OK) return bail(st);
    if (hipMemcpyAsync(P->V.p, V, sizeof(double) * 3 * nV, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(P->F.p, F, sizeof(int32_t) * 3 * nF, hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return bail(fail(TP_E_DEVICE, "copy of V / F failed (are they device pointers?)"));
    if (launch_check_indices(P->F.p, nF, nV, P->flags.p, stream) != hipSuccess)
        return bail(fail(TP_E_DEVICE, "index check launch failed"));
    if ((st = check_flags(P)) != TP_OK) return bail(st);
    if ((st = geometry(P)) != TP_OK) return bail(st);
    // store the faces in the Morton order of their barycenters: face tiles become compact
    // patches (the near-field tile test and the tree build rely on it); results do not
    // depend on the stored order beyond rounding, and the tree breaks ties by the caller's
    // face numbers
    {
        DevBuf<int32_t> Fold;
        if ((st = ensure_bh(P)) != TP_OK) return bail(st);
        if ((st = Fold.ensure(3 * nF, stream)) != TP_OK) return bail(st);
        if ((st = P->face_orig.ensure(nF, stream)) != TP_OK) return bail(st);
        if (hipMemcpyAsync(Fold.p, P->F.p, sizeof(int32_t) * 3 * nF, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
            launch_morton_order(P->bh, P->fd, nF, nullptr, stream) != hipSuccess)
            return bail(fail(TP_E_DEVICE, "face ordering failed"));
        hipLaunchKernelGGL(k_permute_faces, dim3((unsigned)((nF + 255) / 256)), dim3(256), 0, stream, Fold.p,
                           P->bh.order, nF, P->F.p, P->face_orig.p);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
            return bail(fail(TP_E_DEVICE, "face ordering failed"));
        P->geom_valid = false;
        if ((st = geometry(P)) != TP_OK) return bail(st);
    }
    if (P->prm.precision == TP_PREC_FP32_NEAR64) {
        if ((st = P->edge.ensure(P->nF, stream)) != TP_OK) return bail(st);
        hipLaunchKernelGGL(k_face_edges, dim3((unsigned)((nF + 255) / 256)), dim3(256), 0, stream, P->V.p, P->F.p,
                           nF, P->edge.p);
        double es = 0;
        if (hipGetLastError() != hipSuccess) return bail(fail(TP_E_DEVICE, "edge length launch failed"));
        if ((st = device_sum(P, P->edge.p, 1, nF, &es)) != TP_OK) return bail(st);
        const double h = es / (3.0 * (double)nF);
        P->rho2 = 4.0 * h * h;
    }
    *out = P;
    return TP_OK;
}

// Initial area, volume and mean edge length (targets and default step of the descent step).
tp_status ensure_initial_measures(tp_problem* P)
{
    if (P->mean_edge > 0) return TP_OK;
    TP_TRY(ensure_geometry(P));
    TP_TRY(total_area_volume(P, P->V.p, &P->area0, &P->vol0));
    TP_TRY(P->edge.ensure(P->nF, P->stream));
    hipLaunchKernelGGL(k_face_edges, dim3((unsigned)((P->nF + 255) / 256)), dim3(256), 0, P->stream,
                       P->V.p, P->F.p, P->nF, P->edge.p);
    TP_HIP(hipGetLastError());
    double es = 0;
    TP_TRY(device_sum(P, P->edge.p, 1, P->nF, &es));
    P->mean_edge = es / (3.0 * (double)P->nF);
    return TP_OK;
}

struct HostSolve2 {
    // solve the k x k system S z = r (k <= 2)
    static bool solve(int k, const double S[4], const double* r, double* z)
    {
        if (k == 0) return true;
        if (k == 1) {
            if (!(std::fabs(S[0]) > 0)) return false;
            z[0] = r[0] / S[0];
            return std::isfinite(z[0]);
        }
        const double det = S[0] * S[3] - S[1] * S[2];
        const double scale = std::fabs(S[0] * S[3]) + std::fabs(S[1] * S[2]);
        if (!(std::fabs(det) > 1e-14 * scale)) return false;
        z[0] = (S[3] * r[0] - S[1] * r[1]) / det;
        z[1] = (S[0] * r[1] - S[2] * r[0]) / det;
        return std::isfinite(z[0]) && std::isfinite(z[1]);
    }
};

// ------------------------------------------------------------------ descent step
//
// One constrained, preconditioned descent step (Sec. 3 and Sec. 5.4 with A~^{-1} in place
// of the GMRES solve): g = dE; Y = A~^{-1}[g | J_A^T | J_V^T]; Schur system S = J Y; direction
// x = -(y_g - Y S^{-1} J y_g); Armijo line search on E(f + tau x); corrective projection
// f <- f + tau x - Y S^{-1} Phi(f + tau x) (Sec. 3.3.2, Sec. 5.3.1).

// Obstacle potential at the current face data into slot kSlotObs, and its face partials in
// obs_g ([7][nF], for launch_grad_gather).
tp_status enqueue_obstacle(tp_problem* P)
{
    hipStream_t s = P->stream;
    TP_TRY(P->obs_e.ensure((size_t)P->nF, s));
    TP_TRY(P->obs_g.ensure((size_t)7 * P->nF, s));
    if (P->obs_tree.built)
        TP_HIP(launch_obstacle_bh(P->fd.dx, P->nF, P->obs_x.p, P->obs_tree.view, P->obs_n, P->prm.leaf_size,
                                  P->prm.theta, P->obs_p, P->obs_e.p, P->obs_g.p, P->nF, P->obs_tree.counts.p, s));
    else
        TP_HIP(launch_obstacle_pairs(P->fd.dx, P->nF, P->obs_x.p, P->obs_cap, P->obs_p, P->obs_e.p, P->obs_g.p, P->nF, s));
    TP_HIP(launch_dot_cols(P->obs_e.p, 1, nullptr, 0, P->nF, 1, P->red.p, P->scal.p + kSlotObs, s));
    return TP_OK;
}

// Implicit potentials at the current face data into slot kSlotImp, face partials in imp_g.
tp_status enqueue_implicit(tp_problem* P)
{
    hipStream_t s = P->stream;
    TP_TRY(P->imp_e.ensure((size_t)P->nF, s));
    TP_TRY(P->imp_g.ensure((size_t)7 * P->nF, s));
    TP_HIP(launch_implicit(P->fd.dx, P->nF, P->imp, P->imp_e.p, P->imp_g.p, P->nF, s));
    TP_HIP(launch_dot_cols(P->imp_e.p, 1, nullptr, 0, P->nF, 1, P->red.p, P->scal.p + kSlotImp, s));
    return TP_OK;
}

struct StepState {
    tp_problem* P = nullptr;
    tp_step_opts o;
    double A0 = 0, V0 = 0;
    int kc = 0, ncol = 3;
    double E0 = 0, Sm[4] = {0, 0, 0, 0}, mu[2] = {0, 0};
    double tau = 0;
    int bt = 0;
    tp_step_report R;
    tp_status st = TP_OK;
    double* dir_out = nullptr;
    bool alive() const { return st == TP_OK || st == TP_E_NOT_CONVERGED; }
    bool penalized() const { return o.area_penalty > 0.0 || o.volume_penalty > 0.0; }
    bool obstacle() const { return P->obs_w > 0.0 && P->obs_n > 0; }
    bool implicit() const { return P->imp.n > 0; }
    // weighted mesh-obstacle and implicit potentials from the fetched slots
    double extra(const double* hs) const
    {
        return (obstacle() ? P->obs_w * hs[kSlotObs] : 0.0) + (implicit() ? hs[kSlotImp] : 0.0);
    }
    // w_A (A / A0 - 1)^2 + w_V (V / V0 - 1)^2 (Sec. 7.3.1), A and V the total area and volume
    double penalty(double area, double vol) const
    {
        double e = 0.0;
        if (o.area_penalty > 0.0) e += o.area_penalty * (area / A0 - 1.0) * (area / A0 - 1.0);
        if (o.volume_penalty > 0.0) e += o.volume_penalty * (vol / V0 - 1.0) * (vol / V0 - 1.0);
        return e;
    }
    double pen0 = 0.0;   // the penalty at the start of the step
};

// Area and six times the signed volume at Vsrc (the face data must describe Vsrc).
tp_status enqueue_area_volume(tp_problem* P, const double* Vsrc)
{
    hipStream_t s = P->stream;
    TP_HIP(launch_dot_cols(&P->dx.p[0].w, 4, nullptr, 0, P->nF, 1, P->red.p, P->scal.p + kSlotArea, s));
    TP_TRY(P->vol6.ensure(P->nF, s));
    TP_HIP(launch_face_volume(Vsrc, P->F.p, P->nF, P->vol6.p, s));
    TP_HIP(launch_dot_cols(P->vol6.p, 1, nullptr, 0, P->nF, 1, P->red.p, P->scal.p + kSlotVol6, s));
    return TP_OK;
}

void constraint_values(const StepState& S, const double* hs, double* phi)
{
    int m = 0;
    if (S.o.constrain_area) phi[m++] = hs[kSlotArea] - S.A0;
    if (S.o.constrain_volume) phi[m++] = hs[kSlotVol6] / 6.0 - S.V0;
}

// The problems of G share a stream, precision, exponents, sigma and column count.
tp_status run_sobolev_solve(tp_problem* P, const double* b, int k, double rtol, int m, int maxiter, int precond,
                            double* x, tp_gmres_report* rep);

tp_status step_group(std::vector<StepState*>& G)
{
    Batch B;
    for (StepState* S : G) B.push_back(S->P);
    hipStream_t s = B[0]->stream;
    const int ncol = G[0]->ncol;
    EventTimer tm(s);
    for (StepState* S : G) {
        tp_problem* P = S->P;
        const size_t n = (size_t)P->nV;
        TP_TRY(P->R.ensure(n * ncol, s));
        TP_TRY(P->Y.ensure(n * ncol, s));
        TP_TRY(P->gbuf.ensure(n * 3, s));
        TP_TRY(P->dir.ensure(n * 3, s));
        TP_TRY(P->Vt.ensure(n * 3, s));
    }
    // 1. g = dE (all problems in one all-pairs launch)
    tm.mark(0);
    {
        std::vector<double*> gp;
        for (tp_problem* P : B) gp.push_back(P->gbuf.p);
        TP_TRY(enqueue_gradient(B, gp.data(), kSlotE));
    }
    // 1b. penalty potentials (Sec. 7.3.1): their gradients are added to g,
    //     2 w_A (A / A0 - 1) / A0 dA + 2 w_V (V / V0 - 1) / V0 dV
    {
        Batch BP;
        for (StepState* S : G) {
            if (S->penalized()) TP_TRY(enqueue_area_volume(S->P, S->P->V.p));   // face data describes V
            if (S->obstacle()) TP_TRY(enqueue_obstacle(S->P));
            if (S->implicit()) TP_TRY(enqueue_implicit(S->P));
            if (S->penalized() || S->obstacle() || S->implicit()) BP.push_back(S->P);
        }
        if (!BP.empty()) {
            TP_TRY(enqueue_fetch(BP));
            TP_TRY(sync_batch(BP));
        }
        for (StepState* S : G) {
            tp_problem* P = S->P;
            const int64_t n = P->nV;
            if (S->obstacle()) {   // w E_obs and its differential w dE_obs
                const double w = P->obs_w;
                const int c0 = 0;
                S->pen0 += w * P->hs.p[kSlotObs];
                TP_HIP(launch_grad_gather(P->V.p, P->F.p, n, P->nF, P->vf_off.p, P->vf_idx.p, P->obs_g.p, P->nF,
                                          P->Vt.p, s));
                TP_HIP(launch_axpy_block3(n, P->gbuf.p, 3, 1.0, P->Vt.p, 3, 1, &w, &c0, P->gbuf.p, 3, s));
            }
            if (S->implicit()) {   // the implicit potentials (weights applied in the kernel)
                const double one = 1.0;
                const int c0 = 0;
                S->pen0 += P->hs.p[kSlotImp];
                TP_HIP(launch_grad_gather(P->V.p, P->F.p, n, P->nF, P->vf_off.p, P->vf_idx.p, P->imp_g.p, P->nF,
                                          P->Vt.p, s));
                TP_HIP(launch_axpy_block3(n, P->gbuf.p, 3, 1.0, P->Vt.p, 3, 1, &one, &c0, P->gbuf.p, 3, s));
            }
            if (!S->penalized()) continue;
            const double area = P->hs.p[kSlotArea], vol = P->hs.p[kSlotVol6] / 6.0;
            S->pen0 += S->penalty(area, vol);
            const int c0 = 0;
            if (S->o.area_penalty > 0.0) {
                const double cA = 2.0 * S->o.area_penalty * (area / S->A0 - 1.0) / S->A0;
                TP_TRY(ensure_cotan(P));
                TP_HIP(launch_spmm(n, P->lap_off.p, P->lap_col.p, P->lap_val.p, P->V.p, 3, 3, P->Y.p, 3, s));
                TP_HIP(launch_axpy_block3(n, P->gbuf.p, 3, 1.0, P->Y.p, 3, 1, &cA, &c0, P->gbuf.p, 3, s));
            }
            if (S->o.volume_penalty > 0.0) {
                const double cV = 2.0 * S->o.volume_penalty * (vol / S->V0 - 1.0) / S->V0;
                TP_HIP(launch_volume_gradient(P->V.p, P->F.p, n, P->vf_off.p, P->vf_idx.p, P->Vt.p, 3, 0, s));
                TP_HIP(launch_axpy_block3(n, P->gbuf.p, 3, 1.0, P->Vt.p, 3, 1, &cV, &c0, P->gbuf.p, 3, s));
            }
        }
    }
    // 2. right-hand sides: g, area gradient C f (twice the mean curvature normal), volume
    //    gradient
    for (StepState* S : G) {
        tp_problem* P = S->P;
        const int64_t n = P->nV;
        TP_TRY(ensure_cotan(P));   // joins the set-up started with the step
        TP_HIP(launch_copy_cols(n, P->gbuf.p, 3, 3, P->R.p, ncol, s));
        int col = 3;
        if (S->o.constrain_area) {
            TP_HIP(launch_spmm(n, P->lap_off.p, P->lap_col.p, P->lap_val.p, P->V.p, 3, 3, P->R.p + col, ncol, s));
            col += 3;
        }
        if (S->o.constrain_volume) {
            TP_HIP(launch_volume_gradient(P->V.p, P->F.p, n, P->vf_off.p, P->vf_idx.p, P->R.p, ncol, col, s));
            col += 3;
        }
    }
    // 3. Y = A~^{-1} R (shared all-pairs and CG launches), or with solver = 1 Y = A^+ R by
    //    GMRES on the true operator, one problem at a time (Sec. 5.4)
    tm.mark(1);
    const bool gmres = G[0]->o.solver == 1;
    std::vector<tp_gmres_report> grep(G.size());
    std::vector<tp_status> gst(G.size(), TP_OK);
    if (gmres) {
        for (size_t q = 0; q < G.size(); ++q) {
            StepState* S = G[q];
            gst[q] = run_sobolev_solve(S->P, S->P->R.p, ncol, S->o.solver_rtol, std::min(50, 1024 / ncol - 1),
                                       S->o.solver_maxiter, 1, S->P->Y.p, &grep[q]);
            if (gst[q] == TP_E_DEVICE) return gst[q];
        }
        tm.mark(2);
        tm.mark(3);
        tm.mark(4);
    } else {
        std::vector<const double*> Rp;
        std::vector<double*> Yp;
        for (StepState* S : G) {
            tp_problem* P = S->P;
            Rp.push_back(P->R.p);
            Yp.push_back(P->Y.p);
            P->warm_now = S->o.warm_start && P->warm_cols == ncol && !S->penalized();
            S->R.warm_started = P->warm_now ? 1 : 0;
        }
        TP_TRY(enqueue_precond(B, Rp.data(), ncol, Yp.data(), &tm, 2, true));
        for (tp_problem* P : B) {
            P->warm_now = false;
            P->warm_cols = ncol;
        }
    }
    // 4. Schur system S = J Y and J y_g (device dot products of 3 columns each)
    for (StepState* S : G) {
        tp_problem* P = S->P;
        const int64_t n = P->nV;
        for (int a = 0; a < S->kc; ++a) {
            for (int b2 = 0; b2 < S->kc; ++b2)
                TP_HIP(launch_dot_cols(P->R.p + 3 * (1 + a), ncol, P->Y.p + 3 * (1 + b2), ncol, n, 3, P->red.p,
                                       P->scal.p + kSlotS + 3 * (2 * a + b2), s));
            TP_HIP(launch_dot_cols(P->R.p + 3 * (1 + a), ncol, P->Y.p, ncol, n, 3, P->red.p,
                                   P->scal.p + kSlotR + 3 * a, s));
        }
    }
    TP_TRY(enqueue_fetch(B));
    TP_TRY(sync_batch(B));
    std::vector<StepState*> L;
    for (StepState* S : G) {
        tp_problem* P = S->P;
        const double* h = P->hs.p;
        if ((S->st = flag_status(P)) != TP_OK) continue;
        S->R.cg_iters[0] = 0;
        if (gmres) {
            // GMRES iterations and true relative residual; CG iterations of its preconditioner
            const size_t q = (size_t)(std::find(G.begin(), G.end(), S) - G.begin());
            S->R.cg_iters[0] = grep[q].iters;
            S->R.cg_relres[0] = grep[q].relres;
            S->R.cg_iters[1] = grep[q].precond_cg_iters;
            S->R.cg_relres[1] = 0.0;
            if (gst[q] != TP_OK) S->st = gst[q];
        } else {
            const tp_status c1 = cg_result(P, ncol, 0, &S->R.cg_iters[0], &S->R.cg_relres[0]);
            const tp_status c2 = cg_result(P, ncol, 1, &S->R.cg_iters[1], &S->R.cg_relres[1]);
            if (c1 != TP_OK) S->st = c1;
            else if (c2 != TP_OK) S->st = c2;
        }
        S->E0 = gradient_energy(P, h[kSlotE]) + S->pen0;
        if (!finite(S->E0)) {
            S->st = fail(TP_E_NONFINITE, "non-finite energy (coincident face barycenters?)");
            continue;
        }
        double rhs[2] = {0, 0};
        for (int a = 0; a < S->kc; ++a) {
            for (int b2 = 0; b2 < S->kc; ++b2) {
                const double* v = h + kSlotS + 3 * (2 * a + b2);
                S->Sm[a * S->kc + b2] = v[0] + v[1] + v[2];
            }
            const double* v = h + kSlotR + 3 * a;
            rhs[a] = v[0] + v[1] + v[2];
        }
        if (!HostSolve2::solve(S->kc, S->Sm, rhs, S->mu)) {
            S->st = fail(TP_E_SINGULAR_CONSTRAINTS, "Schur complement J A~^{-1} J^T is singular");
            continue;
        }
        L.push_back(S);
    }
    // 5. direction x = -(y_g - Y S^{-1} J y_g), slope g.x, default step, constraint values
    for (StepState* S : L) {
        tp_problem* P = S->P;
        const int64_t n = P->nV;
        const double cf[2] = {S->mu[0], S->mu[1]};
        const int cols[2] = {3, 6};
        TP_HIP(launch_axpy_block3(n, P->Y.p, ncol, -1.0, P->Y.p, ncol, S->kc, cf, cols, P->dir.p, 3, s));
        if (S->o.barycenter_motion) {
            // barycenter motions (Sec. 7.1.1): add back to the direction, per component, the
            // translation by minus the vertex-area-weighted mean of g (face data describes V)
            const int nc = P->ncomp;
            TP_TRY(P->bm_area.ensure((size_t)n, s));
            TP_TRY(P->bm_t.ensure((size_t)3 * nc, s));
            TP_HIP(launch_vertex_area(n, P->vf_off.p, P->vf_idx.p, P->fd.dx, P->bm_area.p, s));
            std::vector<double> gh((size_t)3 * n), ah((size_t)n), t((size_t)3 * nc, 0.0), w((size_t)nc, 0.0);
            std::vector<int32_t> lab((size_t)n);
            TP_HIP(hipMemcpyAsync(gh.data(), P->gbuf.p, sizeof(double) * gh.size(), hipMemcpyDeviceToHost, s));
            TP_HIP(hipMemcpyAsync(ah.data(), P->bm_area.p, sizeof(double) * ah.size(), hipMemcpyDeviceToHost, s));
            TP_HIP(hipMemcpyAsync(lab.data(), P->comp.p, sizeof(int32_t) * lab.size(), hipMemcpyDeviceToHost, s));
            TP_HIP(hipStreamSynchronize(s));
            for (int64_t v = 0; v < n; ++v) {   // vertex order: fixed
                const int c = lab[v];
                w[c] += ah[v];
                for (int q = 0; q < 3; ++q) t[3 * c + q] += ah[v] * gh[3 * v + q];
            }
            for (int c = 0; c < nc; ++c)
                for (int q = 0; q < 3; ++q) t[3 * c + q] = w[c] > 0.0 ? -t[3 * c + q] / w[c] : 0.0;
            TP_HIP(hipMemcpyAsync(P->bm_t.p, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice, s));
            TP_HIP(launch_add_translation(P->dir.p, P->comp.p, P->bm_t.p, n, s));
            TP_HIP(hipStreamSynchronize(s));
        }
        TP_HIP(launch_dot_cols(P->gbuf.p, 3, P->gbuf.p, 3, n, 3, P->red.p, P->scal.p + kSlotGG, s));
        TP_HIP(launch_dot_cols(P->gbuf.p, 3, P->dir.p, 3, n, 3, P->red.p, P->scal.p + kSlotGX, s));
        TP_HIP(launch_max_rownorm3(P->dir.p, n, P->red.p, P->scal.p + kSlotMax, s));
        TP_TRY(enqueue_area_volume(P, P->V.p));    // face data describes V
    }
    {
        Batch BL;
        for (StepState* S : L) BL.push_back(S->P);
        if (!BL.empty()) {
            TP_TRY(enqueue_fetch(BL));
            TP_TRY(sync_batch(BL));
        }
    }
    std::vector<StepState*> search;
    for (StepState* S : L) {
        const double* h = S->P->hs.p;
        S->R.E = S->E0;
        S->R.grad_norm = std::sqrt(h[kSlotGG] + h[kSlotGG + 1] + h[kSlotGG + 2]);
        S->R.slope = h[kSlotGX] + h[kSlotGX + 1] + h[kSlotGX + 2];
        S->R.n_constraints = S->kc;
        constraint_values(*S, h, S->R.phi_before);
        S->tau = S->o.tau0;
        if (!(S->tau > 0)) {
            const double mx = h[kSlotMax];
            if (!(mx > 0) || !finite(mx)) {
                S->st = fail(TP_E_NONFINITE, "zero or non-finite descent direction");
                continue;
            }
            S->tau = 0.5 * S->P->mean_edge / mx;
        }
        S->bt = 0;
        search.push_back(S);
    }
    tm.mark(5);

    // 6. Armijo line search on E(f + tau x): one shared energy launch per round over the
    //    problems still searching
    std::vector<StepState*> accepted;
    while (!search.empty()) {
        Batch BS;
        for (StepState* S : search) {
            tp_problem* P = S->P;
            const double cf = S->tau;
            const int c0 = 0;
            TP_HIP(launch_axpy_block3(P->nV, P->V.p, 3, 1.0, P->dir.p, 3, 1, &cf, &c0, P->Vt.p, 3, s));
            TP_HIP(launch_face_geom(P->Vt.p, P->nV, P->F.p, P->nF, P->fd, P->flags.p, s));
            P->fd_V = P->Vt.p;
            ++P->geom_ver;
            P->geom_valid = false;
            if (S->penalized()) TP_TRY(enqueue_area_volume(P, P->Vt.p));
            if (S->obstacle()) TP_TRY(enqueue_obstacle(P));
            if (S->implicit()) TP_TRY(enqueue_implicit(P));
            BS.push_back(P);
        }
        TP_TRY(enqueue_energy(BS, kSlotE));
        TP_TRY(enqueue_fetch(BS));
        TP_TRY(sync_batch(BS));
        std::vector<StepState*> next;
        for (StepState* S : search) {
            tp_problem* P = S->P;
            const tp_status gs = flag_status(P);
            if (gs != TP_OK && gs != TP_E_DEGENERATE_FACE && gs != TP_E_NONFINITE) {
                S->st = gs;
                continue;
            }
            const double Et = P->hs.p[kSlotE] + (S->penalized() ? S->penalty(P->hs.p[kSlotArea], P->hs.p[kSlotVol6] / 6.0) : 0.0) +
                              S->extra(P->hs.p);
            const bool valid = gs == TP_OK && finite(Et);
            const bool ok = valid && (!S->o.line_search || Et <= S->E0 + S->o.armijo_c * S->tau * S->R.slope);
            if (ok || !S->o.line_search) {
                if (!ok) S->st = fail(TP_E_NONFINITE, "the fixed step produces a degenerate mesh");
                else accepted.push_back(S);
                continue;
            }
            if (S->bt >= S->o.max_backtracks) {
                if (!valid) S->st = fail(TP_E_NONFINITE, "line search found no valid step");
                else accepted.push_back(S);
                continue;
            }
            S->tau *= S->o.shrink;
            ++S->bt;
            next.push_back(S);
        }
        search.swap(next);
    }
    tm.mark(6);

    // 7. corrective projection h = -Y S^{-1} Phi(f + tau x) (face data describes f + tau x)
    Batch BA;
    for (StepState* S : accepted) {
        S->R.tau = S->tau;
        S->R.backtracks = S->bt;
        TP_TRY(enqueue_area_volume(S->P, S->P->Vt.p));
        BA.push_back(S->P);
    }
    if (!BA.empty()) {
        TP_TRY(enqueue_fetch(BA));
        TP_TRY(sync_batch(BA));
    }
    Batch BF;
    std::vector<StepState*> fin;
    for (StepState* S : accepted) {
        tp_problem* P = S->P;
        double phi[2] = {0, 0}, lam[2] = {0, 0};
        constraint_values(*S, P->hs.p, phi);
        S->R.phi_trial[0] = phi[0];
        S->R.phi_trial[1] = phi[1];
        if (S->kc > 0 && !HostSolve2::solve(S->kc, S->Sm, phi, lam)) {
            S->st = fail(TP_E_SINGULAR_CONSTRAINTS, "Schur complement is singular");
            continue;
        }
        const double cf[2] = {-lam[0], -lam[1]};
        const int cols[2] = {3, 6};
        TP_HIP(launch_axpy_block3(P->nV, P->Vt.p, 3, 1.0, P->Y.p, ncol, S->kc, cf, cols, P->V.p, 3, s));
        if (S->dir_out)
            TP_HIP(hipMemcpyAsync(S->dir_out, P->dir.p, sizeof(double) * 3 * P->nV, hipMemcpyDeviceToDevice, s));
        P->cotan_valid = false;
        TP_HIP(launch_face_geom(P->V.p, P->nV, P->F.p, P->nF, P->fd, P->flags.p, s));
        P->fd_V = P->V.p;
        ++P->geom_ver;
        TP_TRY(enqueue_area_volume(P, P->V.p));
        if (S->obstacle()) TP_TRY(enqueue_obstacle(P));
        if (S->implicit()) TP_TRY(enqueue_implicit(P));
        BF.push_back(P);
        fin.push_back(S);
    }
    TP_TRY(enqueue_energy(BF, kSlotE));
    tm.mark(7);
    if (!BF.empty()) {
        TP_TRY(enqueue_fetch(BF));
        TP_TRY(sync_batch(BF));
    }
    for (StepState* S : fin) {
        tp_problem* P = S->P;
        const tp_status gs = flag_status(P);
        if (gs != TP_OK) {
            S->st = gs;
            continue;
        }
        P->geom_valid = true;
        constraint_values(*S, P->hs.p, S->R.phi_after);
        S->R.E_new = P->hs.p[kSlotE] + S->penalty(P->hs.p[kSlotArea], P->hs.p[kSlotVol6] / 6.0) +
                     S->extra(P->hs.p);
        // the corrective projection can move a barycenter into an obstacle (or onto
        // another one) after the line search accepted the trial point
        if (!finite(S->R.E_new))
            S->st = fail(TP_E_NONFINITE, "the corrected positions give a non-finite energy (a face inside an obstacle?)");
    }
    // timings of the group (shared by its problems)
    const double t[8] = {tm.ms(0, 1), tm.ms(1, 2), tm.ms(1, 4), tm.ms(4, 5),
                         tm.ms(5, 6), tm.ms(6, 7), tm.ms(0, 7), (double)B.size()};
    for (StepState* S : G)
        for (int q = 0; q < 8; ++q) S->R.t_ms[q] = t[q];
    return TP_OK;
}

// Steps of n problems with shared launches.  Problems are grouped by (precision,
// exponents, sigma, number of constraint rows); each group runs as one batch.
tp_status run_step_batch(tp_problem* const* probs, int n, const tp_step_opts* opts, tp_step_report* reps,
                         tp_status* sts, double* const* dir_out)
{
    if (n < 1 || !probs) return fail(TP_E_INVALID_ARGUMENT, "need at least one problem");
    std::vector<StepState> S(n);
    for (int m = 0; m < n; ++m) {
        if (!probs[m]) return fail(TP_E_INVALID_ARGUMENT, "problem is NULL");
        for (int q = 0; q < m; ++q)
            if (probs[q] == probs[m]) return fail(TP_E_INVALID_ARGUMENT, "a problem appears twice in the batch");
        if (probs[m]->device != probs[0]->device || probs[m]->stream != probs[0]->stream)
            return fail(TP_E_INVALID_ARGUMENT, "the problems of a batch must share device and stream");
    }
    TP_HIP(hipSetDevice(probs[0]->device));
    for (int m = 0; m < n; ++m) {
        StepState& T = S[m];
        T.P = probs[m];
        std::memset(&T.R, 0, sizeof(T.R));
        tp_step_opts_default(&T.o);
        if (opts) T.o = opts[m];
        T.dir_out = dir_out ? dir_out[m] : nullptr;
        if (!(T.o.shrink > 0.0 && T.o.shrink < 1.0)) {
            T.st = fail(TP_E_INVALID_ARGUMENT, "shrink must lie in (0, 1)");
            continue;
        }
        if (T.o.max_backtracks < 0) {
            T.st = fail(TP_E_INVALID_ARGUMENT, "max_backtracks must be >= 0");
            continue;
        }
        if (T.o.barycenter_motion != 0 && T.o.barycenter_motion != 1) {
            T.st = fail(TP_E_INVALID_ARGUMENT, "barycenter_motion must be 0 or 1");
            continue;
        }
        if (T.P->npins > 0 && (T.o.barycenter_motion || T.o.solver != 0)) {
            T.st = fail(TP_E_INVALID_ARGUMENT, "vertex pins combine with neither barycenter motions nor solver = 1");
            continue;
        }
        if (!(T.o.area_penalty >= 0.0) || !(T.o.volume_penalty >= 0.0)) {
            T.st = fail(TP_E_INVALID_ARGUMENT, "penalty weights must be >= 0");
            continue;
        }
        if ((T.o.solver != 0 && T.o.solver != 1) ||
            (T.o.solver == 1 && (!(T.o.solver_rtol > 0.0) || T.o.solver_maxiter < 1))) {
            T.st = fail(TP_E_INVALID_ARGUMENT, "solver must be 0 or 1 (then solver_rtol > 0, solver_maxiter >= 1)");
            continue;
        }
        tp_problem* P = T.P;
        tp_status st = ensure_initial_measures(P);
        if (st == TP_OK) st = ensure_geometry(P);
        if (st == TP_OK) st = ensure_lap(P);
        if (st == TP_OK) st = start_cotan(P);   // beside the energy and differential
        if (st != TP_OK) {
            if (st == TP_E_DEVICE) return st;
            T.st = st;
            continue;
        }
        T.A0 = std::isnan(T.o.area_target) ? P->area0 : T.o.area_target;
        T.V0 = std::isnan(T.o.volume_target) ? P->vol0 : T.o.volume_target;
        // the potentials divide by their targets: a zero (or non-finite) target is an
        // argument error, not a non-finite energy later in the step
        if ((T.o.area_penalty > 0.0 && (!std::isfinite(T.A0) || T.A0 == 0.0)) ||
            (T.o.volume_penalty > 0.0 && (!std::isfinite(T.V0) || T.V0 == 0.0))) {
            T.st = fail(TP_E_INVALID_ARGUMENT,
                        "area_penalty / volume_penalty need a finite, non-zero area / volume target "
                        "(the initial measure is used when the target is NaN)");
            continue;
        }
        T.kc = (T.o.constrain_area ? 1 : 0) + (T.o.constrain_volume ? 1 : 0);
        T.ncol = 3 * (1 + T.kc);
    }
    std::vector<bool> done(n, false);
    for (int m = 0; m < n; ++m) {
        if (done[m] || S[m].st != TP_OK) continue;
        std::vector<StepState*> G;
        for (int q = m; q < n; ++q) {
            if (done[q] || S[q].st != TP_OK) continue;
            const tp_problem* a = S[m].P;
            const tp_problem* b = S[q].P;
            if (a->prm.precision == b->prm.precision && a->prm.alpha == b->prm.alpha &&
                a->prm.beta == b->prm.beta && a->sigma == b->sigma && S[m].ncol == S[q].ncol &&
                a->prm.theta == b->prm.theta && a->prm.leaf_size == b->prm.leaf_size && a->prm.chi == b->prm.chi &&
                S[m].o.solver == S[q].o.solver) {
                G.push_back(&S[q]);
                done[q] = true;
            }
        }
        TP_TRY(step_group(G));
    }
    tp_status first = TP_OK;
    for (int m = 0; m < n; ++m) {
        if (reps) reps[m] = S[m].R;
        if (sts) sts[m] = S[m].st;
        if (first == TP_OK && S[m].st != TP_OK) first = S[m].st;
    }
    return first;
}

// Upper bound of the device memory a problem holds after descent steps with kc active
// constraint rows (the allocations of alloc_faces, ensure_lap, build_pcg, ensure_cg, the
// pair plans and the step's work arrays, with the ELL width max_degree + 1).
uint64_t estimate_bytes(int64_t nV, int64_t nF, int max_degree, int ncomp, const tp_params& prm, int kc)
{
    const double n = (double)nV, f = (double)nF;
    const int64_t cap = face_capacity(nF, 4);
    const int ncol = 3 * (1 + kc);
    const int prec = prm.precision;
    const double w = (double)max_degree + 1.0;
    double b = 0;
    b += 24 * n + 12 * f + (double)cap * (3 * 16 + 2 * 32) + 4 * kNumFlags;
    // incidence, cotan pattern and values, components, ELL
    b += 4 * (n + 1) * 3 + 12 * f + 4 * (6 * f + 1) + 12 * n * w + 4 * n + 8 * ncomp + 12 * n * w;
    // preconditioner
    if (prm.cg_precond) {
        const double nb = std::ceil(n / pcg_block_size()) + ncomp;
        if (nb <= pcg_max_blocks_multi()) {
            const double bs = pcg_block_size(), ncmax = pcg_max_coarse();
            // permutation, ELL pattern / values / entry slots, block and aggregate tables,
            // row slots, coarse functions and row weights, block inverses, coarse inverse
            b += 4 * n + 13 * n * w + 4 * 2 * (nb + 1) + 4 * nb * (4 + pcg_max_block_aggregates()) + 4 * n +
                 (4 + 32 + 8 * 4 * kPcgRowSlots) * n + 8 * ncmax + 4 * nb * bs * bs + 8 * ncmax * ncmax;
            if (nb <= pcg_max_blocks()) {
                // solve work: two copies of the block solves, block shares of the coarse
                // right-hand side and partial sums, permuted b and x
                b += 8.0 * n * kMaxGroupCols * 4 + 8 * 2 * nb * 4 * kMaxGroupCols + 8 * 6 * nb * kMaxGroupCols;
            } else {
                // multi-launch work: six [n][k] vectors, permuted b and x, block shares, coarse
                // right-hand side, per-workgroup partial sums, state
                b += 8.0 * n * kMaxGroupCols * 8 + 8 * nb * 4 * kMaxGroupCols + 8 * ncmax * kMaxGroupCols +
                     8.0 * (double)pcg_ml_part_doubles(nV) + (double)pcg_ml_state_bytes();
            }
        }
    }
    // CG state and reductions
    b += 8.0 * (double)cg_state_doubles(nV, ncol) + 8 * n * ncol + 8.0 * (double)cg_red_doubles(ncol) +
         4.0 * (double)cg_bar_words(ncol) + 12 * kMaxCols;
    b += 8.0 * (double)std::max(reduce_scratch_doubles(16), project_scratch_doubles(ncol, ncomp)) + 8 * 256;
    // all-pairs partial sums (shared by the kinds), reduced sums, face averages
    const PairPlan pe = plan_for(kKindEnergy, prec, 1, nF, cap);
    const PairPlan pg = plan_for(kKindGrad, prec, 1, nF, cap);
    const int kf = std::min(ncol, kMaxGroupCols);
    const PairPlan pf = plan_for(kKindFrac, prec, kf, nF, cap);
    double part = std::max({(double)(pe.n_split + 1) * pe.irows, 7.0 * (pg.n_split + 1) * pg.irows,
                            (double)kf * pf.n_split * pf.irows});
    if (sym_grad_eligible(prm, nF)) part = std::max(part, (double)pe.irows + (double)sym_units(nF) + (double)nF);
    const double gface = std::max((double)pe.irows, 7.0 * pg.irows);
    const double esz = prec == TP_PREC_FP64 ? 8 : 4;
    b += 8 * part + 8 * gface + 8.0 * kf * pf.irows + (double)cap * ((kf + 3) / 4 * 4) * esz;
    double symb = 0.0;
    if (sym_frac_eligible(prm, nF, kf)) symb = 4.0 * (double)sym_buffer_floats(prm, nF, kf);
    if (sym_grad_eligible(prm, nF)) symb = std::max(symb, 4.0 * (double)sym_buffer_floats(prm, nF, kGradOutputs));
    b += symb;
    // step work arrays, per-face volumes and edge lengths, CG tables
    b += 8 * n * ncol * 4 + 8 * n * 3 * 3 + 16 * f + 4096;
    // Barnes-Hut tree, keys, sort scratch and per-face sums (allocated at creation, where
    // the Morton order of the faces is computed with them)
    {
        const double M = (double)bh_node_count(nF, prm.leaf_size, nullptr);
        b += f * (176.0 + 56.0) + M * (144.0 + 8.0 * kMaxGroupCols) + (double)bh_sort_temp_bytes(nF) + 64;
        // block cluster tree lists and far-field values (chi > 0; about 64 blocks per node)
        if (prm.chi > 0.0) b += M * (8.0 * (kMaxGroupCols + 1) + 4.0 * 64 + 8.0);
    }
    // FP64 near-field grid
    if (prm.precision == TP_PREC_FP32_NEAR64) b += (double)near_grid_bytes(nF);
    return (uint64_t)(b * 1.02) + 65536;
}

struct ProblemGuard {
    tp_problem* p = nullptr;
    ~ProblemGuard()
    {
        if (p) tp_problem_destroy(p);
    }
};

// Every entry point on a problem starts here.  Unless join is false (calls that neither
// write V nor read the cotan values, the solvers' matrix or the preconditioner), the
// problem's stream first waits for a set-up still running on the second stream.
tp_status bind(tp_problem* P, bool join = true)
{
    if (!P) return fail(TP_E_INVALID_ARGUMENT, "problem is NULL");
    TP_HIP(hipSetDevice(P->device));
    if (join) TP_TRY(join_aux(P));
    return TP_OK;
}

}  // namespace

// ------------------------------------------------------------------ allocation-free energy
//
// tp_energy_faces_noalloc keeps all of its device scratch (face data, partial sums,
// reduction scratch, flags and the result) in one file-scope device array, so it never
// allocates.  Each GPU the library runs on holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns on that device.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
constexpr int64_t kNoAllocMaxFaces = 65536;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

struct ScratchAddresses {
    std::mutex mu;
    void* p[64] = {};
};
ScratchAddresses g_scratch;

// The device address of `scratch` on the current device (looked up once per device).
tp_status scratch_address(unsigned char** out)
{
    int dev = 0;
    TP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(TP_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch.mu);
    if (!g_scratch.p[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(TP_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch.p[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch.p[dev]);
    return TP_OK;
}

__global__ void k_zero_ints(int* __restrict__ p, int n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0;
}

}  // namespace

// ======================================================================== C-ABI

extern "C" {

tp_status tp_params_default(tp_params* p)
{
    if (!p) return TP_E_INVALID_ARGUMENT;
    p->alpha = 6.0;
    p->beta = 12.0;
    p->sigma = -1.0;
    p->precision = TP_PREC_FP32_NEAR64;
    p->cg_rtol = 1e-10;
    p->cg_maxiter = 20000;
    p->cg_precond = 1;
    p->theta = 0.0;
    p->leaf_size = 8;
    p->chi = 0.0;
    p->sym_pairs = -1;
    p->sym_band = 0;
    return TP_OK;
}

tp_status tp_step_opts_default(tp_step_opts* o)
{
    if (!o) return TP_E_INVALID_ARGUMENT;
    o->tau0 = 0.0;
    o->line_search = 1;
    o->armijo_c = 1e-4;
    o->shrink = 0.5;
    o->max_backtracks = 30;
    o->constrain_area = 1;
    o->constrain_volume = 1;
    o->area_target = NAN;
    o->volume_target = NAN;
    o->solver = 0;
    o->solver_rtol = 1e-4;
    o->solver_maxiter = 300;
    o->area_penalty = 0.0;
    o->volume_penalty = 0.0;
    o->barycenter_motion = 0;
    o->warm_start = 1;
    return TP_OK;
}

const char* tp_last_error(void) { return get_error(); }

tp_status tp_problem_create(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                            const tp_params* params, void* stream, tp_problem** out)
{
    set_error("");
    return create_problem(V, nV, F, nF, params, (hipStream_t)stream, out);
}

void tp_problem_destroy(tp_problem* prob)
{
    if (!prob) return;
    (void)hipSetDevice(prob->device);
    (void)hipStreamSynchronize(prob->stream);
    if (prob->aux) {
        (void)hipStreamSynchronize(prob->aux);
        (void)hipEventDestroy(prob->aux_fork);
        (void)hipEventDestroy(prob->aux_join);
        (void)hipStreamDestroy(prob->aux);
    }
    delete prob;
}

tp_status tp_problem_set_vertices(tp_problem* P, const double* V)
{
    TP_TRY(bind(P));
    if (!V) return fail(TP_E_INVALID_ARGUMENT, "V is NULL");
    TP_HIP(hipMemcpyAsync(P->V.p, V, sizeof(double) * 3 * P->nV, hipMemcpyDeviceToDevice, P->stream));
    P->geom_valid = false;
    P->cotan_valid = false;
    // a problem whose last positions were solved with will likely be solved with again:
    // start the set-up for the new ones beside the work that comes first
    const bool solved = P->setup_used;
    P->setup_used = false;
    if (solved) TP_TRY(start_cotan(P));
    return geometry(P);
}

tp_status tp_problem_get_vertices(tp_problem* P, double* V_out)
{
    TP_TRY(bind(P));
    if (!V_out) return fail(TP_E_INVALID_ARGUMENT, "V_out is NULL");
    TP_HIP(hipMemcpyAsync(V_out, P->V.p, sizeof(double) * 3 * P->nV, hipMemcpyDeviceToDevice, P->stream));
    TP_HIP(hipStreamSynchronize(P->stream));
    return TP_OK;
}

tp_status tp_problem_energy(tp_problem* P, double* E_out)
{
    TP_TRY(bind(P, false));   // runs beside a pending set-up
    if (!E_out) return fail(TP_E_INVALID_ARGUMENT, "E_out is NULL");
    set_error("");
    TP_TRY(ensure_geometry(P));
    return run_energy(P, E_out);
}

tp_status tp_problem_gradient(tp_problem* P, double* E_out, double* dE_out)
{
    TP_TRY(bind(P, false));   // runs beside a pending set-up
    if (!E_out || !dE_out) return fail(TP_E_INVALID_ARGUMENT, "E_out and dE_out must be non-NULL");
    set_error("");
    TP_TRY(ensure_geometry(P));
    TP_TRY(run_gradient(P, E_out, dE_out));
    TP_HIP(hipStreamSynchronize(P->stream));
    return TP_OK;
}

tp_status tp_problem_fractional_apply(tp_problem* P, const double* u, int k, double* Lu_out)
{
    TP_TRY(bind(P, false));   // runs beside a pending set-up
    if (!u || !Lu_out) return fail(TP_E_INVALID_ARGUMENT, "u and Lu_out must be non-NULL");
    if (k < 1 || k > kMaxCols) return fail(TP_E_INVALID_ARGUMENT, "k must lie in [1, 64]");
    set_error("");
    TP_TRY(ensure_geometry(P));
    TP_TRY(run_fractional(P, u, k, k, Lu_out, k));
    TP_HIP(hipStreamSynchronize(P->stream));
    return TP_OK;
}

tp_status tp_problem_set_obstacle(tp_problem* P, const double* Vo, int64_t nVo, const int32_t* Fo, int64_t nFo,
                                  double p, double weight)
{
    TP_TRY(bind(P));
    set_error("");
    if (nFo == 0 || weight == 0.0) {   // remove the obstacle
        P->obs_n = 0;
        P->obs_w = 0.0;
        P->obs_tree.built = false;
        return TP_OK;
    }
    if (!Vo || !Fo || nVo < 3 || nFo < 1) return fail(TP_E_INVALID_ARGUMENT, "obstacle needs Vo, Fo, nVo >= 3, nFo >= 1");
    if (!(p > 0.0) || !(weight > 0.0) || !std::isfinite(p) || !std::isfinite(weight))
        return fail(TP_E_INVALID_ARGUMENT, "obstacle exponent and weight must be positive and finite");
    if (nFo > (int64_t)(INT32_MAX / 8)) return fail(TP_E_INVALID_ARGUMENT, "obstacle too large");
    hipStream_t s = P->stream;
    std::vector<int32_t> fh((size_t)3 * nFo);
    TP_HIP(hipMemcpyAsync(fh.data(), Fo, sizeof(int32_t) * fh.size(), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    for (int32_t v : fh)
        if (v < 0 || (int64_t)v >= nVo) return fail(TP_E_INVALID_ARGUMENT, "obstacle face index out of range");
    P->obs_cap = obstacle_capacity(nFo);
    P->obs_tree.built = false;
    TP_TRY(P->obs_x.ensure((size_t)P->obs_cap, s));
    TP_HIP(launch_obstacle_faces(Vo, Fo, nFo, P->obs_cap, P->obs_x.p, s));
    if (P->prm.theta > 0.0) {   // Barnes-Hut over the obstacle: its tree, once (the obstacle is static)
        TP_TRY(P->obs_tree.ensure(nFo, P->prm.leaf_size, s));
        FaceData fo;
        fo.nF = nFo;
        fo.cap = P->obs_cap;
        fo.dx = P->obs_x.p;
        TP_HIP(launch_bh_build(P->obs_tree.view, Vo, Fo, nullptr, nFo, P->prm.leaf_size, fo, s));
        TP_HIP(hipMemsetAsync(P->obs_tree.counts.p, 0, 2 * sizeof(unsigned long long), s));
        P->obs_tree.built = true;
    }
    TP_HIP(hipStreamSynchronize(s));
    P->obs_n = nFo;
    P->obs_p = p;
    P->obs_w = weight;
    return TP_OK;
}

tp_status tp_problem_add_implicit(tp_problem* P, int kind, const double* q, double c, double p, double weight,
                                  int attract)
{
    TP_TRY(bind(P));
    set_error("");
    if (kind < 0) {   // remove every implicit potential
        P->imp.n = 0;
        return TP_OK;
    }
    if (P->imp.n >= kMaxImplicit) return fail(TP_E_INVALID_ARGUMENT, "at most 8 implicit potentials");
    if ((kind != 0 && kind != 1) || !q || !(p > 0.0) || !(weight > 0.0) || (attract != 0 && attract != 1) ||
        !std::isfinite(c) || !std::isfinite(p) || !std::isfinite(weight))
        return fail(TP_E_INVALID_ARGUMENT, "implicit potential: kind 0 or 1, q non-NULL, p > 0, weight > 0");
    double qq[3] = {q[0], q[1], q[2]};
    if (kind == 0) {
        const double nn = std::sqrt(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2]);
        if (!(nn > 0.0)) return fail(TP_E_INVALID_ARGUMENT, "plane normal is zero");
        for (double& v : qq) v /= nn;
        c /= nn;
    } else if (!(c > 0.0)) {
        return fail(TP_E_INVALID_ARGUMENT, "sphere radius must be > 0");
    }
    const int k = P->imp.n;
    P->imp.kind[k] = kind;
    P->imp.attract[k] = attract;
    for (int m = 0; m < 3; ++m) P->imp.q[k][m] = qq[m];
    P->imp.c[k] = c;
    P->imp.p[k] = p;
    P->imp.w[k] = weight;
    P->imp.n = k + 1;
    return TP_OK;
}

tp_status tp_problem_implicit_energy(tp_problem* P, double* E_out, double* dE_out)
{
    TP_TRY(bind(P));
    if (!E_out) return fail(TP_E_INVALID_ARGUMENT, "E_out is NULL");
    if (P->imp.n < 1) return fail(TP_E_INVALID_ARGUMENT, "no implicit potential is set");
    set_error("");
    TP_TRY(ensure_geometry(P));
    TP_TRY(ensure_vf(P));
    const Batch B{P};
    TP_TRY(enqueue_implicit(P));
    if (dE_out)
        TP_HIP(launch_grad_gather(P->V.p, P->F.p, P->nV, P->nF, P->vf_off.p, P->vf_idx.p, P->imp_g.p, P->nF, dE_out,
                                  P->stream));
    TP_TRY(enqueue_fetch(B));
    TP_TRY(sync_batch(B));
    *E_out = P->hs.p[kSlotImp];
    if (!std::isfinite(*E_out)) return fail(TP_E_NONFINITE, "non-finite implicit potential (a face inside an obstacle?)");
    return TP_OK;
}

tp_status tp_problem_obstacle_energy(tp_problem* P, double* E_out, double* dE_out)
{
    TP_TRY(bind(P));
    if (!E_out) return fail(TP_E_INVALID_ARGUMENT, "E_out is NULL");
    if (P->obs_n < 1) return fail(TP_E_INVALID_ARGUMENT, "no obstacle is set");
    set_error("");
    TP_TRY(ensure_geometry(P));
    TP_TRY(ensure_vf(P));
    const Batch B{P};
    TP_TRY(enqueue_obstacle(P));
    if (dE_out)
        TP_HIP(launch_grad_gather(P->V.p, P->F.p, P->nV, P->nF, P->vf_off.p, P->vf_idx.p, P->obs_g.p, P->nF, dE_out,
                                  P->stream));
    TP_TRY(enqueue_fetch(B));
    TP_TRY(sync_batch(B));
    *E_out = P->hs.p[kSlotObs];
    if (!std::isfinite(*E_out)) return fail(TP_E_NONFINITE, "non-finite obstacle potential (a barycenter on the obstacle?)");
    return TP_OK;
}

tp_status tp_problem_sobolev_apply(tp_problem* P, const double* u, int k, double* Au_out)
{
    TP_TRY(bind(P));
    if (!u || !Au_out) return fail(TP_E_INVALID_ARGUMENT, "u and Au_out must be non-NULL");
    if (k < 1 || k > kMaxCols) return fail(TP_E_INVALID_ARGUMENT, "k must lie in [1, 64]");
    set_error("");
    TP_TRY(ensure_geometry(P));
    TP_TRY(run_sobolev(P, u, k, k, Au_out, k));
    TP_HIP(hipStreamSynchronize(P->stream));
    return TP_OK;
}

tp_status tp_problem_sobolev_solve(tp_problem* P, const double* b, int k, double rtol, int restart,
                                   int maxiter, int precond, double* x_out, tp_gmres_report* report)
{
    TP_TRY(bind(P));
    if (!b || !x_out) return fail(TP_E_INVALID_ARGUMENT, "b and x_out must be non-NULL");
    if (k < 1 || k > kMaxCols) return fail(TP_E_INVALID_ARGUMENT, "k must lie in [1, 64]");
    if (!(rtol > 0.0) || restart < 1 || restart > 100 || maxiter < 1 || (restart + 1) * k > 1024)
        return fail(TP_E_INVALID_ARGUMENT, "need rtol > 0, 1 <= restart <= 100, (restart + 1) k <= 1024, maxiter >= 1");
    if (precond != 0 && precond != 1) return fail(TP_E_INVALID_ARGUMENT, "precond must be 0 or 1");
    set_error("");
    return run_sobolev_solve(P, b, k, rtol, restart, maxiter, precond, x_out, report);
}

tp_status tp_problem_precond_apply(tp_problem* P, const double* b, int k, double* x_out,
                                   tp_solve_report* report)
{
    TP_TRY(bind(P));
    if (!b || !x_out) return fail(TP_E_INVALID_ARGUMENT, "b and x_out must be non-NULL");
    if (k < 1 || k > kMaxCols) return fail(TP_E_INVALID_ARGUMENT, "k must lie in [1, 64]");
    set_error("");
    return run_precond(P, b, k, x_out, report);
}

tp_status tp_problem_poisson_solve(tp_problem* P, const double* b, int k, double* x_out,
                                   tp_solve_report* report)
{
    TP_TRY(bind(P));
    if (!b || !x_out) return fail(TP_E_INVALID_ARGUMENT, "b and x_out must be non-NULL");
    if (k < 1 || k > kMaxCols) return fail(TP_E_INVALID_ARGUMENT, "k must lie in [1, 64]");
    set_error("");
    TP_TRY(ensure_geometry(P));
    TP_TRY(ensure_lap(P));
    const size_t nk = (size_t)P->nV * k;
    TP_TRY(P->W1.ensure(nk, P->stream));
    TP_HIP(hipMemcpyAsync(P->W1.p, b, nk * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    EventTimer tm(P->stream);
    tm.mark(0);
    int it = 0;
    double res = 0;
    tp_status st = run_cg(P, P->W1.p, x_out, k, &it, &res);
    tm.mark(1);
    if (report) {
        std::memset(report, 0, sizeof(*report));
        report->cg_iters[0] = it;
        report->cg_relres[0] = res;
        report->t_ms[0] = tm.ms(0, 1);
    }
    return st;
}

tp_status tp_precond_step(tp_problem* P, const tp_step_opts* opts, tp_step_report* report,
                          double* direction_out)
{
    TP_TRY(bind(P));
    set_error("");
    return run_step_batch(&P, 1, opts, report, nullptr, &direction_out);
}

tp_status tp_batch_step(tp_problem* const* probs, int n, const tp_step_opts* opts,
                        tp_step_report* reports, tp_status* statuses)
{
    set_error("");
    if (!probs || n < 1) return fail(TP_E_INVALID_ARGUMENT, "need at least one problem");
    return run_step_batch(probs, n, opts, reports, statuses, nullptr);
}

tp_status tp_energy(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                    const tp_params* params, double* E_out, void* stream)
{
    if (!E_out) return fail(TP_E_INVALID_ARGUMENT, "E_out is NULL");
    ProblemGuard g;
    TP_TRY(tp_problem_create(V, nV, F, nF, params, stream, &g.p));
    return run_energy(g.p, E_out);
}

tp_status tp_gradient(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                      const tp_params* params, double* E_out, double* dE_out, void* stream)
{
    ProblemGuard g;
    TP_TRY(tp_problem_create(V, nV, F, nF, params, stream, &g.p));
    return tp_problem_gradient(g.p, E_out, dE_out);
}

tp_status tp_fractional_apply(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                              const tp_params* params, const double* u, int k, double* Lu_out,
                              void* stream)
{
    if (k < 1 || k > kMaxCols) return fail(TP_E_INVALID_ARGUMENT, "k must lie in [1, 64]");
    ProblemGuard g;
    TP_TRY(tp_problem_create(V, nV, F, nF, params, stream, &g.p));
    return tp_problem_fractional_apply(g.p, u, k, Lu_out);
}

tp_status tp_sobolev_apply(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                           const tp_params* params, const double* u, int k, double* Au_out,
                           void* stream)
{
    if (k < 1 || k > kMaxCols) return fail(TP_E_INVALID_ARGUMENT, "k must lie in [1, 64]");
    ProblemGuard g;
    TP_TRY(tp_problem_create(V, nV, F, nF, params, stream, &g.p));
    return tp_problem_sobolev_apply(g.p, u, k, Au_out);
}

tp_status tp_precond_apply(const double* V, int64_t nV, const int32_t* F, int64_t nF,
                           const tp_params* params, const double* b, int k, double* x_out,
                           tp_solve_report* report, void* stream)
{
    if (k < 1 || k > kMaxCols) return fail(TP_E_INVALID_ARGUMENT, "k must lie in [1, 64]");
    ProblemGuard g;
    TP_TRY(tp_problem_create(V, nV, F, nF, params, stream, &g.p));
    return tp_problem_precond_apply(g.p, b, k, x_out, report);
}

tp_status tp_energy_faces(const double* X, const double* N, const double* a, int64_t nF,
                          const tp_params* params, double* E_out, void* stream)
{
    set_error("");
    if (!X || !N || !a || !E_out) return fail(TP_E_INVALID_ARGUMENT, "NULL argument");
    if (nF < 2 || nF > (int64_t)(INT32_MAX / 8)) return fail(TP_E_INVALID_ARGUMENT, "need 2 <= nF < 2^28");
    auto* P = new tp_problem();
    ProblemGuard g;
    g.p = P;
    TP_TRY(validate_params(params, P->prm, P->sigma));
    if (P->prm.theta > 0.0)
        return fail(TP_E_INVALID_ARGUMENT, "Barnes-Hut (theta > 0) needs the mesh: use tp_energy or a problem");
    if (P->prm.precision == TP_PREC_FP32_NEAR64)
        return fail(TP_E_INVALID_ARGUMENT, "TP_PREC_FP32_NEAR64 needs the mesh: use tp_energy or a problem");
    (void)hipGetDevice(&P->device);
    P->stream = (hipStream_t)stream;
    P->nF = nF;
    P->nV = 0;
    TP_TRY(alloc_faces(P));
    TP_HIP(launch_face_from_quantities(X, N, a, nF, P->fd, P->flags.p, P->stream));
    TP_TRY(check_flags(P));
    return run_energy(P, E_out);
}

tp_status tp_energy_faces_noalloc(const double* X, const double* N, const double* a, int64_t nF,
                                  const tp_params* params, double* E_out, void* stream)
{
    set_error("");
    if (!X || !N || !a || !E_out) return fail(TP_E_INVALID_ARGUMENT, "NULL argument");
    if (nF < 2 || nF > kNoAllocMaxFaces)
        return fail(TP_E_INVALID_ARGUMENT, "tp_energy_faces_noalloc needs 2 <= nF <= 65536");
    tp_params prm;
    double sigma = 0.0;
    TP_TRY(validate_params(params, prm, sigma));
    if (prm.theta > 0.0)
        return fail(TP_E_INVALID_ARGUMENT, "Barnes-Hut (theta > 0) needs the mesh: use tp_energy or a problem");
    if (prm.precision == TP_PREC_FP32_NEAR64)
        return fail(TP_E_INVALID_ARGUMENT, "TP_PREC_FP32_NEAR64 needs the mesh: use tp_energy or a problem");
    hipStream_t s = (hipStream_t)stream;
    unsigned char* base = nullptr;
    TP_TRY(scratch_address(&base));

    // layout of the scratch: header (flags, result), reduction scratch, tile boxes, face
    // data, reduced per-face sums, then as many j-splits of partial sums as fit
    const int64_t cap = face_capacity(nF, 4);
    PairPlan pl = plan_for(kKindEnergy, prm.precision, 1, nF, cap);
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_hdr = take(64);
    const size_t o_red = take(sizeof(double) * reduce_scratch_doubles(16));
    const size_t o_box = take(sizeof(float4) * 2 * (size_t)(cap / kTileJ));
    const size_t o_fx = take(sizeof(float4) * (size_t)cap);
    const size_t o_fl = take(sizeof(float4) * (size_t)cap);
    const size_t o_fn = take(sizeof(float4) * (size_t)cap);
    const size_t o_dx = take(sizeof(double4) * (size_t)cap);
    const size_t o_dn = take(sizeof(double4) * (size_t)cap);
    const size_t o_gf = take(sizeof(double) * (size_t)pl.irows);
    const size_t per_split = sizeof(double) * (size_t)pl.irows;
    if (off + per_split > kNoAllocScratchBytes)
        return fail(TP_E_INVALID_ARGUMENT, "nF too large for the scratch of tp_energy_faces_noalloc");
    const int max_split = (int)std::min<size_t>((kNoAllocScratchBytes - off) / per_split, 1 << 20);
    if (pl.n_split > max_split) {
        pl.tiles_per_split = (pl.ntiles_j + max_split - 1) / max_split;
        pl.n_split = (pl.ntiles_j + pl.tiles_per_split - 1) / pl.tiles_per_split;
    }
    const size_t o_part = take(per_split * (size_t)pl.n_split);
    if (off > kNoAllocScratchBytes) return fail(TP_E_INVALID_ARGUMENT, "scratch layout exceeds its size");

    int* flags = reinterpret_cast<int*>(base + o_hdr);
    double* E_dev = reinterpret_cast<double*>(base + o_hdr + 16);
    double* red = reinterpret_cast<double*>(base + o_red);
    FaceData fd;
    fd.nF = nF;
    fd.cap = cap;
    fd.tbox = reinterpret_cast<float4*>(base + o_box);
    fd.fx = reinterpret_cast<float4*>(base + o_fx);
    fd.fl = reinterpret_cast<float4*>(base + o_fl);
    fd.fn = reinterpret_cast<float4*>(base + o_fn);
    fd.dx = reinterpret_cast<double4*>(base + o_dx);
    fd.dn = reinterpret_cast<double4*>(base + o_dn);
    double* gface = reinterpret_cast<double*>(base + o_gf);
    double* part = reinterpret_cast<double*>(base + o_part);

    // flags start at zero (a fill kernel, so the sequence can be captured in a graph);
    // every other region is written before it is read
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, flags, kNumFlags);
    TP_HIP(hipGetLastError());
    TP_HIP(launch_face_from_quantities(X, N, a, nF, fd, flags, s));
    const PairJob J = make_pair_job(fd, pl, part);
    TP_HIP(launch_pairs_energy(&J, 1, prm.precision, prm.alpha, prm.beta, s));
    TP_HIP(launch_reduce_splits(part, pl.n_split, 1, pl.irows, nF, gface, pl.irows, s));
    TP_HIP(launch_dot_cols(&fd.dx[0].w, 4, gface, 1, nF, 1, red, E_dev, s));
    struct {
        int flags[kNumFlags];
        double E;
    } h;
    static_assert(sizeof(h) == 16 + sizeof(double), "header layout: flags at 0, the result at 16");
    TP_HIP(hipMemcpyAsync(&h, base + o_hdr, sizeof(h), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    if (h.flags[kFlagNonFinite]) return fail(TP_E_NONFINITE, "non-finite vertex coordinates or face quantities");
    if (h.flags[kFlagDegenerate]) return fail(TP_E_DEGENERATE_FACE, "a face has zero area (its normal is undefined)");
    *E_out = h.E;
    if (!std::isfinite(h.E)) return fail(TP_E_NONFINITE, "non-finite energy (coincident face barycenters?)");
    return TP_OK;
}

tp_status tp_problem_set_pins(tp_problem* P, const int32_t* idx, int64_t n)
{
    TP_TRY(bind(P));
    if (n < 0 || (n > 0 && !idx)) return fail(TP_E_INVALID_ARGUMENT, "need n >= 0 pinned vertices (host indices)");
    for (int64_t q = 0; q < n; ++q)
        if (idx[q] < 0 || idx[q] >= P->nV) return fail(TP_E_BAD_INDEX, "a pinned vertex index lies outside [0, nV)");
    TP_TRY(ensure_lap(P));
    hipStream_t s = P->stream;
    std::vector<int8_t> mask(P->nV, 0);
    int64_t cnt = 0;
    for (int64_t q = 0; q < n; ++q)
        if (!mask[idx[q]]) {
            mask[idx[q]] = 1;
            ++cnt;
        }
    if (cnt > 0) {
        std::vector<double> w(P->ncomp, 0.0);
        std::vector<char> pinned(P->ncomp, 0);
        for (int64_t v = 0; v < P->nV; ++v) {
            w[P->comp_host[v]] += 1.0;
            if (mask[v]) pinned[P->comp_host[v]] = 1;
        }
        for (int c = 0; c < P->ncomp; ++c) w[c] = pinned[c] ? 0.0 : 1.0 / w[c];
        TP_TRY(P->pin_mask.ensure(P->nV, s));
        TP_TRY(P->inv_count_pin.ensure(P->ncomp, s));
        TP_HIP(hipMemcpyAsync(P->pin_mask.p, mask.data(), (size_t)P->nV, hipMemcpyHostToDevice, s));
        TP_HIP(hipMemcpyAsync(P->inv_count_pin.p, w.data(), sizeof(double) * P->ncomp, hipMemcpyHostToDevice, s));
        TP_HIP(hipStreamSynchronize(s));
    }
    P->npins = cnt;
    P->cotan_valid = false;     // the solvers' matrix changes
    P->warm_cols = 0;
    return TP_OK;
}

tp_status tp_problem_bct_stats(tp_problem* P, int64_t* admissible, int64_t* inadmissible)
{
    TP_TRY(bind(P));
    if (!admissible || !inadmissible) return fail(TP_E_INVALID_ARGUMENT, "NULL argument");
    *admissible = P->bct_nadm;
    *inadmissible = P->bct_ninad;
    return TP_OK;
}

tp_status tp_problem_bh_stats(tp_problem* P, int64_t* far_terms, int64_t* near_terms)
{
    TP_TRY(bind(P));
    if (!far_terms || !near_terms) return fail(TP_E_INVALID_ARGUMENT, "NULL argument");
    unsigned long long h[2] = {0, 0};
    if (P->bh_counts.p) {
        TP_HIP(hipMemcpyAsync(h, P->bh_counts.p, sizeof(h), hipMemcpyDeviceToHost, P->stream));
        TP_HIP(hipStreamSynchronize(P->stream));
    }
    *far_terms = (int64_t)h[0];
    *near_terms = (int64_t)h[1];
    return TP_OK;
}

tp_status tp_problem_obstacle_stats(tp_problem* P, int64_t* far_terms, int64_t* near_terms)
{
    TP_TRY(bind(P));
    if (!far_terms || !near_terms) return fail(TP_E_INVALID_ARGUMENT, "NULL argument");
    set_error("");
    *far_terms = 0;
    *near_terms = 0;
    if (P->obs_n < 1) return TP_OK;
    if (!P->obs_tree.built) {
        *near_terms = P->nF * P->obs_n;
        return TP_OK;
    }
    unsigned long long h[2] = {0, 0};
    TP_HIP(hipMemcpyAsync(h, P->obs_tree.counts.p, sizeof(h), hipMemcpyDeviceToHost, P->stream));
    TP_HIP(hipStreamSynchronize(P->stream));
    *far_terms = (int64_t)h[0];
    *near_terms = (int64_t)h[1];
    return TP_OK;
}

tp_status tp_problem_device_bytes(const tp_problem* P, uint64_t* bytes)
{
    if (!P || !bytes) return fail(TP_E_INVALID_ARGUMENT, "NULL argument");
    *bytes = (uint64_t)P->device_bytes();
    return TP_OK;
}

tp_status tp_estimate_device_bytes(int64_t nV, int64_t nF, int max_degree, int ncomp,
                                   const tp_params* params, int n_constraints, uint64_t* bytes)
{
    set_error("");
    if (!bytes) return fail(TP_E_INVALID_ARGUMENT, "bytes is NULL");
    if (nV < 3 || nF < 2 || max_degree < 1 || ncomp < 1 || n_constraints < 0 || n_constraints > 2)
        return fail(TP_E_INVALID_ARGUMENT, "need nV >= 3, nF >= 2, max_degree >= 1, ncomp >= 1, 0 <= n_constraints <= 2");
    tp_params prm;
    double sigma = 0;
    TP_TRY(validate_params(params, prm, sigma));
    *bytes = estimate_bytes(nV, nF, max_degree, ncomp, prm, n_constraints);
    return TP_OK;
}

tp_status tp_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    return TP_OK;
}

tp_status tp_set_allocator(tp_alloc_fn alloc, tp_free_fn free_, void* user)
{
    set_error("");
    if ((alloc == nullptr) != (free_ == nullptr))
        return fail(TP_E_INVALID_ARGUMENT, "give both an allocation and a free function, or neither");
    std::lock_guard<std::mutex> lk(g_alloc.mu);
    if (g_alloc.live != 0)
        return fail(TP_E_INVALID_ARGUMENT, std::to_string(g_alloc.live) +
                                               " buffers from the registered allocator are still alive (destroy the problems first)");
    g_alloc.alloc = alloc;
    g_alloc.free_ = free_;
    g_alloc.user = user;
    return TP_OK;
}

tp_status tp_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.resolve(true);
    for (auto& s : g_prof.st) std::memset(&s, 0, sizeof(s));
    return TP_OK;
}

tp_status tp_profile_get(int kind, tp_kernel_stats* out)
{
    if (kind < 0 || kind > 3 || !out) return TP_E_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.resolve(true);
    *out = g_prof.st[kind];
    return TP_OK;
}

}  // extern "C"
