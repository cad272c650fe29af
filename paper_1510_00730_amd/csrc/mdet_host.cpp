// Host side of libmdet: context, the one-time pre-processing of the CI
// expansion (Sec. 2.1), the excitation analysis against the reference
// determinant, device upload, and the C ABI declared in include/mdet.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "mdet_internal.h"

using namespace mdet;

namespace {

struct Status : std::runtime_error {
    mdet_status code;
    Status(mdet_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIP_OK(expr)                                                                   \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess)                                                          \
            throw Status(_e == hipErrorOutOfMemory ? MDET_ENOMEM : MDET_EHIP,          \
                         std::string(#expr) + ": " + hipGetErrorString(_e));           \
    } while (0)

// A device allocation owned by the context.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t n) {
        release();
        if (n == 0) n = 64;
        HIP_OK(hipMalloc(&p, n));
        bytes = n;
    }
    template <typename T>
    void upload(const std::vector<T> &v) {
        alloc(sizeof(T) * v.size());
        if (!v.empty()) HIP_OK(hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

struct SpinHost {
    int n = 0;
    int64_t U = 0;
    std::vector<uint64_t> uniq;      // [U][n_int], public (omega) order
    int64_t ref = 0;                 // public index of the reference
    std::vector<int32_t> occ0;       // [n]
    std::vector<int32_t> exec_of;    // public -> exec
    std::vector<int32_t> pub_of;     // exec -> public
    std::vector<DetDesc> desc;       // exec order
    std::vector<DetDescHi> desc_hi;  // exec order, degrees kFastDegree+1 .. MDET_MAX_DEGREE
    std::vector<int32_t> hi_off;     // [n_hi + 1] offsets of their s*s cofactors
    int64_t n_by_degree[MDET_MAX_DEGREE + 1] = {0};
    bool high_degree = false;  // some determinant above MDET_MAX_DEGREE (chain method only)
    int64_t n_above = 0;
    std::vector<int32_t> adj_off, chunk_det;
    std::vector<uint32_t> gent;
    // Sherman-Morrison chain lists (public order = chain order)
    std::vector<int32_t> sm_exec, sm_off;
    std::vector<uint16_t> sm_occ;
    std::vector<uint32_t> sm_sub;
    DevBuf d_occ0, d_desc, d_adj_off, d_chunk_det, d_gent;
    DevBuf d_sm_exec, d_sm_occ, d_sm_off, d_sm_sub, d_desc_hi, d_hi_off;
    std::array<DevBuf *, 11> bufs() {
        return {&d_occ0, &d_desc, &d_adj_off, &d_chunk_det, &d_gent,
                &d_sm_exec, &d_sm_occ, &d_sm_off, &d_sm_sub, &d_desc_hi, &d_hi_off};
    }
    std::array<const DevBuf *, 11> bufs() const {
        return {&d_occ0, &d_desc, &d_adj_off, &d_chunk_det, &d_gent,
                &d_sm_exec, &d_sm_occ, &d_sm_off, &d_sm_sub, &d_desc_hi, &d_hi_off};
    }
};

}  // namespace

struct mdet_ctx {
    int device = 0;
    bool host_only = false;  // created with hip_device == -1: pre-processing only
    std::string err;
    // orbitals
    bool have_orb = false;
    int n_mo = 0, n_prim = 0;
    std::vector<Prim> prim;
    DevBuf d_prim;
    // optional separate orbitals of the down electrons (same n_mo, n_prim)
    bool two_sets = false;
    std::vector<Prim> prim_dn;
    DevBuf d_prim_dn;
    // expansion
    bool have_exp = false;
    int n_up = 0, n_dn = 0, n_int = 0;
    int64_t n_det = 0;
    SpinHost sp[2];
    std::vector<int32_t> row_i, col_j;
    std::vector<double> val;
    std::vector<int64_t> src_pos;
    DevBuf d_rptr, d_rcol, d_rval, d_rseg, d_cptr, d_crow, d_cval, d_cseg, d_rval32, d_cval32;
    DevBuf d_rseg32, d_cseg32, d_rdeg, d_cdeg;
    int32_t nch_r = 1, nch_c = 1, nch_r32 = 1, nch_c32 = 1;
    LaunchCfg cfg{0, 0, 1, 0};
    // configurations found by mdet_autotune, per shape
    struct TunedShape {
        int64_t W;
        int32_t precision, uneven;
        LaunchCfg cfg;
    };
    std::vector<TunedShape> tuned;
    LaunchCfg cfg_for(int64_t W, int32_t precision, bool uneven) const {
        for (const auto &t : tuned)
            if (t.W == W && t.precision == precision && t.uneven == (uneven ? 1 : 0)) return t.cfg;
        return cfg;
    }
    // the fallback's second stream and its fork/join events (created once,
    // before any capture)
    AuxStreams aux{nullptr, {nullptr, nullptr, nullptr, nullptr}};
    void ensure_aux() {
        if (aux.s) return;
        HIP_OK(hipStreamCreateWithFlags(&aux.s, hipStreamNonBlocking));
        for (auto &e : aux.ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    void drop_aux() {
        for (auto &e : aux.ev)
            if (e) (void)hipEventDestroy(e);
        if (aux.s) (void)hipStreamDestroy(aux.s);
        aux = AuxStreams{nullptr, {nullptr, nullptr, nullptr, nullptr}};
    }
    int32_t method = MDET_METHOD_TABLE;
    double sm_threshold = 1e-3;
    int32_t sm_chunk = 64;
    bool sm_ran = false;  // a chain evaluation has been queued since the last reset
    bool jastrow_on = false;
    JastrowParams jastrow{0.0, 0.0, 0.0};
    // DMC work buffers (grow-only)
    DevBuf q_eold, q_cum, q_src, q_R, q_sign, q_logabs, q_gl, q_el;
    hipStream_t own_stream = nullptr;

    // captured evaluations (mdet_eval_graph), keyed by every argument
    struct GraphEntry {
        int64_t W;
        const void *ptr[7];
        int32_t precision;
        hipStream_t stream;
        hipGraphExec_t exec;
        uint64_t last_use;
    };
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    void drop_graphs() {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    double prep_seconds = 0.0;
    // reference-conditioning thresholds of the table method, per precision
    // (index MDET_FP64 / MDET_MIXED)
    double kappa_max[2] = {MDET_KAPPA_FP64_DEFAULT, MDET_KAPPA_MIXED_DEFAULT};
    // optional per-kernel timing with HIP events (a start and an end event
    // per kernel, on the stream it runs on): a ring of event sets, harvested
    // when the ring wraps or on request
    static constexpr int kRing = 64;
    static constexpr int kSetEvents = 2 * kNumKernels;
    bool profiling = false;
    uint32_t prof_user_mask = 0xffffffffu;  // kernels to time (mdet_set_profiling_mask)
    std::vector<hipEvent_t> prof_ev;  // [kRing][kSetEvents]
    uint32_t prof_mask[kRing] = {0};  // kernel slots recorded in each set
    int prof_head = 0, prof_pending = 0;
    double prof_ms[kNumKernels] = {0};
    int64_t prof_calls = 0;
    void harvest_one() {  // oldest pending set
        const int slot = (prof_head - prof_pending + kRing) % kRing;
        hipEvent_t *e = &prof_ev[(size_t)slot * kSetEvents];
        for (int k = 0; k < kNumKernels; ++k) {
            if (!((prof_mask[slot] >> k) & 1u)) continue;
            float ms = 0.f;
            (void)hipEventSynchronize(e[2 * k + 1]);
            if (hipEventElapsedTime(&ms, e[2 * k], e[2 * k + 1]) == hipSuccess) prof_ms[k] += ms;
        }
        ++prof_calls;
        --prof_pending;
    }
    void harvest_all() {
        while (prof_pending > 0) harvest_one();
    }
    hipEvent_t *next_event_set(uint32_t mask) {
        if (prof_pending == kRing) harvest_one();
        prof_mask[prof_head] = mask;
        hipEvent_t *e = &prof_ev[(size_t)prof_head * kSetEvents];
        prof_head = (prof_head + 1) % kRing;
        ++prof_pending;
        return e;
    }
    void drop_profile_events() {
        for (auto &e : prof_ev)
            if (e) (void)hipEventDestroy(e);
        prof_ev.clear();
        prof_pending = 0;
        prof_head = 0;
    }
    // walker work buffers
    int64_t wcap = 0;
    DevBuf w_phi, w_E, w_X, w_g0, w_logdet0, w_sign0, w_flag, w_K, w_R64, w_R32, w_uv64,
        w_uv32, w_psi64, w_Rexp, w_Kmax, w_dpart, w_dcount, w_dlist, w_perm, w_Rs, w_mds, w_sign_s, w_logabs_s, w_gl_s,
        w_ws_s, w_smstat, w_adjhi;
    DevBuf w_smg;  // chain method: per-determinant derivative ratios (grown on demand)
    Work wk{};
    // VMC / MLP work buffers (grow-only)
    int64_t vcap = 0;
    MlpShape mshape{0, 0, 0};
    DevBuf v_Rp, v_signp, v_logabsp, v_glp, v_wsp, v_signR, v_logabsR, v_glR, v_wsR;
    DevBuf m_X, m_Xp, m_h1a, m_h2a, m_h1b, m_h2b, m_O1, m_O2, m_wh1, m_wh2, m_dO1, m_dO2, m_dX2,
        m_gRp, m_gell, m_Jw, m_grad;

    void drop_vmc() {
        for (DevBuf *b : {&q_eold, &q_cum, &q_src, &q_R, &q_sign, &q_logabs, &q_gl, &q_el})
            b->release();
        for (DevBuf *b : {&v_Rp, &v_signp, &v_logabsp, &v_glp, &v_wsp, &v_signR, &v_logabsR, &v_glR,
                          &v_wsR, &m_X, &m_Xp, &m_h1a, &m_h2a, &m_h1b, &m_h2b, &m_O1, &m_O2,
                          &m_wh1, &m_wh2, &m_dO1, &m_dO2, &m_dX2, &m_gRp, &m_gell, &m_Jw, &m_grad})
            b->release();
        vcap = 0;
        mshape = MlpShape{0, 0, 0};
    }

    void drop_expansion() {
        have_exp = false;
        for (auto &s : sp) {
            for (DevBuf *b : s.bufs()) b->release();
            s = SpinHost();
        }
        drop_vmc();
        for (DevBuf *b : {&d_rptr, &d_rcol, &d_rval, &d_rseg, &d_cptr, &d_crow, &d_cval, &d_rval32,
                          &d_cval32,
                          &d_cseg, &d_rseg32, &d_cseg32, &d_rdeg, &d_cdeg})
            b->release();
        drop_work();
    }
    void drop_work() {
        for (DevBuf *b : {&w_phi, &w_E, &w_X, &w_g0, &w_logdet0, &w_sign0, &w_flag, &w_K,
                          &w_R64, &w_R32, &w_uv64, &w_uv32, &w_psi64, &w_Rexp, &w_Kmax, &w_dpart, &w_dcount, &w_dlist,
                          &w_perm, &w_Rs, &w_mds, &w_sign_s, &w_logabs_s, &w_gl_s, &w_ws_s, &w_smstat,
                          &w_smg, &w_adjhi})
            b->release();
        sm_ran = false;
        wcap = 0;
        drop_graphs();
    }
    int64_t work_bytes() const {
        int64_t t = 0;
        for (const DevBuf *b : {&w_phi, &w_E, &w_X, &w_g0, &w_logdet0, &w_sign0, &w_flag,
                                &w_K, &w_R64, &w_R32, &w_uv64, &w_uv32, &w_psi64, &w_Rexp,
                                &w_Kmax, &w_dpart, &w_dcount, &w_dlist, &w_perm, &w_Rs, &w_mds, &w_sign_s,
                                &w_logabs_s, &w_gl_s, &w_ws_s, &w_smstat, &w_smg, &w_adjhi})
            t += (int64_t)b->bytes;
        return t;
    }
    int64_t exp_bytes() const {
        int64_t t = (int64_t)(d_prim.bytes + d_prim_dn.bytes);
        for (const DevBuf *b : {&d_rptr, &d_rcol, &d_rval, &d_rseg, &d_cptr, &d_crow, &d_rval32,
                                &d_cval32,
                                &d_cval, &d_cseg, &d_rseg32, &d_cseg32, &d_rdeg, &d_cdeg})
            t += (int64_t)b->bytes;
        for (const auto &s : sp)
            for (const DevBuf *b : s.bufs()) t += (int64_t)b->bytes;
        return t;
    }
};

namespace {

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// Key of Eq. (comp) (xor of the words as unsigned), ties broken by the words
// from the last to the first, unsigned.  Returns <0, 0, >0.
int compare_dets(const uint64_t *x, const uint64_t *y, int n_int) {
    uint64_t ox = 0, oy = 0;
    for (int w = 0; w < n_int; ++w) {
        ox ^= x[w];
        oy ^= y[w];
    }
    if (ox != oy) return ox < oy ? -1 : 1;
    for (int w = n_int - 1; w >= 0; --w)
        if (x[w] != y[w]) return x[w] < y[w] ? -1 : 1;
    return 0;
}

std::vector<int32_t> occupied(const uint64_t *d, int n_int) {
    std::vector<int32_t> o;
    for (int w = 0; w < n_int; ++w) {
        uint64_t x = d[w];
        while (x) {
            const int b = __builtin_ctzll(x);
            o.push_back(64 * w + b);
            x &= x - 1;
        }
    }
    return o;
}

// Sort and deduplicate one spin list; pos[k] = distinct index of product k.
void unique_spin_list(const uint64_t *dets, int64_t n_det, int n_int, SpinHost &s,
                      std::vector<int32_t> &pos) {
    std::vector<int64_t> order(n_det);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        const int c = compare_dets(dets + a * n_int, dets + b * n_int, n_int);
        return c < 0 || (c == 0 && a < b);
    });
    pos.assign(n_det, -1);
    s.uniq.clear();
    int64_t U = 0;
    for (int64_t t = 0; t < n_det; ++t) {
        const uint64_t *d = dets + order[t] * n_int;
        if (U == 0 || compare_dets(s.uniq.data() + (U - 1) * n_int, d, n_int) != 0) {
            s.uniq.insert(s.uniq.end(), d, d + n_int);
            ++U;
        }
        pos[order[t]] = (int32_t)(U - 1);
    }
    s.U = U;
}

void validate_spin(const SpinHost &s, int n_int, int n_mo, const char *name) {
    for (int64_t i = 0; i < s.U; ++i) {
        const uint64_t *d = s.uniq.data() + i * n_int;
        int pc = 0;
        for (int w = 0; w < n_int; ++w) pc += popcount64(d[w]);
        if (pc != s.n)
            throw Status(MDET_EPOPCOUNT, std::string(name) + " determinant with " +
                                             std::to_string(pc) + " set bits, expected " +
                                             std::to_string(s.n));
        for (int w = 0; w < n_int; ++w) {
            const int lo = 64 * w;
            if (d[w] == 0) continue;
            const int hi = lo + 63 - __builtin_clzll(d[w]);
            if (hi >= n_mo)
                throw Status(MDET_EORBITAL, std::string(name) + " determinant occupies orbital " +
                                                std::to_string(hi) + " >= n_mo");
        }
    }
}

// Excitation analysis relative to the reference, execution order by degree,
// and the lists that aggregate cofactor entries per (slot, orbital) target.
void analyse_spin(SpinHost &s, int n_int, int n_mo) {
    const uint64_t *ref = s.uniq.data() + s.ref * n_int;
    s.occ0 = occupied(ref, n_int);
    const int n = s.n;
    constexpr int DMAX = MDET_MAX_DEGREE;
    // holes (reference slots, ascending) and particles (orbitals, ascending)
    // of every distinct determinant; above MDET_MAX_DEGREE only the degree is
    // kept (such a determinant is evaluated by the chain method only)
    struct Exc {
        int s = 0, eps = 1;
        int h[DMAX] = {0}, p[DMAX] = {0};
    };
    std::vector<Exc> pub(s.U);
    std::vector<int32_t> slot_of(n_mo, -1);
    for (int c = 0; c < n; ++c) slot_of[s.occ0[c]] = c;
    for (int64_t i = 0; i < s.U; ++i) {
        const uint64_t *d = s.uniq.data() + i * n_int;
        Exc &X = pub[i];
        int nh = 0, np = 0;
        for (int c = 0; c < n; ++c) {
            const int m = s.occ0[c];
            if (!((d[m >> 6] >> (m & 63)) & 1ull)) {
                if (nh < DMAX) X.h[nh] = c;
                ++nh;
            }
        }
        for (int32_t m : occupied(d, n_int)) {
            if (slot_of[m] < 0) {
                if (np < DMAX) X.p[np] = m;
                ++np;
            }
        }
        X.s = nh;
        if (nh > DMAX) {
            s.high_degree = true;
        } else {
            // sign of the permutation sorting occ0 with h[a] -> p[a] substituted in place
            std::vector<int32_t> lst(s.occ0);
            for (int a = 0; a < nh; ++a) lst[X.h[a]] = X.p[a];
            int inv = 0;
            for (int x = 0; x < n; ++x)
                for (int y = x + 1; y < n; ++y) inv += lst[x] > lst[y];
            X.eps = (inv & 1) ? -1 : 1;
        }
    }
    s.pub_of.resize(s.U);
    std::iota(s.pub_of.begin(), s.pub_of.end(), 0);
    std::stable_sort(s.pub_of.begin(), s.pub_of.end(),
                     [&](int32_t a, int32_t b) { return pub[a].s < pub[b].s; });
    s.exec_of.assign(s.U, 0);
    s.desc.resize(s.U);
    s.desc_hi.clear();
    s.hi_off.assign(1, 0);
    for (int k = 0; k <= DMAX; ++k) s.n_by_degree[k] = 0;
    s.n_above = 0;
    std::vector<Exc> ex(s.U);
    for (int64_t e = 0; e < s.U; ++e) {
        s.exec_of[s.pub_of[e]] = (int32_t)e;
        const Exc &X = pub[s.pub_of[e]];
        ex[e] = X;
        DetDesc D;
        std::memset(&D, 0, sizeof(D));
        D.s = (uint8_t)std::min(X.s, 255);
        D.eps = (int8_t)X.eps;
        if (X.s <= kFastDegree) {
            for (int a = 0; a < X.s; ++a) {
                D.h[a] = (uint8_t)X.h[a];
                D.p[a] = (uint16_t)X.p[a];
            }
        } else if (X.s <= DMAX) {
            DetDescHi H;
            std::memset(&H, 0, sizeof(H));
            for (int a = 0; a < X.s; ++a) {
                H.h[a] = (uint8_t)X.h[a];
                H.p[a] = (uint16_t)X.p[a];
            }
            s.desc_hi.push_back(H);
            s.hi_off.push_back(s.hi_off.back() + X.s * X.s);
        }
        s.desc[e] = D;
        if (X.s <= DMAX) s.n_by_degree[X.s]++;
        else ++s.n_above;
    }
    if (s.high_degree) {  // no table-method structures: one empty cofactor chunk
        s.adj_off.assign(s.U + 1, 0);
        s.chunk_det.assign({0, (int32_t)s.U});
        s.gent.assign((size_t)kBlockThreads * kGent, kGentNone);
        s.desc_hi.clear();
        s.hi_off.assign(1, 0);
        return;
    }
    // Derivative aggregation: the s*s scaled cofactor entries of determinant d
    // occupy slots adj_off[d] + a*s + b of a staging buffer; determinants are
    // cut into chunks of at most kAdjChunkDets determinants whose slots fit
    // kAdjChunk.  Per chunk, the targets t = h[a]*M + p[b] are dealt to the
    // kBlockThreads threads of the aggregating block (largest list first, to
    // the least loaded thread), each thread getting at most kGent entries: a
    // thread adds the staged slots of its targets, so no target is shared and
    // the sums need no atomics.  gent[chunk][thread][i] = slot | t << 16,
    // sorted by target, then determinant order; kGentNone pads.
    s.adj_off.assign(s.U + 1, 0);
    for (int64_t e = 0; e < s.U; ++e) s.adj_off[e + 1] = s.adj_off[e] + ex[e].s * ex[e].s;
    const int64_t nt = (int64_t)n * n_mo;
    if (nt >= (int64_t)kGentNone >> 16) throw std::runtime_error("electrons x orbitals too large");
    s.chunk_det.assign(1, 0);
    s.gent.clear();
    std::vector<int32_t> cnt(nt, 0), load(kBlockThreads), owner(nt, -1);
    std::vector<int64_t> targets;
    int64_t start = 0;
    while (start < s.U) {
        int64_t end = start;
        while (end < s.U && end - start < kAdjChunkDets &&
               s.adj_off[end + 1] - s.adj_off[start] <= kAdjChunk)
            ++end;
        if (end == start) throw std::runtime_error("cofactor entries of one determinant exceed the staging buffer");
        for (;;) {
            // entries per target, then largest-first assignment
            targets.clear();
            for (int64_t e = start; e < end; ++e)
                for (int a = 0; a < ex[e].s; ++a)
                    for (int b = 0; b < ex[e].s; ++b) {
                        const int64_t tt = (int64_t)ex[e].h[a] * n_mo + ex[e].p[b];
                        if (cnt[tt]++ == 0) targets.push_back(tt);
                    }
            std::stable_sort(targets.begin(), targets.end(),
                             [&](int64_t x, int64_t y) { return cnt[x] > cnt[y]; });
            std::fill(load.begin(), load.end(), 0);
            int32_t worst = 0;
            for (int64_t tt : targets) {
                const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                owner[tt] = j;
                load[j] += cnt[tt];
                worst = std::max(worst, load[j]);
            }
            if (worst <= kGent || end == start + 1) break;
            for (int64_t tt : targets) cnt[tt] = 0, owner[tt] = -1;
            end = start + std::max<int64_t>(1, (end - start) * 9 / 10);
        }
        // the chunk's lists: per thread, its targets ascending, each target's
        // slots in determinant order
        const size_t base = s.gent.size();
        s.gent.resize(base + (size_t)kBlockThreads * kGent, kGentNone);
        std::vector<std::vector<std::pair<int64_t, int32_t>>> per(kBlockThreads);
        const int32_t slot0 = s.adj_off[start];
        for (int64_t e = start; e < end; ++e)
            for (int a = 0; a < ex[e].s; ++a)
                for (int b = 0; b < ex[e].s; ++b) {
                    const int64_t tt = (int64_t)ex[e].h[a] * n_mo + ex[e].p[b];
                    per[owner[tt]].push_back({tt, s.adj_off[e] - slot0 + a * ex[e].s + b});
                }
        for (int j = 0; j < kBlockThreads; ++j) {
            auto &v = per[j];
            if ((int)v.size() > kGent) throw std::runtime_error("cofactor list exceeds its thread");
            std::stable_sort(v.begin(), v.end(),
                             [](const std::pair<int64_t, int32_t> &x,
                                const std::pair<int64_t, int32_t> &y) { return x.first < y.first; });
            for (size_t i = 0; i < v.size(); ++i)
                s.gent[base + (size_t)j * kGent + i] = (uint32_t)v[i].second | ((uint32_t)v[i].first << 16);
        }
        for (int64_t tt : targets) cnt[tt] = 0, owner[tt] = -1;
        s.chunk_det.push_back((int32_t)end);
        start = end;
    }
    if (s.chunk_det.size() == 1) {  // no determinants: one empty chunk
        s.chunk_det.push_back((int32_t)s.U);
        s.gent.assign((size_t)kBlockThreads * kGent, kGentNone);
    }
}

// Lists of the Sherman-Morrison chain (Sec. 2.2): the public (sorted) order
// is the chain order; between consecutive determinants the orbitals that
// leave (ascending) are paired with those that enter (ascending).
void chain_lists(SpinHost &s, int n_int) {
    const int n = s.n;
    s.sm_exec = s.exec_of;
    s.sm_occ.assign((size_t)s.U * n, 0);
    s.sm_off.assign(s.U + 1, 0);
    s.sm_sub.clear();
    std::vector<int32_t> prev;
    for (int64_t i = 0; i < s.U; ++i) {
        const std::vector<int32_t> occ = occupied(s.uniq.data() + i * n_int, n_int);
        for (int c = 0; c < n; ++c) s.sm_occ[(size_t)i * n + c] = (uint16_t)occ[c];
        if (i > 0) {
            std::vector<int32_t> holes, parts;
            std::set_difference(prev.begin(), prev.end(), occ.begin(), occ.end(),
                                std::back_inserter(holes));
            std::set_difference(occ.begin(), occ.end(), prev.begin(), prev.end(),
                                std::back_inserter(parts));
            for (size_t t = 0; t < holes.size(); ++t)
                s.sm_sub.push_back((uint32_t)holes[t] | ((uint32_t)parts[t] << 16));
        }
        s.sm_off[i + 1] = (int32_t)s.sm_sub.size();
        prev = occ;
    }
}

// Segments of the CSR rows (CSC columns) by chunks of kSpmmCols gathered entries.
std::vector<int32_t> chunk_segments(const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                                    int64_t rows, int64_t cols, int32_t width, int32_t &nch) {
    nch = (int32_t)std::max<int64_t>(1, (cols + width - 1) / width);
    std::vector<int32_t> seg((size_t)(nch + 1) * rows);
    for (int64_t i = 0; i < rows; ++i) {
        int32_t k = ptr[i];
        for (int c = 0; c < nch; ++c) {
            seg[(size_t)c * rows + i] = k;
            while (k < ptr[i + 1] && idx[k] < (c + 1) * width) ++k;
        }
        seg[(size_t)nch * rows + i] = ptr[i + 1];
    }
    return seg;
}

template <typename Fn>
mdet_status guarded(mdet_ctx *ctx, Fn &&fn) {
    if (!ctx) return MDET_EINVAL;
    try {
        ctx->err.clear();
        fn();
        return MDET_OK;
    } catch (const Status &s) {
        ctx->err = s.what();
        return s.code;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return MDET_ENOMEM;
    } catch (const std::exception &e) {
        ctx->err = e.what();
        return MDET_EINVAL;
    }
}

void require(bool cond, mdet_status code, const char *msg) {
    if (!cond) throw Status(code, msg);
}

// doubles per (walker, spin) of the cofactors of the determinants of degree
// above kFastDegree (the larger of the two spins' totals)
int64_t hi_stride(const mdet_ctx *c) {
    int64_t h = 0;
    for (const auto &s : c->sp)
        if (!s.hi_off.empty()) h = std::max<int64_t>(h, s.hi_off.back());
    return h;
}

void ensure_work(mdet_ctx *c, int64_t W) {
    c->ensure_aux();
    if (W <= c->wcap) return;
    c->drop_work();
    const int M = c->n_mo, N = c->n_up + c->n_dn;
    const int nmax = std::max(c->n_up, c->n_dn);
    const int64_t Upad = (c->sp[0].U + 63) / 64 * 64, Vpad = (c->sp[1].U + 63) / 64 * 64;
    const int64_t RV = Upad + Vpad;
    const int64_t Wld = (W + 63) / 64 * 64;
    c->w_phi.alloc(sizeof(double) * W * N * 5 * M);
    c->w_E.alloc(sizeof(int32_t) * W * 2 * M);
    c->w_X.alloc(sizeof(double) * W * 2 * nmax * nmax);
    c->w_g0.alloc(sizeof(double) * W * N * 4);
    c->w_logdet0.alloc(sizeof(double) * W * 2);
    c->w_sign0.alloc(sizeof(double) * W * 2);
    c->w_flag.alloc(sizeof(int32_t) * W * 2);
    c->w_K.alloc(sizeof(int32_t) * W * 2);
    c->w_R64.alloc(sizeof(double) * Wld * RV);
    c->w_R32.alloc(sizeof(float) * Wld * RV);
    c->w_uv64.alloc(sizeof(double) * Wld * RV);
    c->w_uv32.alloc(sizeof(float) * Wld * RV);
    c->w_psi64.alloc(sizeof(double) * W * 2 * kPsiParts);
    c->w_Rexp.alloc(sizeof(int32_t) * Wld * RV);
    c->w_Kmax.alloc(sizeof(int32_t) * W * 2);
    c->w_dpart.alloc(sizeof(double) * W * kDirectSplitMax * N * 4);
    const int64_t hs = hi_stride(c);
    c->w_adjhi.alloc(sizeof(double) * std::max<int64_t>(1, W * 2 * hs));
    c->w_dcount.alloc(sizeof(int32_t));
    c->w_dlist.alloc(sizeof(int32_t) * 2 * W);
    c->w_perm.alloc(sizeof(int32_t) * W);
    c->w_Rs.alloc(sizeof(double) * W * N * 3);
    c->w_mds.alloc(W);
    c->w_sign_s.alloc(sizeof(double) * W);
    c->w_logabs_s.alloc(sizeof(double) * W);
    c->w_gl_s.alloc(sizeof(double) * W * N * 4);
    c->w_ws_s.alloc(sizeof(int32_t) * W);
    c->w_smstat.alloc(sizeof(unsigned long long) * 4);
    Work &k = c->wk;
    k.W = W;
    k.Wld = Wld;
    k.M = M;
    k.N = N;
    k.nmax = nmax;
    k.Upad = (int32_t)Upad;
    k.Vpad = (int32_t)Vpad;
    k.phi = c->w_phi.as<double>();
    k.E = c->w_E.as<int32_t>();
    k.X = c->w_X.as<double>();
    k.g0 = c->w_g0.as<double>();
    k.logdet0 = c->w_logdet0.as<double>();
    k.sign0 = c->w_sign0.as<double>();
    k.flag = c->w_flag.as<int32_t>();
    k.K = c->w_K.as<int32_t>();
    k.R64 = c->w_R64.as<double>();
    k.R32 = c->w_R32.as<float>();
    k.uv64 = c->w_uv64.as<double>();
    k.uv32 = c->w_uv32.as<float>();
    k.psi64 = c->w_psi64.as<double>();
    k.Rexp = c->w_Rexp.as<int32_t>();
    k.Kmax = c->w_Kmax.as<int32_t>();
    k.dpart = c->w_dpart.as<double>();
    k.hi_stride = hs;
    k.adjhi = hs > 0 ? c->w_adjhi.as<double>() : nullptr;
    k.dcount = c->w_dcount.as<int32_t>();
    k.dlist = c->w_dlist.as<int32_t>();
    k.perm = c->w_perm.as<int32_t>();
    k.Rs = c->w_Rs.as<double>();
    k.mds = c->w_mds.as<int8_t>();
    k.sign_s = c->w_sign_s.as<double>();
    k.logabs_s = c->w_logabs_s.as<double>();
    k.gl_s = c->w_gl_s.as<double>();
    k.ws_s = c->w_ws_s.as<int32_t>();
    k.Umax = (int32_t)std::max(c->sp[0].U, c->sp[1].U);
    k.smstat = c->w_smstat.as<unsigned long long>();
    k.smg64 = nullptr;
    k.smg32 = nullptr;
    c->wcap = W;
}

// Chain method: per-determinant derivative ratios for W walkers, allocated
// before any capture (a reallocation drops the captured graphs).
void ensure_chain(mdet_ctx *c, int64_t W) {
    if (c->method != MDET_METHOD_SM_CHAIN) return;
    const size_t need = sizeof(double) * (size_t)W * 2 * (size_t)c->wk.Umax * 4 *
                        (size_t)std::max(1, c->wk.nmax);
    if (c->w_smg.bytes < need) {
        c->drop_graphs();
        c->w_smg.alloc(need);
    }
    c->wk.smg64 = c->w_smg.as<double>();
    c->wk.smg32 = c->w_smg.as<float>();
}

// The work buffers of one evaluation of W walkers carved out of one device
// region starting at `base` (each piece 256-byte aligned, in a fixed order);
// returns the bytes the carving needs.  With base == nullptr only the size is
// computed.  Used by the allocation-free evaluation; the buffers, sizes and
// uses are those of ensure_work and ensure_chain.
size_t carve_work(const mdet_ctx *c, int64_t W, char *base, Work &k) {
    const int M = c->n_mo, N = c->n_up + c->n_dn;
    const int nmax = std::max(c->n_up, c->n_dn);
    const int64_t Upad = (c->sp[0].U + 63) / 64 * 64, Vpad = (c->sp[1].U + 63) / 64 * 64;
    const int64_t RV = Upad + Vpad;
    const int64_t Wld = (W + 63) / 64 * 64;
    const int32_t Umax = (int32_t)std::max(c->sp[0].U, c->sp[1].U);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? static_cast<void *>(base + off) : nullptr;
        off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return p;
    };
    k = Work{};
    k.W = W;
    k.Wld = Wld;
    k.M = M;
    k.N = N;
    k.nmax = nmax;
    k.Upad = (int32_t)Upad;
    k.Vpad = (int32_t)Vpad;
    k.Umax = Umax;
    k.phi = (double *)take(sizeof(double) * W * N * 5 * M);
    k.E = (int32_t *)take(sizeof(int32_t) * W * 2 * M);
    k.X = (double *)take(sizeof(double) * W * 2 * nmax * nmax);
    k.g0 = (double *)take(sizeof(double) * W * N * 4);
    k.logdet0 = (double *)take(sizeof(double) * W * 2);
    k.sign0 = (double *)take(sizeof(double) * W * 2);
    k.flag = (int32_t *)take(sizeof(int32_t) * W * 2);
    k.K = (int32_t *)take(sizeof(int32_t) * W * 2);
    k.R64 = (double *)take(sizeof(double) * Wld * RV);
    k.R32 = (float *)take(sizeof(float) * Wld * RV);
    k.uv64 = (double *)take(sizeof(double) * Wld * RV);
    k.uv32 = (float *)take(sizeof(float) * Wld * RV);
    k.psi64 = (double *)take(sizeof(double) * W * 2 * kPsiParts);
    k.Rexp = (int32_t *)take(sizeof(int32_t) * Wld * RV);
    k.Kmax = (int32_t *)take(sizeof(int32_t) * W * 2);
    k.dpart = (double *)take(sizeof(double) * W * kDirectSplitMax * N * 4);
    k.hi_stride = hi_stride(c);
    k.adjhi = (double *)take(sizeof(double) * W * 2 * k.hi_stride);
    if (k.hi_stride == 0) k.adjhi = nullptr;
    k.dcount = (int32_t *)take(sizeof(int32_t));
    k.dlist = (int32_t *)take(sizeof(int32_t) * 2 * W);
    k.perm = (int32_t *)take(sizeof(int32_t) * W);
    k.Rs = (double *)take(sizeof(double) * W * N * 3);
    k.mds = (int8_t *)take(W);
    k.sign_s = (double *)take(sizeof(double) * W);
    k.logabs_s = (double *)take(sizeof(double) * W);
    k.gl_s = (double *)take(sizeof(double) * W * N * 4);
    k.ws_s = (int32_t *)take(sizeof(int32_t) * W);
    k.smstat = (unsigned long long *)take(sizeof(unsigned long long) * 4);
    if (c->method == MDET_METHOD_SM_CHAIN) {
        void *g = take(sizeof(double) * (size_t)W * 2 * (size_t)Umax * 4 *
                       (size_t)std::max(1, nmax));
        k.smg64 = (double *)g;
        k.smg32 = (float *)g;
    }
    return off;
}

// Queue one evaluation (all kernels) on `st`; arguments already validated.
// With `fixed` the kernels use those work buffers (nothing is allocated and
// no timing events are recorded); otherwise the context's grow-only buffers.
void enqueue_eval(mdet_ctx *ctx, int64_t n_walk, const double *R_dev, int32_t precision,
                  const int8_t *max_degree_dev, double *sign_dev, double *logabs_dev,
                  double *gl_dev, int32_t *wstatus_dev, hipStream_t st,
                  const Work *fixed = nullptr) {
    const bool high = ctx->sp[0].high_degree || ctx->sp[1].high_degree;
    if (high && ctx->method != MDET_METHOD_SM_CHAIN)
        throw Status(MDET_EDEGREE, "excitation degree above " + std::to_string(MDET_MAX_DEGREE) +
                                       ": evaluate with MDET_METHOD_SM_CHAIN (mdet_set_method)");
    if (high && max_degree_dev)
        throw Status(MDET_EINVAL, "per-walker degree limits need excitation degrees <= " +
                                      std::to_string(MDET_MAX_DEGREE));
    if (!fixed) {
        ensure_work(ctx, n_walk);
        ensure_chain(ctx, n_walk);
    }
    KernelArgs a{};
    a.n_up = ctx->n_up;
    a.n_dn = ctx->n_dn;
    a.N = ctx->n_up + ctx->n_dn;
    a.M = ctx->n_mo;
    a.P = ctx->n_prim;
    a.nmax = std::max(ctx->n_up, ctx->n_dn);
    a.kappa_max = ctx->kappa_max[precision == MDET_MIXED ? 1 : 0];
    a.prim = ctx->d_prim.as<Prim>();
    a.prim_dn = ctx->two_sets ? ctx->d_prim_dn.as<Prim>() : a.prim;
    for (int s = 0; s < 2; ++s) {
        SpinDev &d = a.sp[s];
        d.n = ctx->sp[s].n;
        d.e0 = s == 0 ? 0 : ctx->n_up;
        d.U = (int32_t)ctx->sp[s].U;
        d.nchunk = (int32_t)ctx->sp[s].chunk_det.size() - 1;
        {
            int32_t acc = 0;
            for (int k = 0; k <= MDET_MAX_DEGREE; ++k) {
                acc += (int32_t)ctx->sp[s].n_by_degree[k];
                d.deg_end[k] = acc;
            }
            d.deg_end[MDET_MAX_DEGREE] += (int32_t)ctx->sp[s].n_above;  // the last bucket: all the rest
        }
        d.occ0 = ctx->sp[s].d_occ0.as<int32_t>();
        d.desc = ctx->sp[s].d_desc.as<DetDesc>();
        d.desc_hi = ctx->sp[s].d_desc_hi.as<DetDescHi>();
        d.hi_off = ctx->sp[s].d_hi_off.as<int32_t>();
        d.adj_off = ctx->sp[s].d_adj_off.as<int32_t>();
        d.chunk_det = ctx->sp[s].d_chunk_det.as<int32_t>();
        d.gent = ctx->sp[s].d_gent.as<uint32_t>();
        d.sm_exec = ctx->sp[s].d_sm_exec.as<int32_t>();
        d.sm_occ = ctx->sp[s].d_sm_occ.as<uint16_t>();
        d.sm_off = ctx->sp[s].d_sm_off.as<int32_t>();
        d.sm_sub = ctx->sp[s].d_sm_sub.as<uint32_t>();
    }
    a.C.U = (int32_t)ctx->sp[0].U;
    a.C.V = (int32_t)ctx->sp[1].U;
    a.C.Z = ctx->n_det;
    a.C.rptr = ctx->d_rptr.as<int32_t>();
    a.C.rcol = ctx->d_rcol.as<int32_t>();
    a.C.rval = ctx->d_rval.as<double>();
    a.C.cptr = ctx->d_cptr.as<int32_t>();
    a.C.crow = ctx->d_crow.as<int32_t>();
    a.C.cval = ctx->d_cval.as<double>();
    a.C.rval32 = ctx->d_rval32.as<float>();
    a.C.cval32 = ctx->d_cval32.as<float>();
    a.C.rseg64 = ctx->d_rseg.as<int32_t>();
    a.C.cseg64 = ctx->d_cseg.as<int32_t>();
    a.C.rseg32 = ctx->d_rseg32.as<int32_t>();
    a.C.cseg32 = ctx->d_cseg32.as<int32_t>();
    a.C.nch_r64 = ctx->nch_r;
    a.C.nch_c64 = ctx->nch_c;
    a.C.nch_r32 = ctx->nch_r32;
    a.C.nch_c32 = ctx->nch_c32;
    a.C.rdeg = ctx->d_rdeg.as<int32_t>();
    a.C.cdeg = ctx->d_cdeg.as<int32_t>();
    a.cfg = ctx->cfg_for(n_walk, precision, max_degree_dev != nullptr);
    a.method = ctx->method;
    a.sm_threshold = ctx->sm_threshold;
    a.sm_chunk = ctx->sm_chunk;
    if (a.method == MDET_METHOD_SM_CHAIN && !fixed) ctx->sm_ran = true;  // counters in ctx->wk
    a.wk = fixed ? *fixed : ctx->wk;
    a.W = n_walk;
    a.R = R_dev;
    a.max_degree = max_degree_dev;
    a.precision = precision;
    a.sign_out = sign_dev;
    a.logabs_out = logabs_dev;
    a.gl_out = gl_dev;
    a.wstatus = wstatus_dev;
    a.ev_mask = kernels_of_method(a.method) & ctx->prof_user_mask;
    hipEvent_t *ev = (ctx->profiling && !fixed) ? ctx->next_event_set(a.ev_mask) : nullptr;
    HIP_OK(launch_eval(a, st, ev, fixed ? nullptr : &ctx->aux));
    if (ctx->jastrow_on)
        launch_jastrow(n_walk, a.N, a.n_up, ctx->jastrow, R_dev, logabs_dev, gl_dev, st);
}

template <typename T>
T *grow(DevBuf &b, int64_t count) {
    const size_t need = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    if (b.bytes < need) b.alloc(need);
    return b.as<T>();
}

// VMC / MLP buffers for W walkers and an MLP of hidden width H
void ensure_vmc(mdet_ctx *c, int64_t W, int H) {
    const int N = c->n_up + c->n_dn;
    const MlpShape sh{3 * N, H, 4 * N};
    if (W <= c->vcap && sh.n_hid == c->mshape.n_hid) return;
    const int64_t Wc = std::max(W, c->vcap);
    grow<double>(c->v_Rp, Wc * N * 3);
    grow<double>(c->v_signp, Wc);
    grow<double>(c->v_logabsp, Wc);
    grow<double>(c->v_glp, Wc * N * 4);
    grow<int32_t>(c->v_wsp, Wc);
    grow<double>(c->v_signR, Wc);
    grow<double>(c->v_logabsR, Wc);
    grow<double>(c->v_glR, Wc * N * 4);
    grow<int32_t>(c->v_wsR, Wc);
    if (H > 0) {
        grow<float>(c->m_X, Wc * sh.n_in);
        grow<float>(c->m_Xp, Wc * sh.n_in);
        grow<float>(c->m_h1a, Wc * H);
        grow<float>(c->m_h2a, Wc * H);
        grow<float>(c->m_h1b, Wc * H);
        grow<float>(c->m_h2b, Wc * H);
        grow<float>(c->m_O1, Wc * sh.n_out);
        grow<float>(c->m_O2, Wc * sh.n_out);
        grow<float>(c->m_wh1, Wc * H);
        grow<float>(c->m_wh2, Wc * H);
        grow<float>(c->m_dO1, Wc * sh.n_out);
        grow<float>(c->m_dO2, Wc * sh.n_out);
        grow<float>(c->m_dX2, Wc * sh.n_in);
        grow<double>(c->m_gRp, Wc * sh.n_in);
        grow<double>(c->m_gell, Wc);
        grow<double>(c->m_Jw, Wc);
        grow<float>(c->m_grad, sh.n_params());
        c->mshape = sh;
    }
    c->vcap = Wc;
}

}  // namespace

namespace {
std::vector<Prim> pack_primitives(int32_t n_mo, int32_t n_prim, const int32_t *pow_abc,
                                  const double *alpha, const double *coef) {
    require(pow_abc && alpha && coef, MDET_EINVAL, "null orbital array");
    std::vector<Prim> pr((size_t)n_mo * n_prim);
    for (int64_t t = 0; t < (int64_t)n_mo * n_prim; ++t) {
        Prim &p = pr[t];
        p.alpha = alpha[t];
        p.coef = coef[t];
        p.a = pow_abc[3 * t];
        p.b = pow_abc[3 * t + 1];
        p.c = pow_abc[3 * t + 2];
        p.pad = 0;
        require(p.a >= 0 && p.a <= 4 && p.b >= 0 && p.b <= 4 && p.c >= 0 && p.c <= 4,
                MDET_EINVAL, "monomial power outside 0..4");
        require(std::isfinite(p.alpha) && p.alpha > 0.0 && std::isfinite(p.coef), MDET_EINVAL,
                "exponents must be finite and positive, coefficients finite");
    }
    return pr;
}
}  // namespace

extern "C" {


mdet_status mdet_create(mdet_ctx **out, int32_t hip_device) {
    if (!out) return MDET_EINVAL;
    *out = nullptr;
    if (hip_device == -1) {
        mdet_ctx *c = new (std::nothrow) mdet_ctx();
        if (!c) return MDET_ENOMEM;
        c->device = -1;
        c->host_only = true;
        *out = c;
        return MDET_OK;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
        return MDET_EHIP;
    if (hipSetDevice(hip_device) != hipSuccess) return MDET_EHIP;
    mdet_ctx *c = new (std::nothrow) mdet_ctx();
    if (!c) return MDET_ENOMEM;
    c->device = hip_device;
    *out = c;
    return MDET_OK;
}

void mdet_destroy(mdet_ctx *ctx) {
    if (!ctx) return;
    if (!ctx->host_only) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
    }
    ctx->drop_expansion();
    ctx->d_prim.release();
    ctx->d_prim_dn.release();
    ctx->drop_graphs();
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    ctx->drop_aux();
    ctx->drop_vmc();
    ctx->drop_profile_events();
    delete ctx;
}

const char *mdet_last_error(const mdet_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }


mdet_status mdet_init_orbitals(mdet_ctx *ctx, int32_t n_mo, int32_t n_prim, const int32_t *pow_abc,
                               const double *alpha, const double *coef) {
    return guarded(ctx, [&] {
        require(n_mo >= 1 && n_mo <= MDET_MAX_MO, MDET_EDIM, "n_mo out of range");
        require(n_prim >= 1 && n_prim <= 16, MDET_EDIM, "n_prim out of range");
        std::vector<Prim> pr = pack_primitives(n_mo, n_prim, pow_abc, alpha, coef);
        if (!ctx->host_only) HIP_OK(hipSetDevice(ctx->device));
        ctx->drop_expansion();
        if (!ctx->host_only) ctx->d_prim.upload(pr);
        ctx->prim.swap(pr);
        ctx->two_sets = false;
        ctx->prim_dn.clear();
        ctx->d_prim_dn.release();
        ctx->n_mo = n_mo;
        ctx->n_prim = n_prim;
        ctx->have_orb = true;
    });
}

mdet_status mdet_init_orbitals_dn(mdet_ctx *ctx, const int32_t *pow_abc, const double *alpha,
                                  const double *coef) {
    return guarded(ctx, [&] {
        require(ctx->have_orb, MDET_ESTATE, "mdet_init_orbitals must come first");
        std::vector<Prim> pr = pack_primitives(ctx->n_mo, ctx->n_prim, pow_abc, alpha, coef);
        if (!ctx->host_only) {
            HIP_OK(hipSetDevice(ctx->device));
            HIP_OK(hipDeviceSynchronize());  // no evaluation may still read the old set
            ctx->d_prim_dn.upload(pr);
        }
        ctx->prim_dn.swap(pr);
        ctx->two_sets = true;
        ctx->drop_graphs();
    });
}

mdet_status mdet_set_expansion(mdet_ctx *ctx, int32_t n_up, int32_t n_dn, int32_t n_int,
                               int64_t n_det, const uint64_t *det_up, const uint64_t *det_dn,
                               const double *c) {
    return guarded(ctx, [&] {
        const auto t0 = std::chrono::steady_clock::now();
        require(ctx->have_orb, MDET_ESTATE, "mdet_init_orbitals must come first");
        require(det_up && det_dn && c, MDET_EINVAL, "null expansion array");
        require(n_det >= 1 && n_det <= INT32_MAX, MDET_EDIM, "n_det out of range");
        require(n_up >= n_dn, MDET_ESPIN, "n_up < n_dn: the up spin must hold the larger count");
        require(n_dn >= 1 && n_up <= MDET_MAX_SPIN_ELEC, MDET_EDIM, "electron count out of range");
        require(n_det <= (int64_t)INT32_MAX / 2, MDET_EDIM, "n_det too large");
        require(n_up <= ctx->n_mo, MDET_EDIM, "more electrons of one spin than orbitals");
        require((int64_t)n_up * ctx->n_mo <= 6144, MDET_EDIM,
                "n_up * n_mo above 6144 (per-walker tables must fit in LDS)");
        require(n_int == (ctx->n_mo + 63) / 64, MDET_EORBITAL, "n_int must equal ceil(n_mo/64)");
        for (int64_t k = 0; k < n_det; ++k)
            require(std::isfinite(c[k]), MDET_EINVAL, "non-finite coefficient");
        if (!ctx->host_only) HIP_OK(hipSetDevice(ctx->device));
        ctx->drop_expansion();
        SpinHost sp[2];
        sp[0].n = n_up;
        sp[1].n = n_dn;
        std::vector<int32_t> pos_u, pos_d;
        unique_spin_list(det_up, n_det, n_int, sp[0], pos_u);
        unique_spin_list(det_dn, n_det, n_int, sp[1], pos_d);
        validate_spin(sp[0], n_int, ctx->n_mo, "up");
        validate_spin(sp[1], n_int, ctx->n_mo, "down");
        const int64_t U = sp[0].U, V = sp[1].U;
        // column-major coordinate order: key U*j + i
        std::vector<int64_t> order(n_det);
        std::iota(order.begin(), order.end(), 0);
        std::vector<int64_t> key(n_det);
        for (int64_t k = 0; k < n_det; ++k) key[k] = U * (int64_t)pos_d[k] + pos_u[k];
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
            return key[a] < key[b] || (key[a] == key[b] && a < b);
        });
        for (int64_t t = 1; t < n_det; ++t)
            if (key[order[t]] == key[order[t - 1]])
                throw Status(MDET_EDUPLICATE, "product (det_up, det_dn) given twice, at positions " +
                                                  std::to_string(order[t - 1]) + " and " +
                                                  std::to_string(order[t]));
        int64_t kref = 0;
        for (int64_t k = 1; k < n_det; ++k)
            if (std::fabs(c[k]) > std::fabs(c[kref])) kref = k;
        sp[0].ref = pos_u[kref];
        sp[1].ref = pos_d[kref];
        analyse_spin(sp[0], n_int, ctx->n_mo);
        analyse_spin(sp[1], n_int, ctx->n_mo);
        chain_lists(sp[0], n_int);
        chain_lists(sp[1], n_int);

        std::vector<int32_t> row_i(n_det), col_j(n_det);
        std::vector<double> val(n_det);
        std::vector<int64_t> src(n_det);
        for (int64_t t = 0; t < n_det; ++t) {
            const int64_t k = order[t];
            row_i[t] = pos_u[k];
            col_j[t] = pos_d[k];
            val[t] = c[k];
            src[t] = k;
        }
        // sparse C in execution indices: CSR over up rows and CSC over down columns
        std::vector<int32_t> rptr(U + 1, 0), cptr(V + 1, 0);
        for (int64_t t = 0; t < n_det; ++t) {
            rptr[sp[0].exec_of[row_i[t]] + 1]++;
            cptr[sp[1].exec_of[col_j[t]] + 1]++;
        }
        for (int64_t i = 0; i < U; ++i) rptr[i + 1] += rptr[i];
        for (int64_t j = 0; j < V; ++j) cptr[j + 1] += cptr[j];
        std::vector<int32_t> rcol(n_det), crow(n_det);
        std::vector<double> rval(n_det), cval(n_det);
        {
            std::vector<int32_t> fr(rptr.begin(), rptr.end() - 1), fc(cptr.begin(), cptr.end() - 1);
            // visit entries in (exec col, exec row) order so both structures are sorted
            std::vector<int64_t> ord(n_det);
            std::iota(ord.begin(), ord.end(), 0);
            std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
                const int64_t ja = sp[1].exec_of[col_j[a]], jb = sp[1].exec_of[col_j[b]];
                if (ja != jb) return ja < jb;
                return sp[0].exec_of[row_i[a]] < sp[0].exec_of[row_i[b]];
            });
            for (int64_t t : ord) {
                const int32_t ie = sp[0].exec_of[row_i[t]], je = sp[1].exec_of[col_j[t]];
                rcol[fr[ie]] = je;
                rval[fr[ie]++] = val[t];
                crow[fc[je]] = ie;
                cval[fc[je]++] = val[t];
            }
        }

        // entries of each CSR row / CSC column whose other determinant has degree <= d
        constexpr int DD = MDET_MAX_DEGREE + 1;
        std::vector<int32_t> rdeg((size_t)U * DD), cdeg((size_t)V * DD);
        {
            std::vector<int> deg_up(U), deg_dn(V);
            // degrees above MDET_MAX_DEGREE (chain method only) share the last bucket
            for (int64_t e = 0; e < U; ++e) deg_up[e] = std::min<int>(sp[0].desc[e].s, MDET_MAX_DEGREE);
            for (int64_t e = 0; e < V; ++e) deg_dn[e] = std::min<int>(sp[1].desc[e].s, MDET_MAX_DEGREE);
            for (int64_t i = 0; i < U; ++i)
                for (int d = 0; d < DD; ++d) {
                    int32_t k = rptr[i];
                    while (k < rptr[i + 1] && deg_dn[rcol[k]] <= d) ++k;
                    rdeg[(size_t)i * DD + d] = k;
                }
            for (int64_t j = 0; j < V; ++j)
                for (int d = 0; d < DD; ++d) {
                    int32_t k = cptr[j];
                    while (k < cptr[j + 1] && deg_up[crow[k]] <= d) ++k;
                    cdeg[(size_t)j * DD + d] = k;
                }
        }
        int32_t nch_r = 1, nch_c = 1, nch_r32 = 1, nch_c32 = 1;
        std::vector<int32_t> rseg = chunk_segments(rptr, rcol, U, V, kSpmmCols64, nch_r);
        std::vector<int32_t> cseg = chunk_segments(cptr, crow, V, U, kSpmmCols64, nch_c);
        std::vector<int32_t> rseg32 = chunk_segments(rptr, rcol, U, V, kSpmmCols32, nch_r32);
        std::vector<int32_t> cseg32 = chunk_segments(cptr, crow, V, U, kSpmmCols32, nch_c32);
        for (int s = 0; s < 2 && !ctx->host_only; ++s) {
            sp[s].d_occ0.upload(sp[s].occ0);
            sp[s].d_desc.upload(sp[s].desc);
            sp[s].d_adj_off.upload(sp[s].adj_off);
            sp[s].d_chunk_det.upload(sp[s].chunk_det);
            sp[s].d_gent.upload(sp[s].gent);
            sp[s].d_sm_exec.upload(sp[s].sm_exec);
            sp[s].d_sm_occ.upload(sp[s].sm_occ);
            sp[s].d_sm_off.upload(sp[s].sm_off);
            sp[s].d_sm_sub.upload(sp[s].sm_sub);
            sp[s].d_desc_hi.upload(sp[s].desc_hi);
            sp[s].d_hi_off.upload(sp[s].hi_off);
        }
        if (!ctx->host_only) {
            ctx->d_rptr.upload(rptr);
            ctx->d_rcol.upload(rcol);
            ctx->d_rval.upload(rval);
            ctx->d_cptr.upload(cptr);
            ctx->d_crow.upload(crow);
            ctx->d_cval.upload(cval);
            ctx->d_rval32.upload(std::vector<float>(rval.begin(), rval.end()));
            ctx->d_cval32.upload(std::vector<float>(cval.begin(), cval.end()));
            ctx->d_rseg.upload(rseg);
            ctx->d_cseg.upload(cseg);
            ctx->d_rseg32.upload(rseg32);
            ctx->d_cseg32.upload(cseg32);
            ctx->d_rdeg.upload(rdeg);
            ctx->d_cdeg.upload(cdeg);
        }
        ctx->nch_r = nch_r;
        ctx->nch_c = nch_c;
        ctx->nch_r32 = nch_r32;
        ctx->nch_c32 = nch_c32;
        for (int s = 0; s < 2; ++s) {
            ctx->sp[s].n = sp[s].n;
            ctx->sp[s].U = sp[s].U;
            ctx->sp[s].uniq.swap(sp[s].uniq);
            ctx->sp[s].ref = sp[s].ref;
            ctx->sp[s].occ0.swap(sp[s].occ0);
            ctx->sp[s].exec_of.swap(sp[s].exec_of);
            ctx->sp[s].pub_of.swap(sp[s].pub_of);
            ctx->sp[s].desc.swap(sp[s].desc);
            ctx->sp[s].desc_hi.swap(sp[s].desc_hi);
            ctx->sp[s].hi_off.swap(sp[s].hi_off);
            std::swap(ctx->sp[s].d_desc_hi, sp[s].d_desc_hi);
            std::swap(ctx->sp[s].d_hi_off, sp[s].d_hi_off);
            for (int k = 0; k <= MDET_MAX_DEGREE; ++k) ctx->sp[s].n_by_degree[k] = sp[s].n_by_degree[k];
            ctx->sp[s].high_degree = sp[s].high_degree;
            ctx->sp[s].n_above = sp[s].n_above;
            ctx->sp[s].adj_off.swap(sp[s].adj_off);
            ctx->sp[s].chunk_det.swap(sp[s].chunk_det);
            ctx->sp[s].gent.swap(sp[s].gent);
            std::swap(ctx->sp[s].d_occ0, sp[s].d_occ0);
            std::swap(ctx->sp[s].d_desc, sp[s].d_desc);
            std::swap(ctx->sp[s].d_adj_off, sp[s].d_adj_off);
            std::swap(ctx->sp[s].d_chunk_det, sp[s].d_chunk_det);
            std::swap(ctx->sp[s].d_gent, sp[s].d_gent);
            ctx->sp[s].sm_exec.swap(sp[s].sm_exec);
            ctx->sp[s].sm_occ.swap(sp[s].sm_occ);
            ctx->sp[s].sm_off.swap(sp[s].sm_off);
            ctx->sp[s].sm_sub.swap(sp[s].sm_sub);
            std::swap(ctx->sp[s].d_sm_exec, sp[s].d_sm_exec);
            std::swap(ctx->sp[s].d_sm_occ, sp[s].d_sm_occ);
            std::swap(ctx->sp[s].d_sm_off, sp[s].d_sm_off);
            std::swap(ctx->sp[s].d_sm_sub, sp[s].d_sm_sub);
        }
        ctx->row_i.swap(row_i);
        ctx->col_j.swap(col_j);
        ctx->val.swap(val);
        ctx->src_pos.swap(src);
        ctx->n_up = n_up;
        ctx->n_dn = n_dn;
        ctx->n_int = n_int;
        ctx->n_det = n_det;
        ctx->have_exp = true;
        ctx->prep_seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    });
}

mdet_status mdet_norm_truncation(int32_t n_int, int64_t n_det, const uint64_t *det_up,
                                 const uint64_t *det_dn, const double *c, double eps_up,
                                 double eps_dn, uint8_t *keep, int64_t *n_kept,
                                 int64_t *n_up_kept, int64_t *n_dn_kept) {
    try {
        if (!det_up || !det_dn || !c) return MDET_EINVAL;
        if (n_int < 1 || n_det < 1) return MDET_EDIM;
        if (!(eps_up >= 0.0) || !(eps_dn >= 0.0)) return MDET_EINVAL;
        SpinHost su, sd;
        std::vector<int32_t> pu, pd;
        unique_spin_list(det_up, n_det, n_int, su, pu);
        unique_spin_list(det_dn, n_det, n_int, sd, pd);
        double total = 0.0;
        std::vector<double> nu(su.U, 0.0), nd(sd.U, 0.0);
        for (int64_t k = 0; k < n_det; ++k) {  // input order
            const double c2 = c[k] * c[k];
            total += c2;
            nu[pu[k]] += c2;
            nd[pd[k]] += c2;
        }
        if (!(total > 0.0)) return MDET_EINVAL;
        std::vector<uint8_t> ku(su.U, 0), kd(sd.U, 0), used_u(su.U, 0), used_d(sd.U, 0);
        for (int64_t i = 0; i < su.U; ++i) ku[i] = nu[i] / total > eps_up;
        for (int64_t j = 0; j < sd.U; ++j) kd[j] = nd[j] / total > eps_dn;
        int64_t nk = 0, nuk = 0, ndk = 0;
        for (int64_t k = 0; k < n_det; ++k) {
            const uint8_t kk = ku[pu[k]] && kd[pd[k]];
            if (keep) keep[k] = kk;
            if (!kk) continue;
            ++nk;
            if (!used_u[pu[k]]) {
                used_u[pu[k]] = 1;
                ++nuk;
            }
            if (!used_d[pd[k]]) {
                used_d[pd[k]] = 1;
                ++ndk;
            }
        }
        if (n_kept) *n_kept = nk;
        if (n_up_kept) *n_up_kept = nuk;
        if (n_dn_kept) *n_dn_kept = ndk;
        return MDET_OK;
    } catch (const std::bad_alloc &) {
        return MDET_ENOMEM;
    } catch (...) {
        return MDET_EINVAL;
    }
}

mdet_status mdet_get_indexing(const mdet_ctx *cctx, int64_t *n_uniq_up, int64_t *n_uniq_dn,
                              uint64_t *uniq_up, uint64_t *uniq_dn, int32_t *row_i, int32_t *col_j,
                              double *val, int64_t *src_pos, int64_t *ref_up, int64_t *ref_dn) {
    mdet_ctx *ctx = const_cast<mdet_ctx *>(cctx);
    return guarded(ctx, [&] {
        require(ctx->have_exp, MDET_ESTATE, "no expansion loaded");
        if (n_uniq_up) *n_uniq_up = ctx->sp[0].U;
        if (n_uniq_dn) *n_uniq_dn = ctx->sp[1].U;
        if (uniq_up) std::memcpy(uniq_up, ctx->sp[0].uniq.data(), sizeof(uint64_t) * ctx->sp[0].uniq.size());
        if (uniq_dn) std::memcpy(uniq_dn, ctx->sp[1].uniq.data(), sizeof(uint64_t) * ctx->sp[1].uniq.size());
        if (row_i) std::memcpy(row_i, ctx->row_i.data(), sizeof(int32_t) * ctx->n_det);
        if (col_j) std::memcpy(col_j, ctx->col_j.data(), sizeof(int32_t) * ctx->n_det);
        if (val) std::memcpy(val, ctx->val.data(), sizeof(double) * ctx->n_det);
        if (src_pos) std::memcpy(src_pos, ctx->src_pos.data(), sizeof(int64_t) * ctx->n_det);
        if (ref_up) *ref_up = ctx->sp[0].ref;
        if (ref_dn) *ref_dn = ctx->sp[1].ref;
    });
}

mdet_status mdet_eval_walkers(mdet_ctx *ctx, int64_t n_walk, const double *R_dev, int32_t precision,
                              const int8_t *max_degree_dev, double *sign_dev, double *logabs_dev,
                              double *gl_dev, int32_t *wstatus_dev, void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context (hip_device -1) cannot evaluate");
        require(ctx->have_exp, MDET_ESTATE, "mdet_set_expansion must come first");
        require(n_walk >= 0 && n_walk <= (int64_t)1 << 30, MDET_EDIM, "n_walk out of range");
        require(precision == MDET_FP64 || precision == MDET_MIXED, MDET_EINVAL, "unknown precision");
        if (n_walk == 0) return;
        require(R_dev && sign_dev && logabs_dev && gl_dev, MDET_EINVAL, "null output pointer");
        HIP_OK(hipSetDevice(ctx->device));
        enqueue_eval(ctx, n_walk, R_dev, precision, max_degree_dev, sign_dev, logabs_dev, gl_dev,
                     wstatus_dev, static_cast<hipStream_t>(hip_stream));
    });
}

mdet_status mdet_eval_walkers_noalloc(mdet_ctx *ctx, int64_t n_walk, const double *R_dev,
                                      int32_t precision, const int8_t *max_degree_dev,
                                      double *sign_dev, double *logabs_dev, double *gl_dev,
                                      int32_t *wstatus_dev, void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context (hip_device -1) cannot evaluate");
        require(ctx->have_exp, MDET_ESTATE, "mdet_set_expansion must come first");
        require(n_walk >= 0 && n_walk <= (int64_t)1 << 30, MDET_EDIM, "n_walk out of range");
        require(precision == MDET_FP64 || precision == MDET_MIXED, MDET_EINVAL, "unknown precision");
        if (n_walk == 0) return;
        require(R_dev && sign_dev && logabs_dev && gl_dev, MDET_EINVAL, "null output pointer");
        Work wk;
        const size_t need = carve_work(ctx, n_walk, nullptr, wk);
        if (need > kNoallocBytes)
            throw Status(MDET_EDIM, "mdet_eval_walkers_noalloc: " + std::to_string(n_walk) +
                                        " walkers need " + std::to_string(need) +
                                        " bytes of scratch, more than its " +
                                        std::to_string(kNoallocBytes) + " bytes");
        HIP_OK(hipSetDevice(ctx->device));
        void *base = nullptr;
        HIP_OK(noalloc_scratch(ctx->device, &base));
        carve_work(ctx, n_walk, static_cast<char *>(base), wk);
        enqueue_eval(ctx, n_walk, R_dev, precision, max_degree_dev, sign_dev, logabs_dev, gl_dev,
                     wstatus_dev, static_cast<hipStream_t>(hip_stream), &wk);
    });
}

mdet_status mdet_set_profiling(mdet_ctx *ctx, int32_t enable) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        HIP_OK(hipSetDevice(ctx->device));
        ctx->harvest_all();
        if (enable && ctx->prof_ev.empty()) {
            ctx->prof_ev.assign((size_t)mdet_ctx::kRing * mdet_ctx::kSetEvents, nullptr);
            for (auto &e : ctx->prof_ev) HIP_OK(hipEventCreate(&e));
        }
        ctx->profiling = enable != 0;
        ctx->prof_user_mask = 0xffffffffu;
        for (double &m : ctx->prof_ms) m = 0.0;
        ctx->prof_calls = 0;
    });
}

mdet_status mdet_set_profiling_mask(mdet_ctx *ctx, uint32_t mask) {
    const mdet_status st = mdet_set_profiling(ctx, mask != 0);
    if (st == MDET_OK) ctx->prof_user_mask = mask ? mask : 0xffffffffu;
    return st;
}

mdet_status mdet_get_kernel_times(mdet_ctx *ctx, int32_t capacity, double *ms_total,
                                  const char **names, int32_t *n_kernels, int64_t *n_calls) {
    return guarded(ctx, [&] {
        ctx->harvest_all();
        if (n_kernels) *n_kernels = kNumKernels;
        if (n_calls) *n_calls = ctx->prof_calls;
        for (int k = 0; k < kNumKernels && k < capacity; ++k) {
            if (ms_total) ms_total[k] = ctx->prof_ms[k];
            if (names) names[k] = kernel_name(k);
        }
    });
}

mdet_status mdet_set_fallback_threshold(mdet_ctx *ctx, int32_t precision, double kappa_max) {
    return guarded(ctx, [&] {
        require(precision == MDET_FP64 || precision == MDET_MIXED || precision == -1,
                MDET_EINVAL, "precision must be MDET_FP64, MDET_MIXED or -1 (both)");
        require(kappa_max > 0.0, MDET_EINVAL, "threshold must be positive");
        if (precision != MDET_MIXED) ctx->kappa_max[0] = kappa_max;
        if (precision != MDET_FP64) ctx->kappa_max[1] = kappa_max;
        ctx->drop_graphs();  // captured steps hold the threshold by value
    });
}

mdet_status mdet_set_method(mdet_ctx *ctx, int32_t method, double sm_threshold,
                            int32_t sm_chunk) {
    return guarded(ctx, [&] {
        require(method == MDET_METHOD_TABLE || method == MDET_METHOD_SM_CHAIN, MDET_EINVAL,
                "unknown method");
        if (method == MDET_METHOD_SM_CHAIN) {
            require(sm_threshold > 0.0 && std::isfinite(sm_threshold), MDET_EINVAL,
                    "sm_threshold must be positive and finite");
            require(sm_chunk >= 1, MDET_EINVAL, "sm_chunk must be >= 1");
            ctx->sm_threshold = sm_threshold;
            ctx->sm_chunk = sm_chunk;
        }
        ctx->method = method;
        ctx->drop_graphs();
    });
}

mdet_status mdet_get_sm_counters(mdet_ctx *ctx, int64_t *out4) {
    return guarded(ctx, [&] {
        require(out4 != nullptr, MDET_EINVAL, "null output");
        for (int k = 0; k < 4; ++k) out4[k] = 0;
        if (ctx->host_only || !ctx->sm_ran || ctx->w_smstat.p == nullptr) return;
        HIP_OK(hipSetDevice(ctx->device));
        HIP_OK(hipDeviceSynchronize());
        unsigned long long h[4];
        HIP_OK(hipMemcpy(h, ctx->w_smstat.p, sizeof(h), hipMemcpyDeviceToHost));
        for (int k = 0; k < 4; ++k) out4[k] = (int64_t)h[k];
    });
}

mdet_status mdet_get_stats(const mdet_ctx *cctx, mdet_stats *out) {
    mdet_ctx *ctx = const_cast<mdet_ctx *>(cctx);
    return guarded(ctx, [&] {
        require(out != nullptr, MDET_EINVAL, "null stats pointer");
        std::memset(out, 0, sizeof(*out));
        out->n_mo = ctx->n_mo;
        out->n_prim = ctx->n_prim;
        if (ctx->have_exp) {
            out->n_det = ctx->n_det;
            out->n_uniq_up = ctx->sp[0].U;
            out->n_uniq_dn = ctx->sp[1].U;
            out->n_up = ctx->n_up;
            out->n_dn = ctx->n_dn;
            out->n_int = ctx->n_int;
            out->ref_up = ctx->sp[0].ref;
            out->ref_dn = ctx->sp[1].ref;
            for (int k = 0; k <= MDET_MAX_DEGREE; ++k) {
                out->n_by_degree_up[k] = ctx->sp[0].n_by_degree[k];
                out->n_by_degree_dn[k] = ctx->sp[1].n_by_degree[k];
            }
        }
        out->workspace_bytes = ctx->work_bytes();
        out->expansion_bytes = ctx->exp_bytes();
        out->preprocess_seconds = ctx->prep_seconds;
    });
}

mdet_status mdet_rng_fill(mdet_ctx *ctx, uint64_t seed, uint64_t stream_id, uint64_t step,
                          int64_t n, int32_t kind, double *out_dev, void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        require(n >= 0 && (kind == 0 || kind == 1), MDET_EINVAL, "bad size or kind");
        if (n == 0) return;
        require(out_dev != nullptr, MDET_EINVAL, "null output");
        HIP_OK(hipSetDevice(ctx->device));
        launch_philox(seed, stream_id, step, n, kind, out_dev, static_cast<hipStream_t>(hip_stream));
        HIP_OK(hipGetLastError());
    });
}

mdet_status mdet_vmc_step(mdet_ctx *ctx, int64_t n_walk, int32_t proposal, double step,
                          const float *mlp_params, int32_t n_hidden, double *R_dev,
                          double *sign_dev, double *logabs_dev, double *gl_dev,
                          const double *noise_dev, const double *uniform_dev,
                          double nuclear_charge, int32_t precision, double *elocal_dev,
                          int32_t *accepted_dev, void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        require(ctx->have_exp, MDET_ESTATE, "mdet_set_expansion must come first");
        require(proposal >= 0 && proposal <= 2, MDET_EINVAL, "unknown proposal");
        require(proposal == 2 || step > 0.0, MDET_EINVAL, "step must be positive");
        require(proposal != 2 || (mlp_params && n_hidden >= 1 && n_hidden <= 4096), MDET_EINVAL,
                "MLP proposal needs parameters and 1 <= n_hidden <= 4096");
        require(precision == MDET_FP64 || precision == MDET_MIXED, MDET_EINVAL, "unknown precision");
        require(n_walk >= 0 && n_walk <= (int64_t)1 << 24, MDET_EDIM, "n_walk out of range");
        if (n_walk == 0) return;
        require(R_dev && sign_dev && logabs_dev && gl_dev && noise_dev && uniform_dev &&
                    elocal_dev && accepted_dev,
                MDET_EINVAL, "null pointer");
        HIP_OK(hipSetDevice(ctx->device));
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const int N = ctx->n_up + ctx->n_dn;
        ensure_vmc(ctx, n_walk, proposal == 2 ? n_hidden : 0);
        double *Rp = ctx->v_Rp.as<double>();
        const float *o1 = nullptr, *o2 = nullptr;
        const MlpShape sh{3 * N, n_hidden, 4 * N};
        if (proposal == 2) {
            launch_to_f32(n_walk * 3 * N, R_dev, ctx->m_X.as<float>(), st);
            launch_mlp_forward(sh, mlp_params, n_walk, ctx->m_X.as<float>(), ctx->m_h1a.as<float>(),
                               ctx->m_h2a.as<float>(), ctx->m_O1.as<float>(), st);
            launch_mlp_propose(n_walk, N, R_dev, ctx->m_O1.as<float>(), noise_dev, Rp, st);
        } else {
            launch_vmc_propose(n_walk, N, proposal, step, R_dev, gl_dev, noise_dev, Rp, st);
        }
        enqueue_eval(ctx, n_walk, Rp, precision, nullptr, ctx->v_signp.as<double>(),
                     ctx->v_logabsp.as<double>(), ctx->v_glp.as<double>(), ctx->v_wsp.as<int32_t>(), st);
        if (proposal == 2) {
            launch_to_f32(n_walk * 3 * N, Rp, ctx->m_Xp.as<float>(), st);
            launch_mlp_forward(sh, mlp_params, n_walk, ctx->m_Xp.as<float>(), ctx->m_h1b.as<float>(),
                               ctx->m_h2b.as<float>(), ctx->m_O2.as<float>(), st);
            o1 = ctx->m_O1.as<float>();
            o2 = ctx->m_O2.as<float>();
        }
        launch_vmc_accept(n_walk, N, proposal, step, nuclear_charge, R_dev, sign_dev, logabs_dev,
                          gl_dev, Rp, ctx->v_signp.as<double>(), ctx->v_logabsp.as<double>(),
                          ctx->v_glp.as<double>(), uniform_dev, o1, o2, elocal_dev, accepted_dev, 0,
                          st);
        HIP_OK(hipGetLastError());
    });
}

mdet_status mdet_set_jastrow(mdet_ctx *ctx, int32_t enable, double b_ee, double a_en,
                             double b_en) {
    return guarded(ctx, [&] {
        if (enable) {
            require(std::isfinite(b_ee) && b_ee >= 0.0 && std::isfinite(a_en) &&
                        std::isfinite(b_en) && b_en >= 0.0,
                    MDET_EINVAL, "Jastrow parameters must be finite, b_ee and b_en >= 0");
            ctx->jastrow = JastrowParams{b_ee, a_en, b_en};
        }
        ctx->jastrow_on = enable != 0;
        ctx->drop_graphs();
    });
}

mdet_status mdet_dmc_step(mdet_ctx *ctx, int64_t n_walk, double tau, double e_trial,
                          double nuclear_charge, int32_t precision, double *R_dev,
                          double *sign_dev, double *logabs_dev, double *gl_dev, double *elocal_dev,
                          double *weight_dev, const double *noise_dev, const double *uniform_dev,
                          double comb_u, double *sums_dev, int32_t *accepted_dev,
                          void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        require(ctx->have_exp, MDET_ESTATE, "mdet_set_expansion must come first");
        require(tau > 0.0 && std::isfinite(tau) && std::isfinite(e_trial), MDET_EINVAL,
                "tau must be positive, e_trial finite");
        require(comb_u >= 0.0 && comb_u < 1.0, MDET_EINVAL, "comb_u must lie in [0, 1)");
        require(precision == MDET_FP64 || precision == MDET_MIXED, MDET_EINVAL, "unknown precision");
        require(n_walk >= 0 && n_walk <= (int64_t)1 << 24, MDET_EDIM, "n_walk out of range");
        if (n_walk == 0) return;
        require(R_dev && sign_dev && logabs_dev && gl_dev && elocal_dev && weight_dev && noise_dev &&
                    uniform_dev && sums_dev && accepted_dev,
                MDET_EINVAL, "null pointer");
        HIP_OK(hipSetDevice(ctx->device));
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const int N = ctx->n_up + ctx->n_dn;
        ensure_vmc(ctx, n_walk, 0);
        DmcWork d{};
        double *e_old = grow<double>(ctx->q_eold, n_walk);
        d.cum = grow<double>(ctx->q_cum, n_walk);
        d.src = grow<int32_t>(ctx->q_src, n_walk);
        d.R = grow<double>(ctx->q_R, n_walk * 3 * N);
        d.sign = grow<double>(ctx->q_sign, n_walk);
        d.logabs = grow<double>(ctx->q_logabs, n_walk);
        d.gl = grow<double>(ctx->q_gl, n_walk * 4 * N);
        d.elocal = grow<double>(ctx->q_el, n_walk);
        double *Rp = ctx->v_Rp.as<double>();
        launch_dmc_save(n_walk, elocal_dev, e_old, st);
        launch_vmc_propose(n_walk, N, 1, tau, R_dev, gl_dev, noise_dev, Rp, st);
        enqueue_eval(ctx, n_walk, Rp, precision, nullptr, ctx->v_signp.as<double>(),
                     ctx->v_logabsp.as<double>(), ctx->v_glp.as<double>(), ctx->v_wsp.as<int32_t>(), st);
        launch_vmc_accept(n_walk, N, 1, tau, nuclear_charge, R_dev, sign_dev, logabs_dev, gl_dev, Rp,
                          ctx->v_signp.as<double>(), ctx->v_logabsp.as<double>(),
                          ctx->v_glp.as<double>(), uniform_dev, nullptr, nullptr, elocal_dev,
                          accepted_dev, 1, st);
        launch_dmc_branch(n_walk, N, tau, e_trial, comb_u, e_old, accepted_dev, d, R_dev, sign_dev,
                          logabs_dev, gl_dev, elocal_dev, weight_dev, sums_dev, st);
        HIP_OK(hipGetLastError());
    });
}

mdet_status mdet_mlp_forward(mdet_ctx *ctx, int32_t n_in, int32_t n_hidden, int32_t n_out,
                             const float *params, int64_t batch, const float *X, float *Y,
                             void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        require(n_in >= 1 && n_hidden >= 1 && n_out >= 1 && batch >= 0, MDET_EINVAL, "bad shape");
        if (batch == 0) return;
        require(params && X && Y, MDET_EINVAL, "null pointer");
        HIP_OK(hipSetDevice(ctx->device));
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        float *h1 = grow<float>(ctx->m_h1a, batch * n_hidden);
        float *h2 = grow<float>(ctx->m_h2a, batch * n_hidden);
        launch_mlp_forward(MlpShape{n_in, n_hidden, n_out}, params, batch, X, h1, h2, Y, st);
        HIP_OK(hipGetLastError());
    });
}

mdet_status mdet_mlp_backward(mdet_ctx *ctx, int32_t n_in, int32_t n_hidden, int32_t n_out,
                              const float *params, int64_t batch, const float *X, const float *dY,
                              float *dparams, float *dX, void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        require(n_in >= 1 && n_hidden >= 1 && n_out >= 1 && batch >= 1, MDET_EINVAL, "bad shape");
        require(params && X && dY && dparams, MDET_EINVAL, "null pointer");
        HIP_OK(hipSetDevice(ctx->device));
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const MlpShape sh{n_in, n_hidden, n_out};
        float *h1 = grow<float>(ctx->m_h1a, batch * n_hidden);
        float *h2 = grow<float>(ctx->m_h2a, batch * n_hidden);
        float *O = grow<float>(ctx->m_O1, batch * n_out);
        float *w1 = grow<float>(ctx->m_wh1, batch * n_hidden);
        float *w2 = grow<float>(ctx->m_wh2, batch * n_hidden);
        launch_mlp_forward(sh, params, batch, X, h1, h2, O, st);
        launch_mlp_backward(sh, params, batch, X, h1, h2, dY, dparams, 0, dX, w1, w2, st);
        HIP_OK(hipGetLastError());
    });
}

mdet_status mdet_mlp_adam(mdet_ctx *ctx, int64_t n, float *params, const float *grads, float *m,
                          float *v, int32_t t, float lr, float beta1, float beta2, float eps,
                          void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        require(n >= 0 && t >= 1 && lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f &&
                    beta2 < 1.f && eps > 0.f,
                MDET_EINVAL, "bad Adam arguments");
        if (n == 0) return;
        require(params && grads && m && v, MDET_EINVAL, "null pointer");
        HIP_OK(hipSetDevice(ctx->device));
        launch_adam(n, params, grads, m, v, lr, beta1, beta2, eps, t,
                    static_cast<hipStream_t>(hip_stream));
        HIP_OK(hipGetLastError());
    });
}

mdet_status mdet_mlp_train_step(mdet_ctx *ctx, int64_t n_walk, int32_t n_hidden, float *params,
                                float *adam_m, float *adam_v, int32_t t, float lr,
                                const double *R_dev, const double *noise_dev, int32_t precision,
                                double jump_ref, int32_t objective, double nuclear_charge,
                                double *loss_dev, float *grad_dev, void *hip_stream) {
    return guarded(ctx, [&] {
        require(std::isfinite(jump_ref), MDET_EINVAL, "jump_ref must be finite");
        require(objective == MDET_OBJ_JUMP || objective == MDET_OBJ_POTENTIAL, MDET_EINVAL,
                "unknown training objective");
        require(std::isfinite(nuclear_charge), MDET_EINVAL, "nuclear charge must be finite");
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        require(ctx->have_exp, MDET_ESTATE, "mdet_set_expansion must come first");
        require(n_walk >= 1 && n_walk <= (int64_t)1 << 24 && n_hidden >= 1 && n_hidden <= 4096,
                MDET_EDIM, "bad batch or width");
        require(t >= 1 && lr > 0.f, MDET_EINVAL, "bad step count or learning rate");
        require(precision == MDET_FP64 || precision == MDET_MIXED, MDET_EINVAL, "unknown precision");
        require(params && adam_m && adam_v && R_dev && noise_dev && loss_dev, MDET_EINVAL,
                "null pointer");
        HIP_OK(hipSetDevice(ctx->device));
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const int N = ctx->n_up + ctx->n_dn;
        const MlpShape sh{3 * N, n_hidden, 4 * N};
        ensure_vmc(ctx, n_walk, n_hidden);
        double *Rp = ctx->v_Rp.as<double>();
        float *grad = grad_dev ? grad_dev : ctx->m_grad.as<float>();
        // ln|Psi(R)|, the network at R, the proposal, Psi and the network at R'
        enqueue_eval(ctx, n_walk, R_dev, precision, nullptr, ctx->v_signR.as<double>(),
                     ctx->v_logabsR.as<double>(), ctx->v_glR.as<double>(), ctx->v_wsR.as<int32_t>(), st);
        launch_to_f32(n_walk * 3 * N, R_dev, ctx->m_X.as<float>(), st);
        launch_mlp_forward(sh, params, n_walk, ctx->m_X.as<float>(), ctx->m_h1a.as<float>(),
                           ctx->m_h2a.as<float>(), ctx->m_O1.as<float>(), st);
        launch_mlp_propose(n_walk, N, R_dev, ctx->m_O1.as<float>(), noise_dev, Rp, st);
        enqueue_eval(ctx, n_walk, Rp, precision, nullptr, ctx->v_signp.as<double>(),
                     ctx->v_logabsp.as<double>(), ctx->v_glp.as<double>(), ctx->v_wsp.as<int32_t>(), st);
        launch_to_f32(n_walk * 3 * N, Rp, ctx->m_Xp.as<float>(), st);
        launch_mlp_forward(sh, params, n_walk, ctx->m_Xp.as<float>(), ctx->m_h1b.as<float>(),
                           ctx->m_h2b.as<float>(), ctx->m_O2.as<float>(), st);
        // loss and gradient: through the second evaluation, then the first
        launch_esjd_head(n_walk, N, R_dev, Rp, noise_dev, ctx->v_logabsR.as<double>(),
                         ctx->v_signp.as<double>(), ctx->v_logabsp.as<double>(),
                         ctx->v_glp.as<double>(), ctx->m_O1.as<float>(), ctx->m_O2.as<float>(),
                         ctx->m_dO2.as<float>(), ctx->m_gRp.as<double>(), ctx->m_gell.as<double>(),
                         ctx->m_Jw.as<double>(), jump_ref, objective, nuclear_charge, st);
        launch_mlp_backward(sh, params, n_walk, ctx->m_Xp.as<float>(), ctx->m_h1b.as<float>(),
                            ctx->m_h2b.as<float>(), ctx->m_dO2.as<float>(), grad, 0,
                            ctx->m_dX2.as<float>(), ctx->m_wh1.as<float>(), ctx->m_wh2.as<float>(), st);
        launch_esjd_chain(n_walk, N, noise_dev, ctx->m_O1.as<float>(), ctx->m_gRp.as<double>(),
                          ctx->m_dX2.as<float>(), ctx->m_gell.as<double>(), ctx->m_dO1.as<float>(), st);
        launch_mlp_backward(sh, params, n_walk, ctx->m_X.as<float>(), ctx->m_h1a.as<float>(),
                            ctx->m_h2a.as<float>(), ctx->m_dO1.as<float>(), grad, 1, nullptr,
                            ctx->m_wh1.as<float>(), ctx->m_wh2.as<float>(), st);
        launch_esjd_loss(n_walk, ctx->m_Jw.as<double>(), loss_dev, st);
        launch_adam(sh.n_params(), params, grad, adam_m, adam_v, lr, 0.9f, 0.999f, 1e-8f, t, st);
        HIP_OK(hipGetLastError());
    });
}

mdet_status mdet_set_launch_config(mdet_ctx *ctx, int32_t spmm_row_splits, int32_t direct_split,
                                   int32_t sort_walkers, int32_t overlap_fallback) {
    return guarded(ctx, [&] {
        require(spmm_row_splits >= 0 && spmm_row_splits <= kPsiParts, MDET_EINVAL,
                "spmm_row_splits must be 0 (auto) .. 16");
        require(direct_split >= 0 && direct_split <= kDirectSplitMax, MDET_EINVAL,
                "direct_split must be 0 (auto) .. 8");
        ctx->cfg = LaunchCfg{spmm_row_splits, direct_split, sort_walkers ? 1 : 0,
                             overlap_fallback ? 1 : 0};
        ctx->tuned.clear();
        ctx->drop_graphs();
    });
}

mdet_status mdet_get_launch_config(const mdet_ctx *cctx, int32_t *spmm_row_splits,
                                   int32_t *direct_split, int32_t *sort_walkers,
                                   int32_t *overlap_fallback) {
    mdet_ctx *ctx = const_cast<mdet_ctx *>(cctx);
    return guarded(ctx, [&] {
        if (spmm_row_splits) *spmm_row_splits = ctx->cfg.spmm_rsplit;
        if (direct_split) *direct_split = ctx->cfg.direct_split;
        if (sort_walkers) *sort_walkers = ctx->cfg.sort_walkers;
        if (overlap_fallback) *overlap_fallback = ctx->cfg.overlap_fallback;
    });
}

mdet_status mdet_eval_graph(mdet_ctx *ctx, int64_t n_walk, const double *R_dev, int32_t precision,
                            const int8_t *max_degree_dev, double *sign_dev, double *logabs_dev,
                            double *gl_dev, int32_t *wstatus_dev, void *hip_stream) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context (hip_device -1) cannot evaluate");
        require(ctx->have_exp, MDET_ESTATE, "mdet_set_expansion must come first");
        require(n_walk >= 0 && n_walk <= (int64_t)1 << 30, MDET_EDIM, "n_walk out of range");
        require(precision == MDET_FP64 || precision == MDET_MIXED, MDET_EINVAL, "unknown precision");
        if (n_walk == 0) return;
        require(R_dev && sign_dev && logabs_dev && gl_dev, MDET_EINVAL, "null output pointer");
        HIP_OK(hipSetDevice(ctx->device));
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        if (st == nullptr) {  // the legacy default stream cannot be captured: use a blocking stream of our own
            if (!ctx->own_stream) HIP_OK(hipStreamCreate(&ctx->own_stream));
            st = ctx->own_stream;
        }
        ensure_work(ctx, n_walk);  // any allocation happens before capture
        ensure_chain(ctx, n_walk);
        const void *key[7] = {R_dev, max_degree_dev, sign_dev, logabs_dev, gl_dev, wstatus_dev, nullptr};
        mdet_ctx::GraphEntry *hit = nullptr;
        for (auto &g : ctx->graphs)
            if (g.W == n_walk && g.precision == precision && g.stream == st &&
                std::equal(key, key + 7, g.ptr))
                hit = &g;
        if (!hit) {
            if (ctx->graphs.size() >= 8) {  // evict the least recently used
                auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                            [](const auto &x, const auto &y) { return x.last_use < y.last_use; });
                (void)hipGraphExecDestroy(lru->exec);
                ctx->graphs.erase(lru);
            }
            const bool prof = ctx->profiling;
            ctx->profiling = false;  // no event records inside a graph
            HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
                enqueue_eval(ctx, n_walk, R_dev, precision, max_degree_dev, sign_dev, logabs_dev,
                             gl_dev, wstatus_dev, st);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(st, &g);
                if (g) (void)hipGraphDestroy(g);
                ctx->profiling = prof;
                throw;
            }
            ctx->profiling = prof;
            hipGraph_t graph = nullptr;
            HIP_OK(hipStreamEndCapture(st, &graph));
            hipGraphExec_t exec = nullptr;
            const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIP_OK(e);
            mdet_ctx::GraphEntry ge{};
            ge.W = n_walk;
            std::copy(key, key + 7, ge.ptr);
            ge.precision = precision;
            ge.stream = st;
            ge.exec = exec;
            ctx->graphs.push_back(ge);
            hit = &ctx->graphs.back();
        }
        hit->last_use = ++ctx->graph_clock;
        HIP_OK(hipGraphLaunch(hit->exec, st));
    });
}

mdet_status mdet_autotune(mdet_ctx *ctx, int64_t n_walk, const double *R_dev, int32_t precision,
                          const int8_t *max_degree_dev, int32_t n_rep, mdet_tune_result *out) {
    return guarded(ctx, [&] {
        require(!ctx->host_only, MDET_ESTATE, "host-only context");
        require(ctx->have_exp, MDET_ESTATE, "mdet_set_expansion must come first");
        require(n_walk >= 1 && R_dev && n_rep >= 1 && n_rep <= 1000, MDET_EINVAL, "bad arguments");
        require(precision == MDET_FP64 || precision == MDET_MIXED, MDET_EINVAL, "unknown precision");
        HIP_OK(hipSetDevice(ctx->device));
        const int N = ctx->n_up + ctx->n_dn;
        DevBuf sg, la, gl, ws;
        sg.alloc(sizeof(double) * n_walk);
        la.alloc(sizeof(double) * n_walk);
        gl.alloc(sizeof(double) * n_walk * N * 4);
        ws.alloc(sizeof(int32_t) * n_walk);
        hipStream_t st = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const LaunchCfg saved = ctx->cfg;
        const bool prof = ctx->profiling;
        ctx->profiling = false;
        auto cleanup = [&] {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (st) (void)hipStreamDestroy(st);
            sg.release();
            la.release();
            gl.release();
            ws.release();
            ctx->profiling = prof;
        };
        try {
            HIP_OK(hipStreamCreate(&st));
            HIP_OK(hipEventCreate(&e0));
            HIP_OK(hipEventCreate(&e1));
            std::vector<LaunchCfg> cand;
            for (int rs : {0, 4, 8, 16})
                for (int ds : {0, 4, 8})
                    for (int ov : {1, 0})
                        for (int so : {1, 0}) {
                            if (!max_degree_dev && so == 0) continue;
                            cand.push_back(LaunchCfg{rs, ds, so, ov});
                        }
            const bool uneven = max_degree_dev != nullptr;
            // time the candidates with no remembered configuration for this shape
            ctx->tuned.erase(std::remove_if(ctx->tuned.begin(), ctx->tuned.end(),
                                            [&](const mdet_ctx::TunedShape &t) {
                                                return t.W == n_walk && t.precision == precision &&
                                                       t.uneven == (uneven ? 1 : 0);
                                            }),
                             ctx->tuned.end());
            double best = 1e300, first = 0.0;
            LaunchCfg best_cfg = saved;
            for (size_t c = 0; c < cand.size(); ++c) {
                ctx->cfg = cand[c];
                enqueue_eval(ctx, n_walk, R_dev, precision, max_degree_dev, sg.as<double>(),
                             la.as<double>(), gl.as<double>(), ws.as<int32_t>(), st);
                HIP_OK(hipEventRecord(e0, st));
                for (int r = 0; r < n_rep; ++r)
                    enqueue_eval(ctx, n_walk, R_dev, precision, max_degree_dev, sg.as<double>(),
                                 la.as<double>(), gl.as<double>(), ws.as<int32_t>(), st);
                HIP_OK(hipEventRecord(e1, st));
                HIP_OK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_OK(hipEventElapsedTime(&ms, e0, e1));
                const double per = ms / n_rep;
                if (c == 0) first = per;
                if (per < best) {
                    best = per;
                    best_cfg = cand[c];
                }
            }
            ctx->cfg = saved;
            if (ctx->tuned.size() >= 32) ctx->tuned.erase(ctx->tuned.begin());
            ctx->tuned.push_back(mdet_ctx::TunedShape{n_walk, precision, uneven ? 1 : 0, best_cfg});
            ctx->drop_graphs();
            if (out) {
                out->spmm_row_splits = best_cfg.spmm_rsplit;
                out->direct_split = best_cfg.direct_split;
                out->sort_walkers = best_cfg.sort_walkers;
                out->overlap_fallback = best_cfg.overlap_fallback;
                out->n_candidates = (int32_t)cand.size();
                out->best_ms = best;
                out->default_ms = first;
            }
        } catch (...) {
            ctx->cfg = saved;
            cleanup();
            throw;
        }
        cleanup();
    });
}

}  // extern "C"
