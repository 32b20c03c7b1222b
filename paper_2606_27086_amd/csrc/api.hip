// Host runtime and C ABI of libsmx (declared in include/smx.h).
//
// Owns device memory for operators (row-aligned CSR of A, row-aligned CSR of
// A^T, float64 row norms, reduced-precision value copies) and problems (bands,
// box, weights, iterate, per-slice state, reduction scratch, history), builds
// the per-iteration launch sequence, and captures it into HIP graphs.
#include "../../include/smx.h"
#include "smx_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace smx;

// The fixed device scratch of smx_slot_load_noalloc (32 MiB).
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct HipError {
    hipError_t e;
    const char *what;
};

inline void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw HipError{e, what};
}

int from_hip(const HipError &h)
{
    if (h.e == hipErrorOutOfMemory) return fail(SMX_ENOMEM, "%s: out of device memory", h.what);
    return fail(SMX_EDEVICE, "%s: %s", h.what, hipGetErrorString(h.e));
}

// Owning device allocation.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b, const char *what)
    {
        release();
        if (b == 0) b = 256;
        hip_check(hipMalloc(&p, b), what);
        bytes = b;
    }
    template <typename T>
    T *as() const
    {
        return static_cast<T *>(p);
    }
};

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// One row-aligned layout on the host before upload.
struct HostLayout {
    std::vector<int32_t> ptr;
    std::vector<int32_t> idx;
    std::vector<float> val;
    int64_t slots = 0;
};

// Pads every row to a multiple of kRowAlign entries (value 0, index of the
// row's last entry or 0).  Returns false if the padded size reaches 2^31.
bool pad_rows(int64_t rows, const int64_t *rp, const int32_t *idx, const float *val, HostLayout &L)
{
    L.ptr.resize(rows + 1);
    int64_t slots = 0;
    for (int64_t r = 0; r < rows; ++r) {
        L.ptr[r] = (int32_t)slots;
        slots += round_up(rp[r + 1] - rp[r], kRowAlign);
        if (slots >= (int64_t(1) << 31)) return false;
    }
    L.ptr[rows] = (int32_t)slots;
    L.slots = slots;
    L.idx.assign(slots, 0);
    L.val.assign(slots, 0.f);
    for (int64_t r = 0; r < rows; ++r) {
        int64_t s = rp[r], e = rp[r + 1], o = L.ptr[r];
        std::memcpy(&L.idx[o], idx + s, sizeof(int32_t) * (e - s));
        std::memcpy(&L.val[o], val + s, sizeof(float) * (e - s));
        const int32_t fill = (e > s) ? idx[e - 1] : 0;
        for (int64_t p = o + (e - s); p < L.ptr[r + 1]; ++p) L.idx[p] = fill;
    }
    return true;
}

// Row blocks for the streaming kernels: consecutive rows with at most kBlock
// rows and kStreamEntries padded entries per block; a longer row is a block
// of its own.
std::vector<int32_t> build_row_blocks(const std::vector<int32_t> &ptr, int64_t rows)
{
    std::vector<int32_t> rb;
    rb.push_back(0);
    int64_t r = 0;
    while (r < rows) {
        const int64_t start = r;
        if (ptr[r + 1] - ptr[r] > kStreamEntries) {
            ++r;
        } else {
            int64_t ent = 0;
            while (r < rows && r - start < kBlock && ent + (ptr[r + 1] - ptr[r]) <= kStreamEntries) {
                ent += ptr[r + 1] - ptr[r];
                ++r;
            }
        }
        rb.push_back((int32_t)r);
    }
    return rb;
}

struct DevLayout {
    int64_t rows = 0, slots = 0;
    DBuf ptr, idx, val32, val16, packed, rowblk; // packed: 16-bit value | 16-bit index << 16
    DBuf idx16; // 16-bit copy of idx beside the float32 values (index range <= 65536)
    int nblk = 0;
    float f16_scale = 1.f;
    RowBlocks blocks() const
    {
        RowBlocks r;
        r.rb = rowblk.as<int32_t>();
        r.nblk = nblk;
        return r;
    }
    SpView view(int vk) const
    {
        SpView v;
        v.ptr = ptr.as<int32_t>();
        v.idx = idx.as<int32_t>();
        v.val = (vk == VK_F32 || vk == VK_F32U16) ? val32.p : ((vk == VK_BF16P || vk == VK_F16P) ? packed.p : val16.p);
        if (vk == VK_F32U16) v.idx = idx16.as<int32_t>(); // read as uint16 by the kernels
        v.rows = rows;
        v.vscale_inv = (vk == VK_F16 || vk == VK_F16P) ? 1.f / f16_scale : 1.f;
        return v;
    }
};

// Device bytes of one layout: offsets, then per entry the 32-bit index and value
// when float32 is kept, and the reduced-precision value either alone (beside
// the index) or packed with a 16-bit index into one word.
size_t layout_bytes(int64_t rows, int64_t slots, bool f32, bool lp, bool packed, bool short_idx)
{
    const bool idx32 = f32 || !packed;
    return size_t(rows + 1) * 4 + (idx32 ? size_t(slots) * 4 : 0) + (f32 ? size_t(slots) * 4 : 0) +
           (lp ? size_t(slots) * (packed ? 4 : 2) : 0) + (f32 && short_idx ? size_t(slots) * 2 : 0);
}

float f16_scale_for(const std::vector<float> &v)
{
    float amax = 0.f;
    for (float a : v) amax = std::max(amax, std::fabs(a));
    if (!(amax > 0.f)) return 1.f;
    int e;
    const double mant = std::frexp((double)amax, &e);
    const int ce = (mant == 0.5) ? e - 1 : e; // ceil(log2(amax))
    return (float)std::ldexp(1.0, 14 - ce);
}

// Device scratch of smx_slot_load_noalloc: a fixed array in the library's
// code object (each device that loads the library holds its own copy until
// the process ends), so that entry point needs no allocation.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, never through the array's name.
constexpr size_t kScratchHead = 256; // flags of the staged-band check

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device (looked up once per
// device, with that device current).
void *scratch_on_current_device()
{
    int dev = 0;
    hip_check(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxDevices) throw HipError{hipErrorInvalidDevice, "scratch: device index"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

} // namespace

struct smx_operator {
    int device = 0;
    int64_t m = 0, n = 0, nnz = 0;
    int storage = SMX_STORE_F32;
    bool has_f32 = true;
    DevLayout csr, csc;
    DBuf panel_ptr;              // row panels of the column copy (m > kLdsPassFloats): (np+1) x n entry offsets
    DBuf panel_idx16;            // the column copy's rows as 16-bit offsets within their panel
    DBuf panel_packed;           // reduced-precision value | panel offset << 16 (when values are stored so)
    int panel_np = 0, panel_P = 0;
    DBuf q32, q16; // float64 row norms of the float32 and the reduced-precision operator
    DBuf zcol;     // DROP column factors 1/(nonzeros in column j), 0 for an empty column [n]
    // image operators: the column layout grouped by image tiles (TileView);
    // t_idx16 holds its 16-bit row positions for the float32 copy
    int img_rows = 0, img_cols = 0;
    DevLayout tiles;
    DBuf t_tcol, t_pptr, t_rptr, t_rlist, t_idx16;
    int t_ntiles = 0, t_max_rows = 0;
    bool has_tiles() const { return t_ntiles > 0; }
    TileView tile_view(int vk) const
    {
        TileView T;
        T.A = tiles.view(vk);
        if (vk == VK_F32) T.A.idx = t_idx16.as<int32_t>(); // read as uint16 by the float32 entries
        T.tcol = t_tcol.as<int32_t>();
        T.pptr = t_pptr.as<int32_t>();
        T.rptr = t_rptr.as<int32_t>();
        T.rlist = t_rlist.as<int32_t>();
        T.ntiles = t_ntiles;
        T.max_rows = t_max_rows;
        return T;
    }
    std::atomic<int> refs{1};
    size_t bytes = 0; // device bytes of every buffer above (device_bytes() after creation)
    size_t device_bytes() const
    {
        size_t t = 0;
        for (const DevLayout *L : {&csr, &csc, &tiles})
            for (const DBuf *b : {&L->ptr, &L->idx, &L->val32, &L->val16, &L->packed, &L->rowblk, &L->idx16})
                t += b->bytes;
        for (const DBuf *b : {&panel_ptr, &panel_idx16, &panel_packed, &q32, &q16, &zcol, &t_tcol, &t_pptr, &t_rptr,
                              &t_rlist, &t_idx16})
            t += b->bytes;
        return t;
    }
    int lp_kind() const { return storage == SMX_STORE_BF16 ? VK_BF16 : (storage == SMX_STORE_F16 ? VK_F16 : VK_F32); }
};

struct smx_problem {
    smx_operator *op = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;
    int B = 1;
    int64_t m = 0, n = 0;
    float lambda = 1.f;
    int refine_iters = -1;
    PertParams pp{};
    DBuf x, g, c, lower, upper, box_lo, box_hi, lin_c, w, D32, D16, st, qout;
    DBuf part_pass, part_query, part_phase, part_trial[2]; // per-workgroup partial sums of each kernel kind
    int cur = 0; // which of the two state buffers (st holds 2*B states) is current
    bool tuned = false;
    SliceState *state(int which) const { return st.as<SliceState>() + size_t(which) * B; }
    DBuf h_prox, h_fs, h_fe, h_tr, h_ac;
    Hist hist{};
    int hist_cap = 0;
    PassCfg cfg1[3]{}, cfg2[3]{};
    int fmt1[3] = {0, 1, 2}, fmt2[3] = {0, 1, 2}; // stored format each pass reads, per value kind
    // fused single pass (one slice, y in LDS): usable, and in use, per value kind
    bool fused_ok[3] = {false, false, false}, fused[3] = {false, false, false};
    int fused_mode = 1; // 0: always the two passes
    int phase_form = SMX_PHASE_AUTO; // one launch per perturbation phase where eligible, or one per trial batch
    FusedCfg fcfg[3]{};
    DBuf ypart; // grid x n partial vectors of y = A^T c
    DBuf part_lin; // the linear objective's direction partials written by the fused pass's apply kernel
    // basic algorithm (SMX_BASIC_*) and what its step needs beyond D
    int basic = SMX_BASIC_SIMULT;
    DBuf S32, S16; // step weights when they differ from D (CQ: 1/||A||_F^2, EMR: w)
    DBuf ybuf;     // EL / EMR: y = A^T c kept for the extrapolated step, float64 [n*B]
    DBuf ybuf32;   // EMR: y rounded to float32, the vector its second product gathers [n*B]
    DBuf part_y, part_q; // EL / EMR: partials of ||y||^2 and of sum w (A y)^2
    int lds_grid = 0; // one slice: workgroups of the LDS-staged pass 1 (one per CU), 0 when unavailable
    int lds_x = 0;    // entries of the gathered vector it holds in LDS (pass 1: x)
    int lds_c = 0;    // the same for pass 2 (c)
    DBuf ypanel;      // per-panel column sums of the panel pass 2 (np x n)
    PanelView panels() const
    {
        PanelView v;
        v.pp = op->panel_ptr.as<int32_t>();
        v.np = op->panel_np;
        v.P = op->panel_P;
        v.m = m;
        v.ypanel = ypanel.as<double>();
        return v;
    }
    bool tiles_ok = false; // pass 2 may use the operator's image-tile layout (a tile's rows x B fit in LDS)
    bool stop_var = false; // the variance stopping rule: x at each iteration's start, norms after it
    DBuf xprev, part_var;
    // dose-volume constraints: their rows' values, keys, per-constraint
    // histograms and selection state, and the band kernel's partials
    DvcTable dvc{};
    DBuf dvc_dose, dvc_key, dvc_hist, dvc_sel, dvc_part;
    RowW row_weights(int vk) const
    {
        const float *D = (vk == VK_F32) ? D32.as<float>() : D16.as<float>();
        const float *S = (vk == VK_F32) ? S32.as<float>() : S16.as<float>();
        RowW r{D, S ? S : D, 0, nullptr, 0, 0};
        if (dvc.n > 0) {
            r.dose = dvc_dose.as<double>();
            r.dose_lo = dvc.lo;
            r.dose_hi = dvc.lo + dvc.span;
        }
        return r;
    }
    // the dose-volume kernels after pass 1 (partials: pass 1's, nparts1 per slice)
    void enqueue_dvc(int vk, double *partials, int nparts1, int which, int query, hipStream_t s)
    {
        const RowW rw = row_weights(vk);
        hip_check(launch_dvc(dvc, dvc_dose.as<double>(), dvc_key.as<unsigned long long>(), dvc_hist.as<unsigned>(),
                             dvc_sel.as<DvcSel>(), rw.D, rw.S, c.as<float>(), dvc_part.as<double>(), partials,
                             nparts1, state(which), B, query, s),
                  "dose-volume constraints");
    }
    ColStep col_step(bool defer) const
    {
        return ColStep{box_lo.as<float>(), box_hi.as<float>(), lambda,
                       basic == SMX_BASIC_DROP ? op->zcol.as<float>() : nullptr,
                       defer ? ybuf.as<double>() : nullptr, defer ? ybuf32.as<float>() : nullptr,
                       defer ? part_y.as<double>() : nullptr, defer ? 1 : 0};
    }
    // captured graphs keyed by (value kind, perturb, iterations)
    std::map<long long, hipGraphExec_t> graphs;
    hipStream_t capture_stream = nullptr; // private stream graphs are captured on
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double t1_ms = 0, t2_ms = 0;
    int64_t t_launches = 0;
    // device bytes of every buffer the problem owns (the plan of problem_plan_bytes)
    size_t device_bytes() const
    {
        size_t t = 0;
        for (const DBuf *b : {&x, &g, &c, &lower, &upper, &box_lo, &box_hi, &lin_c, &w, &D32, &D16, &st, &qout,
                              &part_pass, &part_query, &part_phase, &part_trial[0], &part_trial[1], &h_prox, &h_fs,
                              &h_fe, &h_tr, &h_ac, &ypart, &part_lin, &S32, &S16, &ybuf, &ybuf32, &part_y, &part_q,
                              &ypanel,
                              &xprev, &part_var, &dvc_dose, &dvc_key, &dvc_hist, &dvc_sel, &dvc_part})
            t += b->bytes;
        return t;
    }
    ~smx_problem()
    {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
    }
};

namespace {

// Default launch shape of a pass: row blocks streamed through LDS for one
// slice; several slices use the multi-slice lanes-per-row kernels.
PassCfg pick_cfg(const DevLayout &L, int vk, int B = 1)
{
    PassCfg c;
    c.vec = (vk == VK_F32) ? 4 : 8;
    if (B > 1) {
        c.mode = 0;
        c.lpr = 8;
        const int64_t rpb = kBlock / c.lpr;
        c.grid = (int)std::max<int64_t>(1, std::min<int64_t>((L.rows + rpb - 1) / rpb, kMaxPassGrid));
        return c;
    }
    c.mode = 1;
    c.lpr = 64;
    c.grid = std::max(1, std::min(L.nblk, kMaxPassGrid));
    return c;
}

// The lanes-per-row shape (mode 0) for the same layout.
PassCfg pick_cfg_rows(const DevLayout &L, int vk)
{
    PassCfg c;
    c.mode = 0;
    c.vec = (vk == VK_F32) ? 4 : 8;
    const double mean = L.rows > 0 ? double(L.slots) / double(L.rows) : 0.0;
    int lpr = 2;
    while (lpr < 64 && lpr * c.vec * 8 < mean) lpr *= 2;
    c.lpr = lpr;
    const int64_t rpb = kBlock / lpr;
    int64_t grid = (L.rows + rpb - 1) / rpb;
    c.grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, kMaxPassGrid));
    return c;
}

SpView view_for(const smx_operator *op, bool transposed, int vk)
{
    return transposed ? op->csc.view(vk) : op->csr.view(vk);
}

// Format the fused pass reads for value kind vk (the same copy as pass 1).
int fused_fmt(const smx_problem *p, int vk);

int validate_csr_host(const smx_csr *A, const int32_t *rp, const int32_t *ci, const float *v)
{
    if (rp[0] != 0) return fail(SMX_EINVAL, "row_ptr[0] must be 0 (got %d)", rp[0]);
    for (int64_t i = 0; i < A->m; ++i)
        if (rp[i + 1] < rp[i]) return fail(SMX_EINVAL, "row_ptr decreases at row %lld", (long long)i);
    if ((int64_t)rp[A->m] != A->nnz)
        return fail(SMX_EINVAL, "row_ptr[m] = %d differs from nnz = %lld", rp[A->m], (long long)A->nnz);
    for (int64_t p = 0; p < A->nnz; ++p) {
        if (ci[p] < 0 || ci[p] >= A->n)
            return fail(SMX_EINVAL, "column index %d at entry %lld outside [0, %lld)", ci[p], (long long)p,
                        (long long)A->n);
        if (!std::isfinite(v[p])) return fail(SMX_EINVAL, "non-finite value at entry %lld", (long long)p);
    }
    return SMX_OK;
}

template <typename T>
std::vector<T> fetch(const T *p, int64_t count, bool on_device)
{
    std::vector<T> h(count);
    if (count == 0) return h;
    if (on_device) hip_check(hipMemcpy(h.data(), p, sizeof(T) * count, hipMemcpyDeviceToHost), "copy input to host");
    else std::memcpy(h.data(), p, sizeof(T) * count);
    return h;
}

template <typename T>
void upload(DBuf &b, const std::vector<T> &h, hipStream_t s, const char *what)
{
    b.alloc(sizeof(T) * std::max<size_t>(h.size(), 1), what);
    if (!h.empty()) hip_check(hipMemcpyAsync(b.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s), what);
    hip_check(hipStreamSynchronize(s), what);
}

void upload_layout(DevLayout &D, HostLayout &H, int64_t rows, int64_t index_range, bool keep32, int lp, hipStream_t s)
{
    D.rows = rows;
    D.slots = H.slots;
    {
        std::vector<int32_t> rb = build_row_blocks(H.ptr, rows);
        D.nblk = (int)rb.size() - 1;
        upload(D.rowblk, rb, s, "upload row blocks");
    }
    upload(D.ptr, H.ptr, s, "upload row pointers");
    upload(D.idx, H.idx, s, "upload indices");
    upload(D.val32, H.val, s, "upload values");
    if (keep32 && index_range <= 65536) { // float32 values with 16-bit indices: 6 bytes per entry
        std::vector<uint16_t> i16(H.idx.size());
        for (size_t p = 0; p < H.idx.size(); ++p) i16[p] = (uint16_t)H.idx[p];
        upload(D.idx16, i16, s, "upload 16-bit indices");
    }
    if (lp != VK_F32) {
        D.val16.alloc(sizeof(uint16_t) * std::max<int64_t>(H.slots, 1), "allocate reduced-precision values");
        if (lp == VK_BF16) hip_check(launch_to_bf16(D.val32.as<float>(), D.val16.as<uint16_t>(), H.slots, s), "to bf16");
        else {
            D.f16_scale = f16_scale_for(H.val);
            hip_check(launch_to_f16(D.val32.as<float>(), D.val16.as<uint16_t>(), H.slots, D.f16_scale, s), "to f16");
        }
        const bool pack = index_range <= 65536; // one 32-bit word per entry: value and index
        if (pack) {
            D.packed.alloc(sizeof(uint32_t) * std::max<int64_t>(H.slots, 1), "allocate packed entries");
            hip_check(launch_pack16(D.val16.as<uint16_t>(), D.idx.as<int32_t>(), D.packed.as<uint32_t>(), H.slots, s),
                      "pack entries");
        }
        hip_check(hipStreamSynchronize(s), "convert values");
        if (!keep32) D.val32.release();
        if (pack) { // the packed words replace the separate reduced-precision values
            D.val16.release();
            if (!keep32) D.idx.release();
        }
    }
    // release host copies early
    std::vector<int32_t>().swap(H.ptr);
    std::vector<int32_t>().swap(H.idx);
    std::vector<float>().swap(H.val);
}

// Host form of the image-tile column layout (TileView).
struct TileHost {
    std::vector<int32_t> tcol, pptr, rptr, rlist, ptr, idx;
    std::vector<float> val;
    int max_rows = 0;
};

constexpr int kTileMaxRows = 16384; // rows of one tile: 64 KB of LDS, 16-bit positions

// Groups the columns of A^T (cp/ri/cv: its unpadded CSR, rows ascending in
// each column) by th x tw tiles of an R x C image (unknown i*C + j is pixel
// (i, j)).  Each tile column's entries keep their order; their indices become
// positions in the tile's ascending row list; columns are padded to
// kRowAlign entries (value 0, the last position).  Returns false when a tile
// touches more than kTileMaxRows rows or the layout reaches 2^31 entries.
bool build_tiles(int64_t R, int64_t C, int th, int tw, const std::vector<int64_t> &cp, const std::vector<int32_t> &ri,
                 const std::vector<float> &cv, TileHost &T)
{
    const int64_t ntr = (R + th - 1) / th, ntc = (C + tw - 1) / tw;
    T.pptr.assign(1, 0);
    T.rptr.assign(1, 0);
    T.ptr.assign(1, 0);
    std::vector<int32_t> rows;
    for (int64_t ti = 0; ti < ntr; ++ti)
        for (int64_t tj = 0; tj < ntc; ++tj) {
            rows.clear();
            const size_t c0 = T.tcol.size();
            for (int64_t i = ti * th; i < std::min(R, ti * th + th); ++i)
                for (int64_t j = tj * tw; j < std::min(C, tj * tw + tw); ++j) {
                    const int64_t col = i * C + j;
                    T.tcol.push_back((int32_t)col);
                    rows.insert(rows.end(), ri.begin() + cp[col], ri.begin() + cp[col + 1]);
                }
            std::sort(rows.begin(), rows.end());
            rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
            if ((int64_t)rows.size() > kTileMaxRows) return false;
            T.max_rows = std::max(T.max_rows, (int)rows.size());
            T.rlist.insert(T.rlist.end(), rows.begin(), rows.end());
            T.rptr.push_back((int32_t)T.rlist.size());
            for (size_t q = c0; q < T.tcol.size(); ++q) {
                const int64_t col = T.tcol[q];
                int32_t last = 0;
                for (int64_t p = cp[col]; p < cp[col + 1]; ++p) {
                    last = (int32_t)(std::lower_bound(rows.begin(), rows.end(), ri[p]) - rows.begin());
                    T.idx.push_back(last);
                    T.val.push_back(cv[p]);
                }
                while (T.val.size() % kRowAlign) {
                    T.idx.push_back(last);
                    T.val.push_back(0.f);
                }
                if (T.val.size() >= (size_t(1) << 31)) return false;
                T.ptr.push_back((int32_t)T.val.size());
            }
            T.pptr.push_back((int32_t)T.tcol.size());
        }
    return true;
}

// Uploads the tile layout; the reduced-precision copy is always packed (the
// positions fit in 16 bits).
void upload_tiles(smx_operator *op, TileHost &T, int lp, hipStream_t s)
{
    DevLayout &D = op->tiles;
    D.rows = op->n;
    D.slots = (int64_t)T.val.size();
    upload(D.ptr, T.ptr, s, "upload tile pointers");
    upload(op->t_tcol, T.tcol, s, "upload tile columns");
    upload(op->t_pptr, T.pptr, s, "upload tile columns");
    upload(op->t_rptr, T.rptr, s, "upload tile rows");
    upload(op->t_rlist, T.rlist, s, "upload tile rows");
    op->t_ntiles = (int)T.pptr.size() - 1;
    op->t_max_rows = T.max_rows;
    upload(D.val32, T.val, s, "upload tile values");
    if (op->has_f32) {
        std::vector<uint16_t> i16(T.idx.size());
        for (size_t p = 0; p < T.idx.size(); ++p) i16[p] = (uint16_t)T.idx[p];
        upload(op->t_idx16, i16, s, "upload tile positions");
    }
    if (lp != VK_F32) {
        upload(D.idx, T.idx, s, "upload tile positions");
        DBuf v16;
        v16.alloc(sizeof(uint16_t) * std::max<int64_t>(D.slots, 1), "tile reduced-precision values");
        if (lp == VK_BF16) hip_check(launch_to_bf16(D.val32.as<float>(), v16.as<uint16_t>(), D.slots, s), "to bf16");
        else {
            D.f16_scale = op->csc.f16_scale;
            hip_check(launch_to_f16(D.val32.as<float>(), v16.as<uint16_t>(), D.slots, D.f16_scale, s), "to f16");
        }
        D.packed.alloc(sizeof(uint32_t) * std::max<int64_t>(D.slots, 1), "tile packed entries");
        hip_check(launch_pack16(v16.as<uint16_t>(), D.idx.as<int32_t>(), D.packed.as<uint32_t>(), D.slots, s),
                  "pack tile entries");
        hip_check(hipStreamSynchronize(s), "pack tile entries");
        D.idx.release();
        if (!op->has_f32) D.val32.release();
    }
}

// Upper bound on the device bytes of an operator with m rows, n columns and
// nnz entries (lp: a reduced-precision copy, f32: the float32 values kept;
// image_rows x image_cols > 0: an image operator with the tile layout): every
// row and column padded by kRowAlign - 1 entries, row blocks at one per row,
// tiles as small as the smallest tile edge, and each tile's row list as long
// as its entries.
size_t operator_bound(int64_t m, int64_t n, int64_t nnz, bool lp, bool f32, int64_t image_rows, int64_t image_cols)
{
    const int64_t s1 = nnz + (kRowAlign - 1) * m, s2 = nnz + (kRowAlign - 1) * n;
    size_t b = layout_bytes(m, s1, f32, lp, lp && n <= 65536, n <= 65536) +
               layout_bytes(n, s2, f32, lp, lp && m <= 65536, m <= 65536) +
               size_t(m + 2) * 4 + size_t(n + 2) * 4 +              // row blocks of both layouts
               size_t(m) * 8 * ((f32 ? 1 : 0) + (lp ? 1 : 0)) + // row norms
               size_t(n) * 4;                                    // DROP column factors
    if (m > kLdsPassFloats) { // row panels of the column copy: offsets (and 16-bit rows, packed entries)
        const int64_t np = (m + kLdsPassFloats - 1) / kLdsPassFloats;
        b += size_t(np + 1) * size_t(n) * 4 + (m > 65536 ? size_t(s2) * (2 + (lp ? 4 : 0)) : 0);
    }
    if (image_rows > 0 && image_cols > 0) { // tile layout (tiles of edge 4 at the least)
        const int64_t T = ((image_rows + 3) / 4) * ((image_cols + 3) / 4);
        b += size_t(n + 1) * 4 + size_t(n) * 4 + 2 * size_t(T + 1) * 4 + size_t(nnz) * 4 +
             size_t(s2) * ((f32 ? 6 : 0) + (lp ? 4 : 0));
    }
    return b;
}

int create_operator(const smx_csr *A, int32_t storage, int32_t keep_f32, hipStream_t s, smx_operator **out,
                    int32_t img_rows = 0, int32_t img_cols = 0)
{
    if (!A || !out) return fail(SMX_EINVAL, "NULL argument");
    *out = nullptr;
    if (A->m < 1 || A->n < 1) return fail(SMX_EINVAL, "m and n must be >= 1 (got %lld, %lld)", (long long)A->m, (long long)A->n);
    if (A->m >= (int64_t(1) << 31) || A->n >= (int64_t(1) << 31) || A->nnz < 0 || A->nnz >= (int64_t(1) << 31))
        return fail(SMX_EINVAL, "dimensions exceed 2^31-1");
    if (storage < SMX_STORE_F32 || storage > SMX_STORE_F16) return fail(SMX_EINVAL, "unknown value storage %d", storage);
    if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val))) return fail(SMX_EINVAL, "NULL CSR array");
    if (A->nnz == 0) return fail(SMX_EINVAL, "the operator has no nonzeros");
    std::unique_ptr<smx_operator> op(new smx_operator());
    op->m = A->m;
    op->n = A->n;
    op->nnz = A->nnz;
    op->storage = storage;
    op->has_f32 = (storage == SMX_STORE_F32) || keep_f32;
    std::vector<int32_t> rp = fetch(A->row_ptr, A->m + 1, A->on_device);
    std::vector<int32_t> ci = fetch(A->col_idx, A->nnz, A->on_device);
    std::vector<float> va = fetch(A->val, A->nnz, A->on_device);
    int rc = validate_csr_host(A, rp.data(), ci.data(), va.data());
    if (rc != SMX_OK) return rc;
    hip_check(hipGetDevice(&op->device), "get device");
    const int64_t m = A->m, n = A->n, nnz = A->nnz;
    std::vector<int64_t> rp64(rp.begin(), rp.end());
    // transpose by a stable counting sort: rows stay in order inside each column
    std::vector<int64_t> cp(n + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) cp[ci[p] + 1]++;
    for (int64_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
    std::vector<int32_t> ri(nnz);
    std::vector<float> cv(nnz);
    {
        // DROP column factors count the nonzero values as given (before any rounding)
        std::vector<float> zc(n, 0.f);
        std::vector<int64_t> cnt(n, 0);
        for (int64_t p = 0; p < nnz; ++p)
            if (va[p] != 0.f) cnt[ci[p]]++;
        for (int64_t j = 0; j < n; ++j) zc[j] = cnt[j] > 0 ? (float)(1.0 / (double)cnt[j]) : 0.f;
        upload(op->zcol, zc, s, "column factors");
    }
    {
        std::vector<int64_t> pos(cp.begin(), cp.end() - 1);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t p = rp64[i]; p < rp64[i + 1]; ++p) {
                const int64_t q = pos[ci[p]]++;
                ri[q] = (int32_t)i;
                cv[q] = va[p];
            }
    }
    const int lp = op->lp_kind();
    TileHost TH;
    bool tiled = false;
    if (img_rows > 0) {
        const char *te = getenv("SMX_TILE"); // tile edge (4, 8 or 16); default 8
        const int edge = te ? std::max(4, std::min(16, atoi(te))) : 8;
        tiled = build_tiles(img_rows, img_cols, edge, edge, cp, ri, cv, TH);
        op->img_rows = img_rows;
        op->img_cols = img_cols;
    }
    {
        HostLayout H;
        if (!pad_rows(m, rp64.data(), ci.data(), va.data(), H)) return fail(SMX_EINVAL, "padded CSR exceeds 2^31 entries");
        std::vector<int32_t>().swap(ci);
        std::vector<float>().swap(va);
        upload_layout(op->csr, H, m, n, op->has_f32, lp, s);
    }
    {
        HostLayout H;
        if (!pad_rows(n, cp.data(), ri.data(), cv.data(), H)) return fail(SMX_EINVAL, "padded CSC exceeds 2^31 entries");
        if (m > kLdsPassFloats) { // row panels of kLdsPassFloats rows for the panel pass 2
            const int P = kLdsPassFloats;
            const int np = (int)((m + P - 1) / P);
            std::vector<int32_t> pp(size_t(np + 1) * n);
            for (int64_t j = 0; j < n; ++j) {
                int64_t k = cp[j];
                for (int p = 0; p <= np; ++p) {
                    const int64_t lim = (p == np) ? m : int64_t(p) * P;
                    while (k < cp[j + 1] && ri[k] < lim) ++k;
                    pp[size_t(p) * n + j] = (int32_t)(H.ptr[j] + (k - cp[j]));
                }
            }
            upload(op->panel_ptr, pp, s, "upload row panels");
            if (m > 65536) { // rows need 32 bits in the column copy: a copy with 16-bit offsets within the panel
                std::vector<uint16_t> lidx(size_t(H.slots), 0); // padding keeps offset 0
                for (int64_t j = 0; j < n; ++j)
                    for (int p = 0; p < np; ++p)
                        for (int32_t k = pp[size_t(p) * n + j]; k < pp[size_t(p + 1) * n + j]; ++k)
                            lidx[size_t(k)] = (uint16_t)(H.idx[size_t(k)] - p * P);
                upload(op->panel_idx16, lidx, s, "upload panel row offsets");
            }
            op->panel_np = np;
            op->panel_P = P;
        }
        std::vector<int32_t>().swap(ri);
        std::vector<float>().swap(cv);
        upload_layout(op->csc, H, n, m, op->has_f32, lp, s);
        // with 32-bit rows the column copy keeps its separate reduced-precision
        // values (it packs, and then drops them, only when rows fit 16 bits)
        if (op->panel_idx16.p && lp != VK_F32 && op->csc.val16.p) {
            op->panel_packed.alloc(sizeof(uint32_t) * size_t(std::max<int64_t>(op->csc.slots, 1)), "panel entries");
            hip_check(launch_pack16u(op->csc.val16.as<uint16_t>(), op->panel_idx16.as<uint16_t>(),
                                     op->panel_packed.as<uint32_t>(), op->csc.slots, s),
                      "pack panel entries");
            hip_check(hipStreamSynchronize(s), "pack panel entries");
        }
    }
    if (tiled) upload_tiles(op.get(), TH, lp, s);
    if (op->has_f32) {
        op->q32.alloc(sizeof(double) * m, "row norms");
        hip_check(launch_rownorm(op->csr.view(VK_F32), VK_F32, op->q32.as<double>(), s), "row norms");
    }
    if (lp != VK_F32) {
        op->q16.alloc(sizeof(double) * m, "row norms (reduced precision)");
        const int fmt = op->csr.packed.p ? (lp == VK_BF16 ? VK_BF16P : VK_F16P) : lp; // the copy the passes read
        hip_check(launch_rownorm(op->csr.view(fmt), fmt, op->q16.as<double>(), s), "row norms (reduced precision)");
    }
    hip_check(hipStreamSynchronize(s), "operator setup");
    op->bytes = op->device_bytes();
    *out = op.release();
    return SMX_OK;
}

void release_operator(smx_operator *op)
{
    if (op && op->refs.fetch_sub(1) == 1) delete op;
}

int vk_for_iteration(const smx_problem *p, int64_t it, int64_t K, int64_t ref)
{
    const int lp = p->op->lp_kind();
    if (lp == VK_F32) return VK_F32;
    if (!p->op->has_f32) return lp;
    return (it >= K - ref) ? VK_F32 : lp;
}

int fused_fmt(const smx_problem *p, int vk) { return p->fmt1[vk]; }

// Entry format of the row-panel pass 2 for value kind vk: 16-bit panel
// offsets beside float32 values, or packed with the reduced-precision values.
int panel_fmt(const smx_problem *p, int vk)
{
    if (vk == VK_F32) return p->op->panel_idx16.p ? VK_F32U16 : p->fmt2[vk];
    if (p->op->panel_packed.p) return p->op->lp_kind() == VK_BF16 ? VK_BF16P : VK_F16P;
    return p->fmt2[vk];
}

// Pass 2 in launch shape c: the image-tile layout (mode 2) or the column copy.
hipError_t pass2_any(const smx_problem *p, int vk, const PassCfg &c, const float *cres, float *x, ColStep cs,
                     const SliceState *st_in, SliceState *st_out, const double *part1, int nparts1, Hist h,
                     hipStream_t s)
{
    if (c.mode == 5) {
        PanelView pv = p->panels();
        const int fk = panel_fmt(p, vk);
        SpView v = p->op->csc.view(fk); // rows <= 65536: the column copy's own 16-bit (global) rows
        pv.local = 0;
        if (fk == VK_F32U16 && p->op->panel_idx16.p) { // read as uint16 by the kernels
            v.idx = p->op->panel_idx16.as<int32_t>();
            pv.local = 1;
        } else if ((fk == VK_BF16P || fk == VK_F16P) && p->op->panel_packed.p) {
            v.val = p->op->panel_packed.p;
            pv.local = 1;
        }
        return launch_pass2_panels(c, v, pv, fk, cres, x, cs, st_in, st_out, part1, nparts1, h, s);
    }
    if (c.mode == 2) {
        const int lp = p->op->lp_kind();
        const int tk = vk == VK_F32 ? VK_F32 : (lp == VK_BF16 ? VK_BF16P : VK_F16P);
        return launch_pass2_tiles(c, p->op->tile_view(tk), tk, cres, x, cs, st_in, st_out, p->B, part1, nparts1, h,
                                  s);
    }
    return launch_pass2(c, view_for(p->op, true, p->fmt2[vk]), p->op->csc.blocks(), p->fmt2[vk], cres, x, cs, st_in,
                        st_out, p->B, part1, nparts1, h, s);
}

// The extrapolated steps after y is kept: EMR's quadratic form sum_i w_i
// (A y)_i^2 (pass 1's kernels gathering y), then k_step_apply, which closes
// the iteration into the other state buffer.  nparts1: partials of pass 1 (or
// the fused pass), nparts_y: partials of ||y||^2.
void enqueue_extrapolated_step(smx_problem *p, int vk, const RowW &rw, int nparts1, int nparts_y, int cur,
                               hipStream_t s)
{
    const bool emr = p->basic == SMX_BASIC_EMR;
    if (emr)
        hip_check(launch_pass1(p->cfg1[vk], view_for(p->op, false, p->fmt1[vk]), p->op->csr.blocks(), p->fmt1[vk],
                               p->ybuf32.as<float>(), p->lower.as<float>(), p->upper.as<float>(), RowW{rw.D, rw.S, 1},
                               p->c.as<float>(), p->state(cur), p->B, 0, p->part_q.as<double>(), s),
                  "quadratic form");
    hip_check(launch_step_apply(p->n, p->B, p->ybuf.as<double>(), p->x.as<float>(), p->box_lo.as<float>(),
                                p->box_hi.as<float>(), p->lambda, emr ? 1 : 0, p->part_pass.as<double>(), nparts1,
                                p->part_y.as<double>(), nparts_y, p->part_q.as<double>(), p->cfg1[vk].grid,
                                p->state(cur), p->state(cur ^ 1), p->hist, s),
              "extrapolated step");
}

enum PhaseKind { PHASE_CHAIN, PHASE_SMALL, PHASE_LINEAR };

// How the problem's perturbation phase runs: as asked, or by default in one
// launch for flat objectives on vectors up to kSmallPhaseAutoN (one
// workgroup streams x at one CU's rate, about 15 GB/s from memory, so its
// time grows with n: ~6 us at n = 324, ~28 us at n = 19,881, where the
// launch chain takes ~22-25 us whatever n), the linear objective beyond that
// with its trials in closed form, anything else as the chain of launches.
PhaseKind phase_kind(const smx_problem *p)
{
    switch (p->phase_form) {
    case SMX_PHASE_BATCHES: return PHASE_CHAIN;
    case SMX_PHASE_ONE_LAUNCH: return PHASE_SMALL;   // eligibility checked when set
    case SMX_PHASE_CLOSED_FORM: return PHASE_LINEAR; // likewise
    default:
        if (phase_in_one_launch(p->pp) && p->n <= kSmallPhaseAutoN) return PHASE_SMALL;
        return p->pp.obj == OBJ_LINEAR ? PHASE_LINEAR : PHASE_CHAIN;
    }
}

// Trial launches of the chain: each reduction step needs at most two (a short
// batch, then every remaining trial up to the cap).
int chain_trial_launches(const smx_problem *p)
{
    return (p->pp.max_trials > p->pp.first_width ? 2 : 1) * p->pp.n_red;
}

// State-buffer flips of one perturbation phase: one per launch that moves
// the state (the chain's trial launches and its closing launch).
int phase_flips(const smx_problem *p)
{
    return phase_kind(p) == PHASE_CHAIN ? chain_trial_launches(p) + 1 : 1;
}

// Whether iterations of value kind vk take the linear objective's direction
// partials from the previous iteration's apply kernel (fused pass, the step
// applied there), so that the phase is the one closed-form launch.
bool lin_from_apply(const smx_problem *p, int vk)
{
    const bool extrap = p->basic == SMX_BASIC_EL || p->basic == SMX_BASIC_EMR;
    return phase_kind(p) == PHASE_LINEAR && p->fused[vk] && !extrap && p->part_lin.p;
}

// Whether iterations of value kind vk take that phase inside the fused pass
// (shapes with z in LDS): every workgroup of the pass opens the phase from the
// partials and stages z = x + s v, and the apply kernel forms z_j again, so
// the phase costs no launch of its own.
bool lin_in_pass(const smx_problem *p, int vk) { return lin_from_apply(p, vk) && p->fcfg[vk].zl; }

// Launches of one perturbation phase (of the first value kind that runs).
int phase_launch_count(const smx_problem *p)
{
    switch (phase_kind(p)) {
    case PHASE_SMALL: return 1;
    case PHASE_LINEAR:
        for (int vk = 0; vk < 3; ++vk) {
            if (lin_in_pass(p, vk)) return 0;
            if (lin_from_apply(p, vk)) return 1;
        }
        return 2;
    default: return chain_trial_launches(p) + 2;
    }
}

// Enqueue one outer iteration with value kind vk on stream s, starting from
// state buffer `cur`; returns the buffer current after it.
int enqueue_iteration_core(smx_problem *p, hipStream_t s, int vk, bool perturb, bool timed, int cur)
{
    const float *gvec = (p->pp.obj == OBJ_LINEAR) ? p->lin_c.as<float>() : p->g.as<float>();
    const PhaseKind pk = phase_kind(p);
    if (perturb && p->pp.obj != OBJ_NONE && pk == PHASE_SMALL) {
        hip_check(launch_phase_small(p->pp, p->x.as<float>(), p->lin_c.as<float>(), p->state(cur), p->state(cur ^ 1),
                                     s),
                  "phase");
        cur ^= 1;
    } else if (perturb && p->pp.obj != OBJ_NONE && pk == PHASE_LINEAR && lin_in_pass(p, vk)) {
        // taken inside the fused pass below
    } else if (perturb && p->pp.obj != OBJ_NONE && pk == PHASE_LINEAR) {
        if (lin_from_apply(p, vk)) { // the partials of x^k came from the last apply (or the run's start)
            hip_check(launch_trial_linear(p->pp, p->x.as<float>(), p->lin_c.as<float>(), p->state(cur),
                                          p->state(cur ^ 1), p->part_lin.as<double>(), s,
                                          fused_apply_grid(p->n)),
                      "linear phase");
        } else {
            hip_check(launch_phase(p->pp, p->x.as<float>(), p->g.as<float>(), p->lin_c.as<float>(), p->state(cur), 0,
                                   p->part_phase.as<double>(), s),
                      "phase");
            hip_check(launch_trial_linear(p->pp, p->x.as<float>(), p->lin_c.as<float>(), p->state(cur),
                                          p->state(cur ^ 1), p->part_phase.as<double>(), s),
                      "linear phase");
        }
        cur ^= 1;
    } else if (perturb && p->pp.obj != OBJ_NONE) {
        hip_check(launch_phase(p->pp, p->x.as<float>(), p->g.as<float>(), p->lin_c.as<float>(), p->state(cur), 0,
                               p->part_phase.as<double>(), s),
                  "phase");
        const int launches = chain_trial_launches(p);
        const double *prev = p->part_phase.as<double>();
        for (int t = 0; t < launches; ++t) {
            double *out = p->part_trial[t & 1].as<double>();
            hip_check(launch_trial(p->pp, p->x.as<float>(), gvec, p->state(cur), p->state(cur ^ 1), t == 0 ? 1 : 0,
                                   1, prev, out, s),
                      "trial");
            cur ^= 1;
            prev = out;
        }
        hip_check(launch_trial_close(p->pp, p->x.as<float>(), gvec, p->state(cur), p->state(cur ^ 1), prev, s),
                  "close phase");
        cur ^= 1;
    }
    const RowW rw = p->row_weights(vk);
    hipEvent_t e[4] = {};
    if (timed) {
        while (p->ev_pool.size() < p->ev_used + 4) {
            hipEvent_t ev;
            hip_check(hipEventCreate(&ev), "event");
            p->ev_pool.push_back(ev);
        }
        for (int i = 0; i < 4; ++i) e[i] = p->ev_pool[p->ev_used + i];
        p->ev_used += 4;
        hip_check(hipEventRecord(e[0], s), "event");
    }
    const bool extrap = p->basic == SMX_BASIC_EL || p->basic == SMX_BASIC_EMR;
    if (p->fused[vk]) {
        const bool lin_pass = perturb && p->pp.obj != OBJ_NONE && pk == PHASE_LINEAR && lin_in_pass(p, vk);
        LinPhase lp{};
        if (lin_pass) {
            lp.c = p->lin_c.as<float>();
            lp.part = p->part_lin.as<double>();
            lp.nparts = fused_apply_grid(p->n);
            lp.st_out = p->state(cur ^ 1);
            lp.pp = p->pp;
        }
        hip_check(launch_fused(p->fcfg[vk], view_for(p->op, false, fused_fmt(p, vk)), fused_fmt(p, vk), p->n, p->x.as<float>(),
                               p->lower.as<float>(), p->upper.as<float>(), rw, p->state(cur),
                               p->part_pass.as<double>(), p->ypart.p, s, lin_pass ? &lp : nullptr),
                  "fused pass");
        if (lin_pass) cur ^= 1; // the phase's state
        if (timed) hip_check(hipEventRecord(e[1], s), "event");
        int nvec = p->fcfg[vk].grid;
        if (p->dvc.n > 0) { // rank the dose-volume rows, then add their c_i a_i as a second set of partials
            p->enqueue_dvc(vk, p->part_pass.as<double>(), p->fcfg[vk].grid, cur, 0, s);
            hip_check(launch_scatter_rows(view_for(p->op, false, fused_fmt(p, vk)), fused_fmt(p, vk), p->n, p->dvc.lo,
                                          p->dvc.lo + p->dvc.span, p->c.as<float>(), p->state(cur),
                                          p->ypart.as<float>() + size_t(nvec) * size_t(p->n), nvec, s),
                      "dose-volume rows");
            nvec *= 2;
        }
        if (timed) hip_check(hipEventRecord(e[2], s), "event");
        const bool lin = lin_from_apply(p, vk);
        hip_check(launch_fused_apply(p->fcfg[vk], p->n, p->ypart.p, nvec, p->x.as<float>(), p->col_step(extrap),
                                     p->state(cur), p->state(cur ^ 1), p->part_pass.as<double>(), p->hist, s,
                                     lin ? p->lin_c.as<float>() : nullptr, lin ? p->part_lin.as<double>() : nullptr,
                                     lin_pass ? 1 : 0),
                  "fused apply");
        if (timed) hip_check(hipEventRecord(e[3], s), "event");
        if (extrap) enqueue_extrapolated_step(p, vk, rw, p->fcfg[vk].grid, fused_apply_grid(p->n), cur, s);
        cur ^= 1;
        return cur;
    }
    hip_check(launch_pass1(p->cfg1[vk], view_for(p->op, false, p->fmt1[vk]), p->op->csr.blocks(), p->fmt1[vk],
                           p->x.as<float>(), p->lower.as<float>(), p->upper.as<float>(), rw, p->c.as<float>(),
                           p->state(cur), p->B, 0,
                           p->part_pass.as<double>(), s),
              "pass 1");
    if (timed) hip_check(hipEventRecord(e[1], s), "event");
    if (p->dvc.n > 0) p->enqueue_dvc(vk, p->part_pass.as<double>(), p->cfg1[vk].grid, cur, 0, s);
    if (timed) hip_check(hipEventRecord(e[2], s), "event");
    hip_check(pass2_any(p, vk, p->cfg2[vk], p->c.as<float>(), p->x.as<float>(), p->col_step(extrap), p->state(cur),
                        p->state(cur ^ 1), p->part_pass.as<double>(), p->cfg1[vk].grid, p->hist, s),
              "pass 2");
    if (timed) hip_check(hipEventRecord(e[3], s), "event");
    if (extrap) enqueue_extrapolated_step(p, vk, rw, p->cfg1[vk].grid, p->cfg2[vk].grid, cur, s);
    cur ^= 1;
    return cur;
}

// One outer iteration; with the variance stopping rule, x is kept at the
// iteration's start and the rule is applied after it.
int enqueue_iteration(smx_problem *p, hipStream_t s, int vk, bool perturb, bool timed, int cur)
{
    if (p->stop_var) hip_check(launch_copy(p->xprev.as<float>(), p->x.as<float>(), p->n * p->B, s), "keep iterate");
    cur = enqueue_iteration_core(p, s, vk, perturb, timed, cur);
    if (p->stop_var) {
        int np = 0;
        hip_check(launch_iter_norms(p->x.as<float>(), p->xprev.as<float>(), p->n, p->B, p->part_var.as<double>(), &np,
                                    s),
                  "iterate change");
        hip_check(launch_stop_var(p->state(cur), p->B, p->part_var.as<double>(), np, s), "variance rule");
    }
    return cur;
}

// Graph of `iters` iterations starting from state buffer `cur`; *cur_after
// receives the buffer current after it.
hipGraphExec_t graph_for(smx_problem *p, int vk, bool perturb, int iters, int cur, int *cur_after)
{
    const long long key = ((long long)vk << 40) | ((long long)(perturb ? 1 : 0) << 33) | ((long long)cur << 32) |
                          (long long)iters;
    // the buffer parity after the chunk does not depend on the data
    int after = cur;
    {
        const bool pert = perturb && p->pp.obj != OBJ_NONE;
        const int flips = (pert ? phase_flips(p) : 0) + 1;
        if ((flips * iters) & 1) after ^= 1;
    }
    *cur_after = after;
    auto it = p->graphs.find(key);
    if (it != p->graphs.end()) return it->second;
    hipGraph_t g = nullptr;
    if (!p->capture_stream) hip_check(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking), "capture stream");
    hip_check(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
        int c = cur;
        for (int i = 0; i < iters; ++i) c = enqueue_iteration(p, p->capture_stream, vk, perturb, false, c);
        if (c != after) throw HipError{hipErrorUnknown, "state buffer parity"};
    } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(p->capture_stream, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        throw;
    }
    hip_check(hipStreamEndCapture(p->capture_stream, &g), "end capture");
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "instantiate graph");
    p->graphs[key] = ex;
    return ex;
}

constexpr int kGraphChunk = 10;

int run_impl(smx_problem *p, int32_t K, uint32_t flags)
{
    if (K < 0) return fail(SMX_EINVAL, "K must be >= 0");
    if (K == 0) return SMX_OK;
    const bool perturb = (flags & SMX_RUN_PERTURB) != 0;
    const bool graph = (flags & SMX_RUN_GRAPH) != 0;
    const int lp = p->op->lp_kind();
    int64_t ref = 0;
    if (lp != VK_F32 && p->op->has_f32) ref = p->refine_iters >= 0 ? p->refine_iters : (K + 19) / 20;
    if (ref > K) ref = K;
    const bool timed = p->timing && !graph;
    if (timed) p->ev_used = 0;
    int64_t it = 0;
    while (it < K) {
        const int vk = vk_for_iteration(p, it, K, ref);
        // run of iterations with the same value kind
        int64_t end = it;
        while (end < K && vk_for_iteration(p, end, K, ref) == vk) ++end;
        int64_t left = end - it;
        // the first phase of the run of iterations needs its direction partials of x
        if (perturb && lin_from_apply(p, vk))
            hip_check(launch_lin_partials(p->x.as<float>(), p->lin_c.as<float>(), p->n, p->part_lin.as<double>(),
                                          p->stream),
                      "direction partials");
        if (graph) {
            while (left > 0) {
                const int chunk = (int)std::min<int64_t>(left, kGraphChunk);
                int after = p->cur;
                hipGraphExec_t ex = graph_for(p, vk, perturb, chunk, p->cur, &after);
                hip_check(hipGraphLaunch(ex, p->stream), "graph launch");
                p->cur = after;
                left -= chunk;
            }
        } else {
            for (int64_t i = 0; i < left; ++i) p->cur = enqueue_iteration(p, p->stream, vk, perturb, timed, p->cur);
        }
        it = end;
    }
    if (timed) {
        hip_check(hipStreamSynchronize(p->stream), "timing sync");
        double a = 0, b = 0;
        for (size_t i = 0; i + 3 < p->ev_used; i += 4) {
            float t1 = 0, t2 = 0;
            hip_check(hipEventElapsedTime(&t1, p->ev_pool[i], p->ev_pool[i + 1]), "elapsed");
            hip_check(hipEventElapsedTime(&t2, p->ev_pool[i + 2], p->ev_pool[i + 3]), "elapsed");
            a += t1;
            b += t2;
        }
        p->t1_ms = a;
        p->t2_ms = b;
        p->t_launches = (int64_t)(p->ev_used / 4);
    }
    return SMX_OK;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Launch shapes of the fused pass tried by the autotuner (same grid and
// accumulator type as `base`): 8/16/32 lanes per row with 4 or 8 entries per
// load re-reading the entries for the scatter, and the register-cached shapes
// (256 entries of a row in registers); zl_only: only the shapes with z in LDS
// (the ones that store dose-volume rows' values).
std::vector<FusedCfg> fused_candidates(const FusedCfg &base, int64_t n, bool zl_only = false)
{
    std::vector<FusedCfg> out;
    if (!zl_only)
    for (int lpr : {8, 16, 32})
        for (int vec : {4, 8}) {
            FusedCfg t = base;
            t.lpr = lpr;
            t.vec = vec;
            t.cap = 0;
            t.zl = 0;
            out.push_back(t);
            if (lpr >= 16) {
                t.cap = 256 / (lpr * vec);
                out.push_back(t);
            }
        }
    if (fused_zl_lds_bytes(n) <= fused_lds_limit()) // z in LDS beside a float32 y
        for (int lpr : {8, 16, 32})
            for (int vec : {4, 8}) {
                FusedCfg t = base;
                t.lpr = lpr;
                t.vec = vec;
                t.cap = 0;
                t.acc64 = 0;
                t.zl = 1;
                out.push_back(t);
                t.cap = fused_zl_cap(lpr, vec); // the row's first entries kept in registers
                out.push_back(t);
            }
    return out;
}

// The dose-volume constraints of a descriptor as the kernels' table
// (validated against m rows).
int build_dvc_table(const smx_problem_desc *d, int64_t m, DvcTable &dt)
{
    dt = DvcTable{};
    if (d->n_dvc < 0 || d->n_dvc > kMaxDvc || (d->n_dvc > 0 && !d->dvc))
        return fail(SMX_EINVAL, "n_dvc must be in 0..%d with a table", kMaxDvc);
    dt.n = d->n_dvc;
    for (int g = 0; g < dt.n; ++g) {
        const smx_dvc &G = d->dvc[g];
        if (!(G.row_begin >= 0 && G.row_begin < G.row_end && G.row_end <= m))
            return fail(SMX_EINVAL, "dose-volume constraint %d: rows [%lld, %lld) not a nonempty block of [0, %lld)", g,
                        (long long)G.row_begin, (long long)G.row_end, (long long)m);
        if (g > 0 && G.row_begin != d->dvc[g - 1].row_end)
            return fail(SMX_EINVAL, "dose-volume constraint %d does not start where constraint %d ends", g, g - 1);
        if (G.sense != SMX_DVC_MAX && G.sense != SMX_DVC_MIN)
            return fail(SMX_EINVAL, "dose-volume constraint %d: unknown sense %d", g, G.sense);
        if (!(G.fraction >= 0.0 && G.fraction <= 1.0))
            return fail(SMX_EINVAL, "dose-volume constraint %d: fraction must be in [0, 1]", g);
        if (!std::isfinite(G.dose)) return fail(SMX_EINVAL, "dose-volume constraint %d: dose must be finite", g);
        if (G.row_end - G.row_begin > (int64_t)0xFFFFFFFFll)
            return fail(SMX_EINVAL, "dose-volume constraint %d: too many rows", g);
        const int64_t N = G.row_end - G.row_begin;
        const double kv = (G.sense == SMX_DVC_MAX) ? std::floor(G.fraction * (double)N) : std::ceil(G.fraction * (double)N);
        dt.begin[g] = G.row_begin;
        dt.end[g] = G.row_end;
        dt.k[g] = (long long)std::min<double>(std::max(kv, 0.0), (double)N);
        dt.dose[g] = G.dose;
        dt.sense[g] = G.sense == SMX_DVC_MAX ? 0 : 1;
        dt.blk_begin[g + 1] = dt.blk_begin[g] + (int)((N + kDvcChunk - 1) / kDvcChunk);
    }
    if (dt.n > 0) {
        dt.nblk = dt.blk_begin[dt.n];
        dt.lo = dt.begin[0];
        dt.span = dt.end[dt.n - 1] - dt.begin[0];
        if (dt.nblk > 65535) return fail(SMX_EINVAL, "dose-volume constraints hold too many rows");
    }
    return SMX_OK;
}

// Launch shape of the fused single pass for a problem of n unknowns and B
// slices on the current device, or false where it has none: one slice, no
// dose-volume rows (their ranking precedes c), an LDS copy of y that fits
// (float64 if it can, else float32), one or two workgroups per CU as the LDS
// allows.
bool fused_plan(int64_t n, int B, int n_dvc, FusedCfg &c, size_t &lds_bytes)
{
    if (B != 1) return false;
    // dose-volume rows: the shapes with z in LDS store their values for the
    // ranking, and a second kernel adds their c_i a_i once it has set them
    if (n_dvc > 0 && fused_zl_lds_bytes(n) > fused_lds_limit()) return false;
    const size_t lim = fused_lds_limit();
    int acc64 = -1;
    if (fused_lds_bytes(n, 1) <= lim) acc64 = 1;
    else if (fused_lds_bytes(n, 0) <= lim) acc64 = 0;
    if (acc64 < 0) return false;
    int dev = 0, cus = 0, lds_cu = 0;
    hip_check(hipGetDevice(&dev), "device");
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
        lds_cu = 0;
    lds_bytes = fused_lds_bytes(n, acc64);
    const int per_cu = (lds_cu > 0 && size_t(lds_cu) >= 2 * (lds_bytes + 1024)) ? 2 : 1;
    c = FusedCfg{};
    c.vec = 4;
    c.cap = 0;
    c.grid = std::max(1, std::min(cus * per_cu, kMaxPassGrid));
    c.acc64 = acc64;
    return true;
}

// Whether one-slice problems on the current device get the LDS-staged passes
// (and, on operators with row panels, the panel pass 2's per-panel sums).
bool lds_passes_available(int B) { return B == 1 && fused_lds_limit() >= sizeof(float) * size_t(kLdsPassFloats); }

// Row panels of the column copy an operator with m rows holds.
int64_t panel_count(int64_t m) { return m > kLdsPassFloats ? (m + kLdsPassFloats - 1) / kLdsPassFloats : 0; }

// Device bytes of every buffer create_problem allocates for an operator with
// m rows, n columns, float32 values (has_f32) and/or the reduced-precision
// kind lp, and the descriptor d (whose fields the sizes depend on are
// validated by the caller), in the order it allocates them.  DBuf takes 256
// bytes for an empty buffer.
size_t problem_plan_bytes(int64_t m, int64_t n, bool has_f32, int lp, const smx_problem_desc *d, const DvcTable &dt)
{
    const size_t B = size_t(d->B), M = size_t(m), N = size_t(n);
    size_t t = 0;
    auto add = [&t](size_t b) { t += (b == 0) ? 256 : b; };
    add(4 * M * B); // lower
    add(4 * M * B); // upper
    add(4 * N);     // box_lo
    add(4 * N);     // box_hi
    add(8 * M);     // weights
    if (d->obj_kind == SMX_OBJ_LINEAR) add(4 * N);
    add(4 * N * B); // x
    add(4 * N * B); // g
    add(4 * M * B); // c
    add(sizeof(SliceState) * 2 * B);
    if (d->stop_on && d->stop_var > 0.0) {
        add(4 * N * B);
        add(8 * 2 * 256 * B);
    }
    const int kinds = (has_f32 ? 1 : 0) + (lp != VK_F32 ? 1 : 0);
    for (int k = 0; k < kinds; ++k) add(4 * M); // D
    if (d->basic == SMX_BASIC_CQ || d->basic == SMX_BASIC_EMR)
        for (int k = 0; k < kinds; ++k) add(4 * M); // step weights
    if (d->basic == SMX_BASIC_EL || d->basic == SMX_BASIC_EMR) {
        add(8 * N * B);
        if (d->basic == SMX_BASIC_EMR) add(4 * N * B);
        add(8 * size_t(kMaxPassGrid) * B);
        add(8 * size_t(kMaxPassGrid) * B);
    }
    if (dt.n > 0) {
        add(8 * size_t(dt.span) * B);
        add(8 * size_t(dt.span) * B);
        add(sizeof(unsigned) * size_t(kDvcBins) * dt.n * B);
        add(sizeof(DvcSel) * dt.n * B);
        add(8 * size_t(dt.nblk) * B);
    }
    FusedCfg fc;
    size_t lds = 0;
    if (fused_plan(n, d->B, dt.n, fc, lds)) {
        add(lds * size_t(fc.grid)); // partial vectors of y
        if (d->obj_kind == SMX_OBJ_LINEAR) add(8 * 2 * size_t(fused_apply_grid(n))); // direction partials
    }
    if (lds_passes_available(d->B) && panel_count(m) > 0) add(8 * size_t(panel_count(m)) * N);
    PertParams pp{};
    pp.obj = d->obj_kind;
    pp.B = d->B;
    pp.n = n;
    pp.tv_rows = d->tv_rows;
    pp.tv_cols = d->tv_cols;
    const size_t pgrid = size_t(phase_grid(pp)),
                 trials = d->step_rule == SMX_STEP_ADAPTIVE ? 1 : size_t(std::max(1, d->max_trials));
    add(8 * size_t(kMaxPassGrid) * B); // pass partials
    add(8 * size_t(kMaxPassGrid) * B); // query partials
    add(8 * pgrid * B * 2);
    add(8 * pgrid * B * trials);
    add(8 * pgrid * B * trials);
    add(8 * 2 * B); // query output
    if (d->history_cap > 0) {
        const size_t hc = size_t(d->history_cap) * B;
        for (int k = 0; k < 3; ++k) add(8 * hc);
        for (int k = 0; k < 2; ++k) add(4 * hc);
    }
    return t;
}

// Fused single pass for one slice when an LDS copy of y fits (float64 if it
// can, else float32).  Lanes per row follow the mean row length; one or two
// workgroups per CU, as many as the LDS allows.
void setup_fused(smx_problem *p)
{
    FusedCfg c;
    size_t bytes = 0;
    if (!fused_plan(p->n, p->B, p->dvc.n, c, bytes)) return;
    const DevLayout &L = p->op->csr;
    const double mean = L.rows > 0 ? double(L.slots) / double(L.rows) : 0.0;
    c.lpr = mean <= 64 ? 8 : (mean <= 256 ? 16 : 32);
    const bool dvc = p->dvc.n > 0;
    if (dvc) { // z in LDS: two sets of float32 partials fit the float64 plan's bytes
        c.zl = 1;
        c.acc64 = 0;
        c.lpr = 8;
    }
    bool any = false;
    for (int vk = 0; vk < 3; ++vk) {
        const bool present = (vk == VK_F32) ? p->op->has_f32 : (vk == p->op->lp_kind());
        if (!present) continue;
        bool ok = true;
        for (const FusedCfg &t : fused_candidates(c, p->n, dvc))
            if (prepare_fused(t, fused_fmt(p, vk), p->n) != hipSuccess) ok = false;
        if (dvc && prepare_scatter_rows(fused_fmt(p, vk), p->n) != hipSuccess) ok = false;
        (void)hipGetLastError();
        p->fused_ok[vk] = p->fused[vk] = ok;
        p->fcfg[vk] = c;
        any = any || ok;
    }
    if (any) p->ypart.alloc(bytes * size_t(c.grid), "fused partial vectors");
    if (any && p->pp.obj == OBJ_LINEAR) // the next phase's direction partials, from the apply kernel
        p->part_lin.alloc(sizeof(double) * 2 * size_t(fused_apply_grid(p->n)), "direction partials");
}

int create_problem(smx_operator *op, const smx_problem_desc *d, hipStream_t s, smx_problem **out)
{
    if (!op || !d || !out) return fail(SMX_EINVAL, "NULL argument");
    *out = nullptr;
    const int64_t m = op->m, n = op->n;
    const int B = d->B;
    if (!(is_pow2(B) && B <= 32)) return fail(SMX_EINVAL, "B must be a power of two in 1..32 (got %d)", B);
    if (d->basic < SMX_BASIC_SIMULT || d->basic > SMX_BASIC_EMR) return fail(SMX_EINVAL, "unknown basic algorithm %d", d->basic);
    // DROP's range depends on the weights and is checked once they are normalised
    if (!(d->lambda > 0.0) || (d->basic != SMX_BASIC_DROP && !(d->lambda <= 2.0)))
        return fail(SMX_EINVAL, "lambda must be in (0, 2] (got %g)", d->lambda);
    if (d->obj_kind < SMX_OBJ_NONE || d->obj_kind > SMX_OBJ_L1) return fail(SMX_EINVAL, "unknown objective %d", d->obj_kind);
    if (d->obj_kind != SMX_OBJ_NONE) {
        if (!(d->gamma > 0.0) || !std::isfinite(d->gamma)) return fail(SMX_EINVAL, "gamma must be > 0 (got %g)", d->gamma);
        if (!(d->alpha > 0.0 && d->alpha < 1.0)) return fail(SMX_EINVAL, "alpha must be in (0, 1) (got %g)", d->alpha);
        if (d->n_red < 1) return fail(SMX_EINVAL, "n_red must be >= 1 (got %d)", d->n_red);
        if (d->max_trials < 1 || d->max_trials > 1024) return fail(SMX_EINVAL, "max_trials must be in 1..1024 (got %d)", d->max_trials);
        if (d->restart_every < 0) return fail(SMX_EINVAL, "restart_every must be >= 0");
    }
    if (d->obj_kind == SMX_OBJ_TV2D) {
        if (d->tv_rows < 1 || d->tv_cols < 1 || (int64_t)d->tv_rows * d->tv_cols != n)
            return fail(SMX_EINVAL, "TV image %d x %d does not match n = %lld", d->tv_rows, d->tv_cols, (long long)n);
        if (!(d->tv_eps >= 0.0) || !std::isfinite(d->tv_eps)) return fail(SMX_EINVAL, "tv_eps must be >= 0");
    }
    if (d->obj_kind == SMX_OBJ_LINEAR && !d->linear_c) return fail(SMX_EINVAL, "LINEAR objective needs linear_c");
    if (d->step_rule != SMX_STEP_POWER && d->step_rule != SMX_STEP_ADAPTIVE)
        return fail(SMX_EINVAL, "unknown step rule %d", d->step_rule);
    if (!d->lower || !d->upper) return fail(SMX_EINVAL, "lower and upper bounds are required");
    if (d->history_cap < 0) return fail(SMX_EINVAL, "history_cap must be >= 0");
    StopParams sp{};
    if (d->stop_on) {
        if (d->stop_n < 1) return fail(SMX_EINVAL, "stop_n must be >= 1 (got %d)", d->stop_n);
        if (d->stop_max_iters < 0) return fail(SMX_EINVAL, "stop_max_iters must be >= 0");
        if (std::isnan(d->stop_prox) || std::isnan(d->stop_dprox) || std::isnan(d->stop_dobj) ||
            !(d->stop_var >= 0.0) || !std::isfinite(d->stop_var))
            return fail(SMX_EINVAL, "invalid stopping thresholds");
        sp = StopParams{1, d->stop_n, (long long)d->stop_max_iters, d->stop_prox, d->stop_dprox, d->stop_dobj,
                        d->stop_var};
    }
    DvcTable dt{};
    if (const int rc = build_dvc_table(d, m, dt); rc != SMX_OK) return rc;
    const bool dev = d->on_device != 0;
    std::vector<float> lo = fetch(d->lower, m * B, dev), up = fetch(d->upper, m * B, dev);
    for (int64_t i = 0; i < m * B; ++i) {
        if (std::isnan(lo[i]) || std::isnan(up[i])) return fail(SMX_EINVAL, "NaN bound at %lld", (long long)i);
        if (lo[i] > up[i]) return fail(SMX_EINVAL, "lower > upper at %lld", (long long)i);
    }
    std::vector<double> w(m, 1.0);
    if (d->weights) {
        w = fetch(d->weights, m, dev);
        for (int64_t i = 0; i < m; ++i)
            if (!(w[i] > 0.0) || !std::isfinite(w[i])) return fail(SMX_EINVAL, "weight %lld must be finite and > 0", (long long)i);
    }
    double wsum = 0.0;
    for (double v : w) wsum += v;
    for (double &v : w) v /= wsum;
    if (d->basic == SMX_BASIC_DROP) {
        double wmax = 0.0;
        for (double v : w) wmax = std::max(wmax, v);
        if (!(d->lambda <= 2.0 / wmax))
            return fail(SMX_EINVAL, "DROP needs lambda in (0, 2/max w] = (0, %g] (got %g)", 2.0 / wmax, d->lambda);
    }
    std::vector<float> blo(n, -INFINITY), bhi(n, INFINITY);
    if (d->box_lo) blo = fetch(d->box_lo, n, dev);
    if (d->box_hi) bhi = fetch(d->box_hi, n, dev);
    for (int64_t j = 0; j < n; ++j) {
        if (std::isnan(blo[j]) || std::isnan(bhi[j]) || blo[j] > bhi[j])
            return fail(SMX_EINVAL, "invalid box at %lld", (long long)j);
    }
    std::vector<float> lc;
    if (d->obj_kind == SMX_OBJ_LINEAR) {
        lc = fetch(d->linear_c, n, dev);
        for (float v : lc)
            if (!std::isfinite(v)) return fail(SMX_EINVAL, "non-finite linear_c");
    }
    std::unique_ptr<smx_problem> p(new smx_problem());
    p->op = op;
    p->device = op->device;
    p->stream = s;
    p->B = B;
    p->m = m;
    p->n = n;
    p->lambda = (float)d->lambda;
    p->refine_iters = d->refine_iters;
    p->basic = d->basic;
    PertParams &pp = p->pp;
    pp.obj = d->obj_kind;
    pp.B = B;
    pp.n = n;
    pp.tv_rows = d->tv_rows;
    pp.tv_cols = d->tv_cols;
    pp.tv_eps2 = d->tv_eps * d->tv_eps;
    pp.gamma = d->gamma;
    pp.alpha = d->alpha;
    pp.n_red = std::max(1, d->n_red);
    pp.restart_every = d->restart_every;
    pp.max_trials = std::max(1, d->max_trials);
    pp.adaptive = d->step_rule == SMX_STEP_ADAPTIVE ? 1 : 0;
    if (pp.adaptive) { // one step per phase
        pp.n_red = 1;
        pp.max_trials = 1;
    }
    // a linear objective accepts its first trial (f(z) - f(x) = -beta ||c||): one
    // trial per first launch instead of a speculative batch
    pp.first_width = pp.obj == OBJ_LINEAR ? 1 : std::min(pp.max_trials, kFirstWidth);
    if (phase_in_one_launch(pp)) hip_check(prepare_phase_small(), "one-launch phase");
    upload(p->lower, lo, s, "bounds");
    upload(p->upper, up, s, "bounds");
    upload(p->box_lo, blo, s, "box");
    upload(p->box_hi, bhi, s, "box");
    upload(p->w, w, s, "weights");
    if (!lc.empty()) upload(p->lin_c, lc, s, "linear objective");
    p->x.alloc(sizeof(float) * n * B, "iterate");
    hip_check(launch_fill(p->x.as<float>(), 0.f, n * B, s), "zero iterate");
    p->g.alloc(sizeof(float) * n * B, "gradient");
    p->c.alloc(sizeof(float) * m * B, "weighted residual");
    p->st.alloc(sizeof(SliceState) * 2 * B, "state");
    hip_check(launch_init_state(p->state(0), B, sp, s), "init state");
    hip_check(launch_init_state(p->state(1), B, sp, s), "init state");
    p->stop_var = sp.on && sp.var > 0.0;
    if (p->stop_var) {
        p->xprev.alloc(sizeof(float) * n * B, "previous iterate");
        p->part_var.alloc(sizeof(double) * 2 * 256 * B, "variance partials");
    }
    p->cur = 0;
    const int lp = op->lp_kind();
    if (op->has_f32) {
        p->D32.alloc(sizeof(float) * m, "D");
        hip_check(launch_make_D(op->q32.as<double>(), p->w.as<double>(), p->D32.as<float>(), m, s), "D");
    }
    if (lp != VK_F32) {
        p->D16.alloc(sizeof(float) * m, "D (reduced precision)");
        hip_check(launch_make_D(op->q16.as<double>(), p->w.as<double>(), p->D16.as<float>(), m, s), "D");
    }
    if (p->basic == SMX_BASIC_CQ || p->basic == SMX_BASIC_EMR) {
        // step weights: CQ 1/||A||_F^2 (the squared Frobenius norm of the stored
        // operator, the sum of its float64 row norms in row order), EMR the weights
        std::vector<int> kinds;
        if (op->has_f32) kinds.push_back(VK_F32);
        if (op->lp_kind() != VK_F32) kinds.push_back(op->lp_kind());
        for (int vk : kinds) {
            std::vector<float> sw(m);
            if (p->basic == SMX_BASIC_EMR) {
                for (int64_t i = 0; i < m; ++i) sw[i] = (float)w[i];
            } else {
                std::vector<double> q(m);
                const DBuf &qd = (vk == VK_F32) ? op->q32 : op->q16;
                hip_check(hipMemcpy(q.data(), qd.p, sizeof(double) * m, hipMemcpyDeviceToHost), "row norms");
                double fro2 = 0.0;
                for (double v : q) fro2 += v;
                const float f = fro2 > 0.0 ? (float)(1.0 / fro2) : 0.f;
                for (int64_t i = 0; i < m; ++i) sw[i] = f;
            }
            upload(vk == VK_F32 ? p->S32 : p->S16, sw, s, "step weights");
        }
    }
    if (p->basic == SMX_BASIC_EL || p->basic == SMX_BASIC_EMR) {
        p->ybuf.alloc(sizeof(double) * n * B, "extrapolated step");
        if (p->basic == SMX_BASIC_EMR) p->ybuf32.alloc(sizeof(float) * n * B, "extrapolated step");
        p->part_y.alloc(sizeof(double) * size_t(kMaxPassGrid) * B, "step partials");
        p->part_q.alloc(sizeof(double) * size_t(kMaxPassGrid) * B, "step partials");
    }
    if (const int lk = op->lp_kind(); lk != VK_F32) { // the packed entries where the index range allows
        const int pk = (lk == VK_BF16) ? VK_BF16P : VK_F16P;
        p->fmt1[lk] = op->csr.packed.p ? pk : lk;
        p->fmt2[lk] = op->csc.packed.p ? pk : lk;
    }
    // "rows" selects the lanes-per-row kernels, "interleaved" the interleaved-lane pass 1
    const char *mode_env = getenv("SMX_PASS_MODE");
    const bool rows_mode = mode_env && std::strcmp(mode_env, "rows") == 0;
    const bool inter_mode = mode_env && std::strcmp(mode_env, "interleaved") == 0;
    // SMX_TILES: "0" keeps the column copy for pass 2; "1" starts every problem
    // whose tiles fit on the tile pass; unset, one-slice problems start there and
    // the autotuner may move any problem whose tiles fit there
    const char *tiles_env = getenv("SMX_TILES");
    const bool tiles_off = tiles_env && std::strcmp(tiles_env, "0") == 0;
    const bool tiles_on = tiles_env && std::strcmp(tiles_env, "1") == 0;
    const bool use_tiles = op->has_tiles() && tiles_fit(op->t_max_rows, B) && !tiles_off;
    const bool start_tiles = use_tiles && (B == 1 || tiles_on);
    if (B == 1 && op->has_f32) { // one slice: the float32 passes read 16-bit indices where the range allows
        if (op->csr.idx16.p) p->fmt1[VK_F32] = VK_F32U16;
        if (op->csc.idx16.p) p->fmt2[VK_F32] = VK_F32U16;
    }
    p->tiles_ok = use_tiles;
    for (int vk = 0; vk < 3; ++vk) {
        p->cfg1[vk] = (rows_mode && B == 1) ? pick_cfg_rows(op->csr, vk) : pick_cfg(op->csr, vk, B);
        p->cfg2[vk] = (rows_mode && B == 1) ? pick_cfg_rows(op->csc, vk) : pick_cfg(op->csc, vk, B);
        if (inter_mode && B == 1) {
            p->cfg1[vk].mode = 0;
            p->cfg1[vk].lpr = 16;
            p->cfg1[vk].vec = 1;
            p->cfg1[vk].grid = (int)std::min<int64_t>(std::max<int64_t>(1, (m + 15) / 16), kMaxPassGrid);
        }
        if (start_tiles) {
            p->cfg2[vk].mode = 2;
            p->cfg2[vk].lpr = 4;
            p->cfg2[vk].vec = 4;
            p->cfg2[vk].grid = std::max(1, std::min(op->t_ntiles, kMaxPassGrid));
        }
    }
    p->dvc = dt;
    if (dt.n > 0) {
        p->dvc_dose.alloc(sizeof(double) * size_t(dt.span) * B, "dose-volume rows");
        p->dvc_key.alloc(sizeof(unsigned long long) * size_t(dt.span) * B, "dose-volume keys");
        p->dvc_hist.alloc(sizeof(unsigned) * size_t(kDvcBins) * dt.n * B, "dose-volume histograms");
        hip_check(hipMemsetAsync(p->dvc_hist.p, 0, sizeof(unsigned) * size_t(kDvcBins) * dt.n * B, s),
                  "dose-volume histograms");
        p->dvc_sel.alloc(sizeof(DvcSel) * dt.n * B, "dose-volume selection");
        hip_check(hipMemsetAsync(p->dvc_sel.p, 0, sizeof(DvcSel) * dt.n * B, s), "dose-volume selection");
        p->dvc_part.alloc(sizeof(double) * size_t(dt.nblk) * B, "dose-volume partials");
    }
    setup_fused(p.get());
    if (lds_passes_available(B)) { // the LDS-staged pass 1
        int dev = 0, cus = 0;
        hip_check(hipGetDevice(&dev), "device");
        hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
        hip_check(prepare_lds_passes(), "LDS pass setup");
        p->lds_grid = std::max(1, std::min(cus, kMaxPassGrid));
        p->lds_x = (int)std::min<int64_t>(n, kLdsPassFloats);
        p->lds_c = (int)std::min<int64_t>(m, kLdsPassFloats);
        if (op->panel_np > 0) p->ypanel.alloc(sizeof(double) * size_t(op->panel_np) * n, "panel sums");
        const char *me = getenv("SMX_PASS_MODE"); // "lds" starts both passes there, "panels" pass 2 in row panels
        if (me && std::strcmp(me, "panels") == 0 && op->panel_np > 0)
            for (int vk = 0; vk < 3; ++vk) {
                PassCfg &c = p->cfg2[vk];
                c.mode = 5;
                c.lpr = 16;
                c.vec = 4;
                c.grid = p->lds_grid;
            }
        if (me && std::strcmp(me, "lds") == 0)
            for (int vk = 0; vk < 3; ++vk)
                for (int k = 0; k < 2; ++k) {
                    PassCfg &c = k ? p->cfg2[vk] : p->cfg1[vk];
                    c.mode = 3;
                    c.lpr = 8;
                    c.vec = 4;
                    c.grid = p->lds_grid;
                    c.xlds = k ? p->lds_c : p->lds_x;
                }
    }
    // per-workgroup partial sums of each kernel kind
    const int64_t pgrid = phase_grid(pp);
    p->part_pass.alloc(sizeof(double) * size_t(kMaxPassGrid) * B, "pass partials");
    p->part_query.alloc(sizeof(double) * size_t(kMaxPassGrid) * B, "query partials");
    p->part_phase.alloc(sizeof(double) * size_t(pgrid) * B * 2, "phase partials");
    p->part_trial[0].alloc(sizeof(double) * size_t(pgrid) * B * pp.max_trials, "trial partials");
    p->part_trial[1].alloc(sizeof(double) * size_t(pgrid) * B * pp.max_trials, "trial partials");
    p->qout.alloc(sizeof(double) * 2 * B, "query output");
    p->hist_cap = d->history_cap;
    if (d->history_cap > 0) {
        const size_t hc = size_t(d->history_cap) * B;
        p->h_prox.alloc(sizeof(double) * hc, "history");
        p->h_fs.alloc(sizeof(double) * hc, "history");
        p->h_fe.alloc(sizeof(double) * hc, "history");
        p->h_tr.alloc(sizeof(int) * hc, "history");
        p->h_ac.alloc(sizeof(int) * hc, "history");
    }
    p->hist.prox = p->h_prox.as<double>();
    p->hist.f_start = p->h_fs.as<double>();
    p->hist.f_end = p->h_fe.as<double>();
    p->hist.trials = p->h_tr.as<int>();
    p->hist.accepts = p->h_ac.as<int>();
    p->hist.cap = d->history_cap;
    hip_check(hipStreamSynchronize(s), "problem setup");
    (void)scratch_on_current_device(); // the no-alloc slot load's scratch is resident from here on
    op->refs.fetch_add(1);
    *out = p.release();
    return SMX_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate launch shapes of both passes on the problem's own
// operator and keeps the fastest.  Timing runs on scratch copies of the
// iterate, the weighted residual and the state, so the problem is unchanged.
// ---------------------------------------------------------------------------

std::vector<PassCfg> pass_candidates(const DevLayout &L, int vk, int B)
{
    std::vector<PassCfg> out;
    auto add = [&](const PassCfg &c) {
        for (auto &o : out)
            if (o.mode == c.mode && o.lpr == c.lpr && o.vec == c.vec && o.grid == c.grid) return;
        out.push_back(c);
    };
    if (B == 1) {
        for (int g : {1024, 2048, 4096}) {
            PassCfg c = pick_cfg(L, vk, 1);
            c.grid = std::max(1, std::min({L.nblk, g, kMaxPassGrid}));
            add(c);
        }
    }
    const std::vector<int> lprs = (B == 1) ? std::vector<int>{2, 4, 8, 16, 32} : std::vector<int>{4, 8, 16};
    const std::vector<int> vecs = (B == 1) ? std::vector<int>{4, 8} : std::vector<int>{(vk == VK_F32) ? 4 : 8};
    for (int lpr : lprs)
        for (int vec : vecs)
            for (int g : {1024, 2048, 4096}) {
                PassCfg c;
                c.mode = 0;
                c.lpr = lpr;
                c.vec = vec;
                const int64_t rpb = kBlock / lpr;
                const int64_t need = std::max<int64_t>(1, (L.rows + rpb - 1) / rpb);
                c.grid = (int)std::min<int64_t>({need, (int64_t)g, (int64_t)kMaxPassGrid});
                add(c);
            }
    return out;
}

int autotune_impl(smx_problem *p, int reps)
{
    if (reps < 1) reps = 10;
    hipStream_t s = p->stream;
    const int64_t m = p->m, n = p->n;
    DBuf xs, cs, sts;
    xs.alloc(sizeof(float) * n * p->B, "tuning scratch");
    cs.alloc(sizeof(float) * m * p->B, "tuning scratch");
    sts.alloc(sizeof(SliceState) * 2 * p->B, "tuning scratch");
    hip_check(hipMemcpyAsync(xs.p, p->x.p, sizeof(float) * n * p->B, hipMemcpyDeviceToDevice, s), "tuning copy");
    SliceState *st0 = sts.as<SliceState>(), *st1 = st0 + p->B;
    hip_check(launch_init_state(st0, p->B, StopParams{}, s), "tuning state");
    hip_check(launch_init_state(st1, p->B, StopParams{}, s), "tuning state");
    Hist none{};
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    const char *log_env = getenv("SMX_TUNE_LOG"); // "1" prints every candidate's time to stderr
    const bool tune_log = log_env && std::strcmp(log_env, "1") == 0;
    auto elapsed = [&]() {
        float ms = 0.f;
        hip_check(hipEventSynchronize(e1), "tuning sync");
        hip_check(hipEventElapsedTime(&ms, e0, e1), "tuning elapsed");
        return (double)ms / reps;
    };
    std::vector<int> kinds;
    if (p->op->has_f32) kinds.push_back(VK_F32);
    if (p->op->lp_kind() != VK_F32) kinds.push_back(p->op->lp_kind());
    try {
        for (int vk : kinds) {
            const RowW rw = p->row_weights(vk);
            const ColStep cstep = p->col_step(false);
            // pass 1 (also with interleaved lanes, vec = 1, for one slice)
            double best = 1e30;
            PassCfg bestc = p->cfg1[vk];
            std::vector<PassCfg> cands1 = pass_candidates(p->op->csr, vk, p->B);
            if (p->B == 1)
                for (int lpr : {8, 16, 32, 64})
                    for (int g : {1024, 2048, 4096}) {
                        PassCfg c;
                        c.mode = 0;
                        c.lpr = lpr;
                        c.vec = 1;
                        const int64_t rpb = kBlock / lpr;
                        c.grid = (int)std::min<int64_t>({std::max<int64_t>(1, (p->m + rpb - 1) / rpb), (int64_t)g,
                                                         (int64_t)kMaxPassGrid});
                        bool dup = false;
                        for (auto &o : cands1) dup = dup || (o.mode == 0 && o.lpr == lpr && o.vec == 1 && o.grid == c.grid);
                        if (!dup) cands1.push_back(c);
                    }
            // the LDS-staged passes, where LDS holds at least half of the gathered vector
            if (p->lds_grid > 0 && 2 * int64_t(p->lds_x) >= n)
                for (int lpr : {4, 8, 16, 32})
                    for (int vec : {4, 8}) {
                        PassCfg c;
                        c.mode = 3;
                        c.lpr = lpr;
                        c.vec = vec;
                        c.grid = p->lds_grid;
                        c.xlds = p->lds_x;
                        cands1.push_back(c);
                    }
            for (const PassCfg &c : cands1) {
                auto launch = [&]() {
                    hip_check(launch_pass1(c, view_for(p->op, false, p->fmt1[vk]), p->op->csr.blocks(), p->fmt1[vk],
                                           xs.as<float>(),
                                           p->lower.as<float>(), p->upper.as<float>(), rw, cs.as<float>(), st0, p->B, 1,
                                           p->part_query.as<double>(), s),
                              "tuning pass 1");
                };
                launch();
                launch();
                hip_check(hipEventRecord(e0, s), "event");
                for (int r = 0; r < reps; ++r) launch();
                hip_check(hipEventRecord(e1, s), "event");
                const double t = elapsed();
                if (tune_log)
                    fprintf(stderr, "smx tune: kind %d mode %d lpr %d vec %d grid %d: %.2f us\n", vk, c.mode, c.lpr, c.vec,
                            c.grid, t * 1e3);
                if (t < best) {
                    best = t;
                    bestc = c;
                }
            }
            p->cfg1[vk] = bestc;
            const double two_pass1 = best;
            // pass 2 (the residual from the chosen pass 1)
            best = 1e30;
            PassCfg bestc2 = p->cfg2[vk];
            std::vector<PassCfg> cands2 = pass_candidates(p->op->csc, vk, p->B);
            if (p->lds_grid > 0 && p->op->panel_np > 0)
                for (int lpr : {8, 16, 32, 64})
                    for (int vec : {4, 8}) {
                        PassCfg c;
                        c.mode = 5;
                        c.lpr = lpr;
                        c.vec = vec;
                        c.grid = p->lds_grid;
                        cands2.push_back(c);
                    }
            if (p->lds_grid > 0 && 2 * int64_t(p->lds_c) >= m)
                for (int lpr : {4, 8, 16, 32})
                    for (int vec : {4, 8}) {
                        PassCfg c;
                        c.mode = 3;
                        c.lpr = lpr;
                        c.vec = vec;
                        c.grid = p->lds_grid;
                        c.xlds = p->lds_c;
                        cands2.push_back(c);
                    }
            if (p->tiles_ok)
                for (int lpr : {2, 4, 8, 16})
                    for (int vec : {4, 8})
                        for (int g : {1024, 2048, 4096}) {
                            PassCfg c;
                            c.mode = 2;
                            c.lpr = lpr;
                            c.vec = vec;
                            c.grid = std::max(1, std::min({p->op->t_ntiles, g, kMaxPassGrid}));
                            bool dup = false;
                            for (auto &o : cands2) dup = dup || (o.mode == 2 && o.lpr == lpr && o.vec == vec && o.grid == c.grid);
                            if (!dup) cands2.push_back(c);
                        }
            for (const PassCfg &c : cands2) {
                auto launch = [&]() {
                    hip_check(pass2_any(p, vk, c, cs.as<float>(), xs.as<float>(), cstep, st0, st1,
                                        p->part_query.as<double>(), bestc.grid, none, s),
                              "tuning pass 2");
                };
                launch();
                launch();
                hip_check(hipEventRecord(e0, s), "event");
                for (int r = 0; r < reps; ++r) launch();
                hip_check(hipEventRecord(e1, s), "event");
                const double t = elapsed();
                if (tune_log)
                    fprintf(stderr, "smx tune: kind %d mode %d lpr %d vec %d grid %d: %.2f us\n", vk, c.mode, c.lpr, c.vec,
                            c.grid, t * 1e3);
                if (t < best) {
                    best = t;
                    bestc2 = c;
                }
            }
            p->cfg2[vk] = bestc2;
            // the fused single pass, timed with its apply kernel, against the two passes
            if (p->fused_ok[vk] && p->fused_mode == 1) {
                double bestf = 1e30;
                FusedCfg bestfc = p->fcfg[vk];
                for (const FusedCfg &c : fused_candidates(p->fcfg[vk], n, p->dvc.n > 0)) {
                    auto launch = [&]() {
                        hip_check(launch_fused(c, view_for(p->op, false, fused_fmt(p, vk)), fused_fmt(p, vk), n, xs.as<float>(),
                                               p->lower.as<float>(), p->upper.as<float>(), rw, st0,
                                               p->part_query.as<double>(), p->ypart.p, s),
                                  "tuning fused pass");
                        int nvec = c.grid;
                        if (p->dvc.n > 0) { // the dose-volume rows' own scatter
                            hip_check(launch_scatter_rows(view_for(p->op, false, fused_fmt(p, vk)), fused_fmt(p, vk),
                                                          n, p->dvc.lo, p->dvc.lo + p->dvc.span, p->c.as<float>(),
                                                          st0, p->ypart.as<float>() + size_t(c.grid) * size_t(n),
                                                          c.grid, s),
                                      "tuning dose-volume rows");
                            nvec *= 2;
                        }
                        hip_check(launch_fused_apply(c, n, p->ypart.p, nvec, xs.as<float>(), cstep, st0, st1,
                                                     p->part_query.as<double>(), none, s),
                                  "tuning fused apply");
                    };
                    launch();
                    launch();
                    hip_check(hipEventRecord(e0, s), "event");
                    for (int r = 0; r < reps; ++r) launch();
                    hip_check(hipEventRecord(e1, s), "event");
                    const double t = elapsed();
                    if (tune_log)
                        fprintf(stderr, "smx tune: kind %d fused lpr %d vec %d cap %d zl %d grid %d: %.2f us\n", vk, c.lpr,
                                c.vec, c.cap, c.zl, c.grid, t * 1e3);
                    if (t < bestf) {
                        bestf = t;
                        bestfc = c;
                    }
                }
                p->fcfg[vk] = bestfc;
                p->fused[vk] = bestf < two_pass1 + best;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hip_check(hipStreamSynchronize(s), "tuning sync");
    // launch shapes are baked into captured graphs
    for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
    p->graphs.clear();
    p->tuned = true;
    return SMX_OK;
}

const char *fmt_name(int f)
{
    switch (f) {
    case VK_F32: return "f32+i32";
    case VK_BF16: return "bf16+i32";
    case VK_F16: return "f16+i32";
    case VK_BF16P: return "bf16+u16";
    case VK_F32U16: return "f32+u16";
    default: return "f16+u16";
    }
}

int describe_impl(const smx_problem *p, char *buf, size_t cap, size_t *need)
{
    std::string out = "{";
    const char *names[3] = {"f32", "bf16", "f16"};
    bool first = true;
    for (int vk = 0; vk < 3; ++vk) {
        if (vk == VK_F32 && !p->op->has_f32) continue;
        if (vk != VK_F32 && p->op->lp_kind() != vk) continue;
        char tmp[768];
        const PassCfg &a = p->cfg1[vk], &b = p->cfg2[vk];
        char fz[320];
        if (p->fused_ok[vk]) {
            const FusedCfg &f = p->fcfg[vk];
            snprintf(fz, sizeof fz,
                     "{\"in_use\": %s, \"lpr\": %d, \"vec\": %d, \"cap\": %d, \"zl\": %d, \"grid\": %d, "
                     "\"acc\": \"%s\", \"format\": \"%s\"}",
                     p->fused[vk] ? "true" : "false", f.lpr, f.vec, f.cap, f.zl, f.grid, f.acc64 ? "f64" : "f32",
                     fmt_name(fused_fmt(p, vk)));
        } else {
            snprintf(fz, sizeof fz, "null");
        }
        snprintf(tmp, sizeof tmp,
                 "%s\"%s\": {\"pass1\": {\"mode\": \"%s\", \"lpr\": %d, \"vec\": %d, \"grid\": %d, \"format\": \"%s\", "
                 "\"xlds\": %d}, "
                 "\"pass2\": {\"mode\": \"%s\", \"lpr\": %d, \"vec\": %d, \"grid\": %d, \"format\": \"%s\", "
                 "\"xlds\": %d}, "
                 "\"fused\": %s}",
                 first ? "" : ", ", names[vk], a.mode == 3 ? "lds" : (a.mode ? "stream" : "rows"), a.lpr, a.vec, a.grid,
                 fmt_name(p->fmt1[vk]), a.mode == 3 ? a.xlds : 0,
                 b.mode == 2 ? "tiles" : (b.mode == 3 ? "lds" : (b.mode == 5 ? "panels" : (b.mode ? "stream" : "rows"))),
                 b.lpr, b.vec, b.grid,
                 b.mode == 2 ? (vk == VK_F32 ? "f32+u16" : (vk == VK_BF16 ? "bf16+u16" : "f16+u16"))
                             : fmt_name(b.mode == 5 ? panel_fmt(p, vk) : p->fmt2[vk]),
                 b.mode == 3 ? b.xlds : 0,
                 fz);
        out += tmp;
        first = false;
    }
    char tail[512];
    static const char *basics[5] = {"simult", "drop", "cq", "el", "emr"};
    char tiles[96] = "null";
    if (p->op->has_tiles())
        snprintf(tiles, sizeof tiles, "{\"count\": %d, \"rows\": %lld, \"slots\": %lld}", p->op->t_ntiles,
                 (long long)(p->op->t_rlist.bytes / 4), (long long)p->op->tiles.slots);
    snprintf(tail, sizeof tail,
             ", \"tuned\": %s, \"row_blocks\": [%d, %d], \"basic\": \"%s\", \"dose_volume\": %d, \"tiles\": %s, "
             "\"device_bytes\": %zu, \"operator_bytes\": %zu, \"phase_launches\": %d}",
             p->tuned ? "true" : "false", p->op->csr.nblk, p->op->csc.nblk, basics[p->basic], p->dvc.n, tiles,
             p->device_bytes(), p->op->device_bytes(), p->pp.obj == OBJ_NONE ? 0 : phase_launch_count(p));
    out += tail;
    if (need) *need = out.size() + 1;
    if (buf && cap > 0) {
        const size_t k = std::min(cap - 1, out.size());
        std::memcpy(buf, out.data(), k);
        buf[k] = 0;
    }
    return SMX_OK;
}

#define SMX_GUARD(...)                                                                                               \
    try {                                                                                                             \
        g_err.clear();                                                                                                \
        __VA_ARGS__                                                                                                   \
    } catch (const HipError &h) {                                                                                     \
        return from_hip(h);                                                                                           \
    } catch (const std::bad_alloc &) {                                                                                \
        return fail(SMX_ENOMEM, "host allocation failed");                                                            \
    } catch (...) {                                                                                                   \
        return fail(SMX_EDEVICE, "unexpected internal error");                                                       \
    }

} // namespace

extern "C" {

int smx_version(int *major, int *minor)
{
    if (!major || !minor) return fail(SMX_EINVAL, "NULL argument");
    *major = SMX_VERSION_MAJOR;
    *minor = SMX_VERSION_MINOR;
    return SMX_OK;
}

const char *smx_last_error(void) { return g_err.c_str(); }

namespace {

// Read-only stream over a buffer: the rate at which a kernel that only reads
// HBM moves bytes on this device, the ceiling the passes' bandwidth is set
// against.  Each thread adds the 16-byte words it reads, four in flight; the
// workgroup's sum (so that no load can be dropped) goes through LDS.
__global__ __launch_bounds__(256) void k_stream_read(const float4 *__restrict__ v, long long n4,
                                                     float *__restrict__ partials)
{
    __shared__ float lds[256];
    float a = 0.f;
    const long long stride = (long long)gridDim.x * 256;
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        float4 t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = v[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) a += (t[u].x + t[u].y) + (t[u].z + t[u].w);
    }
    for (; i < n4; i += stride) {
        const float4 t = v[i];
        a += (t.x + t.y) + (t.z + t.w);
    }
    lds[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = lds[0];
}

} // namespace

int smx_read_rate_probe(const void *buf, size_t bytes, float *partials, int32_t grid, void *stream)
{
    if (!buf || !partials) return fail(SMX_EINVAL, "NULL argument");
    if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0 || bytes == 0 || (bytes & 15) != 0)
        return fail(SMX_EINVAL, "the buffer must be 16-byte aligned and hold a positive multiple of 16 bytes");
    if (grid < 1 || grid > 65535) return fail(SMX_EINVAL, "grid must be in 1..65535 (got %d)", grid);
    SMX_GUARD({
        hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream),
                           static_cast<const float4 *>(buf), (long long)(bytes / 16), partials);
        hip_check(hipGetLastError(), "read rate probe");
        return SMX_OK;
    })
}

int smx_operator_create(const smx_csr *A, int32_t value_storage, int32_t keep_f32, void *stream, smx_operator **out)
{
    SMX_GUARD(return create_operator(A, value_storage, keep_f32, (hipStream_t)stream, out);)
}

int smx_operator_create_image(const smx_csr *A, int32_t value_storage, int32_t keep_f32, int32_t image_rows,
                              int32_t image_cols, void *stream, smx_operator **out)
{
    if (!A) return fail(SMX_EINVAL, "NULL argument");
    if (image_rows < 1 || image_cols < 1 || (int64_t)image_rows * image_cols != A->n)
        return fail(SMX_EINVAL, "image %d x %d does not match n = %lld", image_rows, image_cols, (long long)A->n);
    SMX_GUARD(return create_operator(A, value_storage, keep_f32, (hipStream_t)stream, out, image_rows, image_cols);)
}

int smx_operator_destroy(smx_operator *op)
{
    SMX_GUARD(release_operator(op); return SMX_OK;)
}

int smx_operator_release_panels(smx_operator *op)
{
    if (!op) return fail(SMX_EINVAL, "NULL operator");
    SMX_GUARD({
        if (op->refs.load() != 1)
            return fail(SMX_ESTATE, "problems created from this operator still exist (%d references)",
                        op->refs.load() - 1);
        op->panel_ptr.release();
        op->panel_idx16.release();
        op->panel_packed.release();
        op->panel_np = 0;
        op->panel_P = 0;
        return SMX_OK;
    })
}

int smx_operator_footprint(int64_t m, int64_t n, int64_t nnz, int32_t value_storage, int32_t keep_f32, size_t *bytes)
{
    if (!bytes) return fail(SMX_EINVAL, "NULL argument");
    if (m < 1 || n < 1 || nnz < 0) return fail(SMX_EINVAL, "invalid shape");
    if (value_storage < SMX_STORE_F32 || value_storage > SMX_STORE_F16) return fail(SMX_EINVAL, "unknown storage");
    *bytes = operator_bound(m, n, nnz, value_storage != SMX_STORE_F32, value_storage == SMX_STORE_F32 || keep_f32, 0, 0);
    return SMX_OK;
}

int smx_footprint(int64_t m, int64_t n, int64_t nnz, int32_t value_storage, int32_t keep_f32, int32_t image_rows,
                  int32_t image_cols, const smx_problem_desc *desc, size_t *operator_bytes, size_t *problem_bytes)
{
    if (!operator_bytes || !problem_bytes) return fail(SMX_EINVAL, "NULL argument");
    if ((image_rows != 0 || image_cols != 0) && (image_rows < 1 || image_cols < 1 || (int64_t)image_rows * image_cols != n))
        return fail(SMX_EINVAL, "image %d x %d does not match n = %lld", image_rows, image_cols, (long long)n);
    SMX_GUARD({
        size_t ob = 0;
        if (const int rc = smx_operator_footprint(m, n, nnz, value_storage, keep_f32, &ob); rc != SMX_OK) return rc;
        if (image_rows > 0)
            ob = operator_bound(m, n, nnz, value_storage != SMX_STORE_F32, value_storage == SMX_STORE_F32 || keep_f32,
                                image_rows, image_cols);
        size_t pb = 0;
        if (desc) {
            const smx_problem_desc *d = desc;
            if (!(is_pow2(d->B) && d->B <= 32)) return fail(SMX_EINVAL, "B must be a power of two in 1..32 (got %d)", d->B);
            if (d->basic < SMX_BASIC_SIMULT || d->basic > SMX_BASIC_EMR)
                return fail(SMX_EINVAL, "unknown basic algorithm %d", d->basic);
            if (d->obj_kind < SMX_OBJ_NONE || d->obj_kind > SMX_OBJ_L1)
                return fail(SMX_EINVAL, "unknown objective %d", d->obj_kind);
            if (d->obj_kind != SMX_OBJ_NONE && (d->max_trials < 1 || d->max_trials > 1024))
                return fail(SMX_EINVAL, "max_trials must be in 1..1024 (got %d)", d->max_trials);
            if (d->obj_kind == SMX_OBJ_TV2D && (d->tv_rows < 1 || d->tv_cols < 1 || (int64_t)d->tv_rows * d->tv_cols != n))
                return fail(SMX_EINVAL, "TV image %d x %d does not match n = %lld", d->tv_rows, d->tv_cols, (long long)n);
            if (d->history_cap < 0) return fail(SMX_EINVAL, "history_cap must be >= 0");
            DvcTable dt{};
            if (const int rc = build_dvc_table(d, m, dt); rc != SMX_OK) return rc;
            const bool lp = value_storage != SMX_STORE_F32;
            const int lk = value_storage == SMX_STORE_BF16 ? VK_BF16 : (value_storage == SMX_STORE_F16 ? VK_F16 : VK_F32);
            pb = problem_plan_bytes(m, n, !lp || keep_f32 != 0, lk, d, dt);
        }
        *operator_bytes = ob;
        *problem_bytes = pb;
        return SMX_OK;
    })
}

int smx_problem_create(smx_operator *op, const smx_problem_desc *desc, void *stream, smx_problem **out)
{
    SMX_GUARD(return create_problem(op, desc, (hipStream_t)stream, out);)
}

int smx_problem_destroy(smx_problem *p)
{
    if (!p) return SMX_OK;
    SMX_GUARD({
        (void)hipStreamSynchronize(p->stream);
        smx_operator *op = p->op;
        delete p;
        release_operator(op);
        return SMX_OK;
    })
}

int smx_create(const smx_csr *A, int32_t value_storage, const smx_problem_desc *desc, void *stream, smx_problem **out)
{
    SMX_GUARD({
        if (!out) return fail(SMX_EINVAL, "NULL argument");
        smx_operator *op = nullptr;
        int rc = create_operator(A, value_storage, 1, (hipStream_t)stream, &op);
        if (rc != SMX_OK) return rc;
        rc = create_problem(op, desc, (hipStream_t)stream, out);
        release_operator(op); // the problem holds the remaining reference (or none on failure)
        return rc;
    })
}

int smx_set_stream(smx_problem *p, void *stream)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD({
        if ((hipStream_t)stream != p->stream) {
            hip_check(hipStreamSynchronize(p->stream), "sync old stream");
            p->stream = (hipStream_t)stream;
        }
        return SMX_OK;
    })
}

int smx_set_x(smx_problem *p, const float *x, int32_t on_device)
{
    if (!p || !x) return fail(SMX_EINVAL, "NULL argument");
    SMX_GUARD({
        hip_check(hipMemcpyAsync(p->x.p, x, sizeof(float) * p->n * p->B,
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->stream),
                  "set x");
        if (!on_device) hip_check(hipStreamSynchronize(p->stream), "set x");
        return SMX_OK;
    })
}

int smx_get_x(smx_problem *p, float *out, int32_t on_device)
{
    if (!p || !out) return fail(SMX_EINVAL, "NULL argument");
    SMX_GUARD({
        hip_check(hipMemcpyAsync(out, p->x.p, sizeof(float) * p->n * p->B,
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream),
                  "get x");
        if (!on_device) hip_check(hipStreamSynchronize(p->stream), "get x");
        return SMX_OK;
    })
}

int smx_run(smx_problem *p, int32_t K, uint32_t flags)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD(return run_impl(p, K, flags);)
}

int smx_sync(smx_problem *p)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD({
        hip_check(hipStreamSynchronize(p->stream), "sync");
        std::vector<SliceState> st(p->B);
        hip_check(hipMemcpy(st.data(), p->state(p->cur), sizeof(SliceState) * p->B, hipMemcpyDeviceToHost), "read state");
        bool bad = false;
        for (auto &S : st)
            if (S.nonfinite) bad = true;
        if (bad) {
            for (auto &S : st) S.nonfinite = 0;
            hip_check(hipMemcpy(p->state(p->cur), st.data(), sizeof(SliceState) * p->B, hipMemcpyHostToDevice), "clear flag");
            return fail(SMX_ENUMERIC, "a non-finite proximity or objective was produced");
        }
        return SMX_OK;
    })
}

int smx_query(smx_problem *p, double *proximity, double *objective)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD({
        const int B = p->B;
        const int vk = p->op->has_f32 ? VK_F32 : p->op->lp_kind();
        RowW qw = p->row_weights(vk); // the proximity terms D t^2 (c is scratch here)
        qw.S = qw.D;
        double *q = p->qout.as<double>();
        hip_check(launch_pass1(p->cfg1[vk], view_for(p->op, false, p->fmt1[vk]), p->op->csr.blocks(), p->fmt1[vk],
                               p->x.as<float>(), p->lower.as<float>(), p->upper.as<float>(), qw,
                               p->c.as<float>(),
                               p->state(p->cur), B, 1,
                               p->part_query.as<double>(), p->stream),
                  "query proximity");
        if (p->dvc.n > 0) p->enqueue_dvc(vk, p->part_query.as<double>(), p->cfg1[vk].grid, p->cur, 1, p->stream);
        hip_check(launch_query_prox(p->state(p->cur), B, p->part_query.as<double>(), p->cfg1[vk].grid, q,
                                    p->stream),
                  "query proximity");
        std::vector<double> h(2 * B, 0.0);
        if (p->pp.obj != OBJ_NONE) {
            hip_check(launch_phase(p->pp, p->x.as<float>(), p->g.as<float>(), p->lin_c.as<float>(),
                                   p->state(p->cur), 1, p->part_phase.as<double>(), p->stream),
                      "query objective");
            hip_check(launch_eval_objective(p->state(p->cur), p->pp, p->part_phase.as<double>(), q + B, p->stream),
                      "query objective");
            hip_check(hipMemcpyAsync(h.data(), q, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, p->stream), "query");
        } else {
            hip_check(hipMemcpyAsync(h.data(), q, sizeof(double) * B, hipMemcpyDeviceToHost, p->stream), "query");
        }
        hip_check(hipStreamSynchronize(p->stream), "query");
        for (int s = 0; s < B; ++s) {
            if (proximity) proximity[s] = h[s];
            if (objective) objective[s] = h[B + s];
        }
        return SMX_OK;
    })
}

int smx_get_history(smx_problem *p, double *prox, double *f_start, double *f_end, int32_t *trials, int32_t *accepts,
                    int32_t cap, int32_t *n_out)
{
    if (!p || !n_out) return fail(SMX_EINVAL, "NULL argument");
    if (cap < 0) return fail(SMX_EINVAL, "cap must be >= 0");
    SMX_GUARD({
        hip_check(hipStreamSynchronize(p->stream), "history");
        std::vector<SliceState> st(p->B);
        hip_check(hipMemcpy(st.data(), p->state(p->cur), sizeof(SliceState) * p->B, hipMemcpyDeviceToHost), "read state");
        long long kmax = 0;
        for (auto &S : st) kmax = std::max(kmax, S.k);
        const int64_t nrec = std::min<int64_t>({(int64_t)kmax, (int64_t)p->hist_cap, (int64_t)cap});
        const size_t cnt = size_t(nrec) * p->B;
        if (nrec > 0) {
            if (prox) hip_check(hipMemcpy(prox, p->h_prox.p, sizeof(double) * cnt, hipMemcpyDeviceToHost), "history");
            if (f_start) hip_check(hipMemcpy(f_start, p->h_fs.p, sizeof(double) * cnt, hipMemcpyDeviceToHost), "history");
            if (f_end) hip_check(hipMemcpy(f_end, p->h_fe.p, sizeof(double) * cnt, hipMemcpyDeviceToHost), "history");
            if (trials) hip_check(hipMemcpy(trials, p->h_tr.p, sizeof(int) * cnt, hipMemcpyDeviceToHost), "history");
            if (accepts) hip_check(hipMemcpy(accepts, p->h_ac.p, sizeof(int) * cnt, hipMemcpyDeviceToHost), "history");
        }
        *n_out = (int32_t)nrec;
        return SMX_OK;
    })
}

int smx_get_state(smx_problem *p, smx_slice_state *states, float *x)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD({
        hip_check(hipStreamSynchronize(p->stream), "state");
        std::vector<SliceState> st(p->B);
        hip_check(hipMemcpy(st.data(), p->state(p->cur), sizeof(SliceState) * p->B, hipMemcpyDeviceToHost), "read state");
        if (states)
            for (int s = 0; s < p->B; ++s) {
                states[s].k = st[s].k;
                states[s].ell = st[s].ell;
                states[s].restarts = st[s].restarts;
                states[s].trials = st[s].trials;
                states[s].accepts = st[s].accepts;
                states[s].cap_hits = st[s].cap_hits;
                states[s].stop_reason = st[s].stop_reason;
                states[s].dp_run = st[s].dp_run;
                states[s].feas_ok = st[s].feas_ok;
                states[s].reserved = 0;
                states[s].p_last = st[s].p_last;
                states[s].f_last = st[s].f_last;
                states[s].var_n = st[s].var_n;
                states[s].var_mean = st[s].var_mean;
                states[s].var_m2 = st[s].var_m2;
                states[s].f_ref = st[s].f_ref;
            }
        if (x) hip_check(hipMemcpy(x, p->x.p, sizeof(float) * p->n * p->B, hipMemcpyDeviceToHost), "read x");
        return SMX_OK;
    })
}

int smx_set_state(smx_problem *p, const smx_slice_state *states, const float *x)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD({
        hip_check(hipStreamSynchronize(p->stream), "state");
        if (states) {
            for (int s = 0; s < p->B; ++s)
                if (states[s].k < 0 || states[s].ell < 0 || states[s].restarts < 0 || states[s].dp_run < 0 ||
                    states[s].stop_reason < SMX_STOP_NONE || states[s].stop_reason > SMX_STOP_SM)
                    return fail(SMX_EINVAL, "invalid counter in state of slice %d", s);
            std::vector<SliceState> st(p->B);
            hip_check(hipMemcpy(st.data(), p->state(p->cur), sizeof(SliceState) * p->B, hipMemcpyDeviceToHost), "read state");
            for (int s = 0; s < p->B; ++s) {
                st[s].k = states[s].k;
                st[s].ell = states[s].ell;
                st[s].restarts = states[s].restarts;
                st[s].trials = states[s].trials;
                st[s].accepts = states[s].accepts;
                st[s].cap_hits = states[s].cap_hits;
                st[s].stop_reason = states[s].stop_reason;
                st[s].dp_run = states[s].dp_run;
                st[s].feas_ok = states[s].feas_ok;
                st[s].p_last = states[s].p_last;
                st[s].f_last = states[s].f_last;
                st[s].var_n = states[s].var_n;
                st[s].var_mean = states[s].var_mean;
                st[s].var_m2 = states[s].var_m2;
                st[s].f_ref = states[s].f_ref;
                st[s].phase = 0;
                st[s].live = (st[s].enabled && st[s].k < st[s].k_end && st[s].stop_reason == STOP_NONE) ? 1 : 0;
            }
            hip_check(hipMemcpy(p->state(p->cur), st.data(), sizeof(SliceState) * p->B, hipMemcpyHostToDevice), "write state");
        }
        if (x) hip_check(hipMemcpy(p->x.p, x, sizeof(float) * p->n * p->B, hipMemcpyHostToDevice), "write x");
        return SMX_OK;
    })
}

int smx_problem_dims(const smx_problem *p, int64_t *m, int64_t *n, int64_t *nnz, int32_t *B)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    if (m) *m = p->m;
    if (n) *n = p->n;
    if (nnz) *nnz = p->op->nnz;
    if (B) *B = p->B;
    return SMX_OK;
}

int smx_autotune(smx_problem *p, int32_t reps)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD(return autotune_impl(p, reps);)
}

int smx_describe(const smx_problem *p, char *buf, size_t cap, size_t *need)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD(return describe_impl(p, buf, cap, need);)
}

int smx_slot_load(smx_problem *p, int32_t slot, const float *lower, const float *upper, const float *x0,
                  int32_t on_device, int64_t budget)
{
    if (!p || !lower || !upper || !x0) return fail(SMX_EINVAL, "NULL argument");
    if (slot < 0 || slot >= p->B) return fail(SMX_EINVAL, "slot %d outside [0, %d)", slot, p->B);
    if (budget < 0) return fail(SMX_EINVAL, "budget must be >= 0");
    SMX_GUARD({
        const int64_t m = p->m, n = p->n;
        std::vector<float> lo = fetch(lower, m, on_device != 0), up = fetch(upper, m, on_device != 0);
        for (int64_t i = 0; i < m; ++i) {
            if (std::isnan(lo[i]) || std::isnan(up[i])) return fail(SMX_EINVAL, "NaN bound at %lld", (long long)i);
            if (lo[i] > up[i]) return fail(SMX_EINVAL, "lower > upper at %lld", (long long)i);
        }
        std::vector<float> xs = fetch(x0, n, on_device != 0);
        DBuf tmp;
        tmp.alloc(sizeof(float) * std::max(m, n), "slot staging");
        hipStream_t s = p->stream;
        hip_check(hipMemcpyAsync(tmp.p, lo.data(), sizeof(float) * m, hipMemcpyHostToDevice, s), "slot bounds");
        hip_check(launch_put_column(p->lower.as<float>(), tmp.as<float>(), m, p->B, slot, s), "slot bounds");
        hip_check(hipMemcpyAsync(tmp.p, up.data(), sizeof(float) * m, hipMemcpyHostToDevice, s), "slot bounds");
        hip_check(launch_put_column(p->upper.as<float>(), tmp.as<float>(), m, p->B, slot, s), "slot bounds");
        hip_check(hipMemcpyAsync(tmp.p, xs.data(), sizeof(float) * n, hipMemcpyHostToDevice, s), "slot x0");
        hip_check(launch_put_column(p->x.as<float>(), tmp.as<float>(), n, p->B, slot, s), "slot x0");
        hip_check(launch_reset_slot(p->state(p->cur), slot, budget, s), "slot reset");
        hip_check(hipStreamSynchronize(s), "slot load");
        return SMX_OK;
    })
}

int smx_slot_load_noalloc(smx_problem *p, int32_t slot, const float *lower, const float *upper, const float *x0,
                          int32_t on_device, int64_t budget)
{
    if (!p || !lower || !upper || !x0) return fail(SMX_EINVAL, "NULL argument");
    if (slot < 0 || slot >= p->B) return fail(SMX_EINVAL, "slot %d outside [0, %d)", slot, p->B);
    if (budget < 0) return fail(SMX_EINVAL, "budget must be >= 0");
    const int64_t m = p->m, n = p->n;
    // staging: [check flags][lower m][upper m][x0 n], each part 256-byte aligned
    const size_t off_lo = kScratchHead, off_up = off_lo + size_t(round_up(m * 4, 256)),
                 off_x = off_up + size_t(round_up(m * 4, 256)), need = off_x + size_t(round_up(n * 4, 256));
    if (need > kScratchBytes)
        return fail(SMX_EINVAL, "slot of %lld rows and %lld columns needs %zu bytes of staging; the static scratch "
                    "holds %zu (2m + n up to about %zu floats)", (long long)m, (long long)n, need, kScratchBytes,
                    (kScratchBytes - kScratchHead) / 4);
    SMX_GUARD({
        unsigned char *base = static_cast<unsigned char *>(scratch_on_current_device());
        float *slo = reinterpret_cast<float *>(base + off_lo), *sup = reinterpret_cast<float *>(base + off_up),
              *sx = reinterpret_cast<float *>(base + off_x);
        unsigned *flag = reinterpret_cast<unsigned *>(base);
        hipStream_t s = p->stream;
        const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        hip_check(hipMemcpyAsync(slo, lower, sizeof(float) * m, kind, s), "slot bounds");
        hip_check(hipMemcpyAsync(sup, upper, sizeof(float) * m, kind, s), "slot bounds");
        hip_check(hipMemcpyAsync(sx, x0, sizeof(float) * n, kind, s), "slot x0");
        hip_check(launch_check_bands(slo, sup, m, flag, s), "slot bounds check");
        unsigned h[2] = {0u, 0u};
        hip_check(hipMemcpyAsync(h, flag, sizeof h, hipMemcpyDeviceToHost, s), "slot bounds check");
        hip_check(hipStreamSynchronize(s), "slot bounds check");
        if (h[0] & 1u) return fail(SMX_EINVAL, "NaN bound at %u", h[1]);
        if (h[0] & 2u) return fail(SMX_EINVAL, "lower > upper at %u", h[1]);
        hip_check(launch_put_column(p->lower.as<float>(), slo, m, p->B, slot, s), "slot bounds");
        hip_check(launch_put_column(p->upper.as<float>(), sup, m, p->B, slot, s), "slot bounds");
        hip_check(launch_put_column(p->x.as<float>(), sx, n, p->B, slot, s), "slot x0");
        hip_check(launch_reset_slot(p->state(p->cur), slot, budget, s), "slot reset");
        hip_check(hipStreamSynchronize(s), "slot load");
        return SMX_OK;
    })
}

int smx_slot_disable(smx_problem *p, int32_t slot)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    if (slot < 0 || slot >= p->B) return fail(SMX_EINVAL, "slot %d outside [0, %d)", slot, p->B);
    SMX_GUARD({
        hip_check(launch_disable_slot(p->state(p->cur), slot, p->stream), "slot disable");
        return SMX_OK;
    })
}

int smx_slot_status(smx_problem *p, int64_t *k, int32_t *live)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    SMX_GUARD({
        hip_check(hipStreamSynchronize(p->stream), "slot status");
        std::vector<SliceState> st(p->B);
        hip_check(hipMemcpy(st.data(), p->state(p->cur), sizeof(SliceState) * p->B, hipMemcpyDeviceToHost), "state");
        for (int s = 0; s < p->B; ++s) {
            if (k) k[s] = st[s].k;
            if (live) live[s] = st[s].live;
        }
        return SMX_OK;
    })
}

int smx_slot_get_x(smx_problem *p, int32_t slot, float *out, int32_t on_device)
{
    if (!p || !out) return fail(SMX_EINVAL, "NULL argument");
    if (slot < 0 || slot >= p->B) return fail(SMX_EINVAL, "slot %d outside [0, %d)", slot, p->B);
    SMX_GUARD({
        if (on_device) {
            hip_check(launch_get_column(out, p->x.as<float>(), p->n, p->B, slot, p->stream), "slot x");
            return SMX_OK;
        }
        DBuf tmp;
        tmp.alloc(sizeof(float) * p->n, "slot staging");
        hip_check(launch_get_column(tmp.as<float>(), p->x.as<float>(), p->n, p->B, slot, p->stream), "slot x");
        hip_check(hipMemcpyAsync(out, tmp.p, sizeof(float) * p->n, hipMemcpyDeviceToHost, p->stream), "slot x");
        hip_check(hipStreamSynchronize(p->stream), "slot x");
        return SMX_OK;
    })
}

int smx_set_fused(smx_problem *p, int32_t mode)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    if (mode != 0 && mode != 1) return fail(SMX_EINVAL, "fused mode must be 0 or 1 (got %d)", mode);
    SMX_GUARD({
        p->fused_mode = mode;
        for (int vk = 0; vk < 3; ++vk) p->fused[vk] = p->fused_ok[vk] && mode == 1;
        // the kernel choice is baked into captured graphs
        hip_check(hipStreamSynchronize(p->stream), "sync");
        for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
        p->graphs.clear();
        return SMX_OK;
    })
}

int smx_set_phase_form(smx_problem *p, int32_t form)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    if (form < SMX_PHASE_AUTO || form > SMX_PHASE_CLOSED_FORM)
        return fail(SMX_EINVAL, "phase form must be SMX_PHASE_AUTO, _ONE_LAUNCH, _BATCHES or _CLOSED_FORM (got %d)",
                    form);
    SMX_GUARD({
        if (form == SMX_PHASE_ONE_LAUNCH && !phase_in_one_launch(p->pp))
            return fail(SMX_ESTATE, "the one-launch phase takes the squared-norm, L1 and linear objectives with "
                                    "n <= %d (objective %d, n = %lld)",
                        kSmallPhaseMaxN, p->pp.obj, (long long)p->n);
        if (form == SMX_PHASE_CLOSED_FORM && p->pp.obj != OBJ_LINEAR)
            return fail(SMX_ESTATE, "trials in closed form need the linear objective (objective %d)", p->pp.obj);
        p->phase_form = form;
        // the launch sequence is baked into captured graphs
        hip_check(hipStreamSynchronize(p->stream), "sync");
        for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
        p->graphs.clear();
        return SMX_OK;
    })
}

int smx_set_fused_shape(smx_problem *p, int32_t lpr, int32_t vec, int32_t cap, int32_t z_in_lds)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    if (z_in_lds < 0 || z_in_lds > 1) return fail(SMX_EINVAL, "z_in_lds must be 0 or 1 (got %d)", z_in_lds);
    SMX_GUARD({
        bool any = false;
        for (int vk = 0; vk < 3; ++vk) any = any || p->fused_ok[vk];
        if (!any) return fail(SMX_ESTATE, "this problem has no fused pass");
        bool found = false;
        for (int vk = 0; vk < 3; ++vk) {
            if (!p->fused_ok[vk]) continue;
            for (const FusedCfg &c : fused_candidates(p->fcfg[vk], p->n, p->dvc.n > 0))
                if (c.lpr == lpr && c.vec == vec && c.cap == cap && c.zl == z_in_lds) {
                    p->fcfg[vk] = c;
                    found = true;
                }
        }
        if (!found)
            return fail(SMX_EINVAL, "unsupported fused shape lpr %d vec %d cap %d z_in_lds %d", lpr, vec, cap, z_in_lds);
        hip_check(hipStreamSynchronize(p->stream), "sync");
        for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
        p->graphs.clear();
        return SMX_OK;
    })
}

int smx_stop_status(smx_problem *p, int32_t *reason)
{
    if (!p || !reason) return fail(SMX_EINVAL, "NULL argument");
    SMX_GUARD({
        hip_check(hipStreamSynchronize(p->stream), "state");
        std::vector<SliceState> st(p->B);
        hip_check(hipMemcpy(st.data(), p->state(p->cur), sizeof(SliceState) * p->B, hipMemcpyDeviceToHost),
                  "read state");
        for (int s = 0; s < p->B; ++s) reason[s] = st[s].stop_reason;
        return SMX_OK;
    })
}

int smx_set_timing(smx_problem *p, int32_t enable)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    p->timing = enable != 0;
    return SMX_OK;
}

int smx_get_timing(smx_problem *p, double *pass1_ms, double *pass2_ms, int64_t *launches)
{
    if (!p) return fail(SMX_EINVAL, "NULL problem");
    const int64_t L = p->t_launches;
    if (pass1_ms) *pass1_ms = L ? p->t1_ms / L : 0.0;
    if (pass2_ms) *pass2_ms = L ? p->t2_ms / L : 0.0;
    if (launches) *launches = L;
    return SMX_OK;
}

} // extern "C"
