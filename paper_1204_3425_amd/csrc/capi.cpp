// C ABI of the Hubbard library: argument checks, handle life cycle, and the
// Lanczos driver (Siro & Harju, Sec. 2.2, Alg. 1 in its two-vector form).
//
// Driver.  Two device vectors C and P hold s_c f_j and s_p f_{j-1}; the scale
// factors live in a small block of device scalars, so no host round trip is
// needed between steps.  Step j:
//     P <- (1/s_c) H C - (b_j / s_p) P        = q_j       (one fused H.v kernel)
//     a_j = (P . C) / s_c                                  (fixed-order reduction)
//     P <- P - (a_j / s_c) C                   = q_j - a_j f_j
//     b_{j+1} = |P|                                        (fixed-order reduction)
// after which P holds b_{j+1} f_{j+1}: the two vectors swap roles.  This is
// the paper's split of the three-term recurrence into an in-place update of
// f_{j-1} (eq. split1), with the 1/b_{j+1} normalisation folded into the next
// H.v instead of a separate pass.  The host reads (a_j, b_{j+1}) a few steps
// behind the device, computes the lowest eigenvalue of T_j (eq. Tmatrix) and
// applies the energy test of Sec. 2.2.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "batch.h"
#include "internal.h"

namespace hub {

static thread_local std::string g_last_error;

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        fail(HUBBARD_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
    fail(HUBBARD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
static int guarded(F &&f)
{
    try {
        g_last_error.clear();
        return f();
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return HUBBARD_ENOMEM;
    } catch (...) {
        g_last_error = "unexpected internal error";
        return HUBBARD_EDEVICE;
    }
}

// Device buffer owned by RAII.
struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t bytes)
    {
        if (bytes)
            HUB_HIP(hipMalloc(&p, bytes));
    }
    ~DevBuf()
    {
        if (p)
            (void)hipFree(p);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Pinned host memory, mapped and coherent: kernels may write it directly
// (through dev), and the host reads it once the writing work has completed.
struct PinnedBuf {
    void *p = nullptr;
    void *dev = nullptr;
    explicit PinnedBuf(size_t bytes)
    {
        HUB_HIP(hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocCoherent));
        HUB_HIP(hipHostGetDevicePointer(&dev, p, 0));
    }
    ~PinnedBuf()
    {
        if (p)
            (void)hipHostFree(p);
    }
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

static void free_device(hubbard *h)
{
    if (h->apply_work) {
        (void)hipFree(h->apply_work);
        h->apply_work = nullptr;
        h->apply_work_bytes = 0;
    }
    if (h->apply_ev) {
        (void)hipEventDestroy(h->apply_ev);
        h->apply_ev = nullptr;
    }
    DeviceTables &d = h->dev;
    void *ptrs[] = {d.states_up, d.states_dn, d.up_rows, d.dn_cols, d.nnz_up, d.nnz_dn,
                    d.dn_groups64, d.dn_groups32, d.dn_nq, d.dn_groups16, d.dn_nq8, d.dn_pidx, d.dn_nidx, d.dn_pn, d.up_blk, d.up_nint, d.up_next,
                    d.up_bstart, d.up_line, d.up_cnt, d.tcls};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    d = DeviceTables();
}

template <typename T>
static T *upload(const void *src, size_t bytes, size_t &total)
{
    void *p = nullptr;
    HUB_HIP(hipMalloc(&p, bytes ? bytes : 16));
    if (bytes)
        HUB_HIP(hipMemcpy(p, src, bytes, hipMemcpyHostToDevice));
    total += bytes;
    return static_cast<T *>(p);
}

// Blocks of up configurations for the blocked slab pass: the largest number p
// of low sites such that rows sharing the occupation of sites p.. form blocks
// of at most kMaxBlockRows rows (configurations in ascending order keep each
// block contiguous).
constexpr int kMaxBlockRows = 1024;

static void upload_blocked_up(hubbard *h, size_t &total)
{
    DeviceTables &d = h->dev;
    const SpinTable &up = h->up;
    const int64_t du = up.dim;
    std::vector<int32_t> bstart;
    for (int p = h->sites; p >= 0; p--) {
        bstart.assign(1, 0);
        int64_t longest = 0, run = 1;
        auto key = [&](int64_t r) { return p >= 32 ? 0u : up.states[(size_t)r] >> p; };
        for (int64_t r = 1; r < du; r++) {
            if (key(r) != key(r - 1)) {
                bstart.push_back((int32_t)r);
                longest = std::max(longest, run);
                run = 1;
            } else {
                run++;
            }
        }
        longest = std::max(longest, run);
        bstart.push_back((int32_t)du);
        if (longest <= kMaxBlockRows)
            break;
    }
    const int nb = (int)bstart.size() - 1;
    std::vector<int32_t> blk_of((size_t)du);
    int longest = 0;
    for (int b = 0; b < nb; b++) {
        longest = std::max(longest, bstart[(size_t)b + 1] - bstart[(size_t)b]);
        for (int32_t r = bstart[(size_t)b]; r < bstart[(size_t)b + 1]; r++)
            blk_of[(size_t)r] = b;
    }
    const int w = std::max(1, up.width);
    std::vector<uint32_t> ent((size_t)du * (size_t)w, 0u);
    std::vector<uint16_t> nint((size_t)du), next((size_t)du);
    for (int64_t r = 0; r < du; r++) {
        const int b = blk_of[(size_t)r];
        size_t o = (size_t)r * (size_t)w;
        int ni = 0, ne = 0;
        for (int pass = 0; pass < 2; pass++)
            for (int k = 0; k < up.row_nnz[(size_t)r]; k++) {
                const size_t src = (size_t)k * (size_t)du + (size_t)r;
                const int32_t c = up.col[src];
                const bool inside = blk_of[(size_t)c] == b;
                if (inside != (pass == 0))
                    continue;
                const uint32_t sg = up.sgn[src] < 0 ? 0x80000000u : 0u;
                // per-bond handles: the amplitude class in bits 24..25 (rows below 2^24)
                const uint32_t cls = h->tcls.empty() ? 0u : (uint32_t)h->bond_cls[up.bond[src]] << 24;
                ent[o++] = (uint32_t)(inside ? c - bstart[(size_t)b] : c) | cls | sg;
                (inside ? ni : ne)++;
            }
        nint[(size_t)r] = (uint16_t)ni;
        next[(size_t)r] = (uint16_t)ne;
    }
    if (up.width <= 64) {
        // per row group of eight (block rows 8g..8g+7, the rows one wave step
        // of the line kernel takes): the largest internal and external counts
        std::vector<uint8_t> gmi((size_t)du), gme((size_t)du);
        for (int b = 0; b < nb; b++)
            for (int32_t g0 = bstart[(size_t)b]; g0 < bstart[(size_t)b + 1]; g0 += 8) {
                const int32_t g1 = std::min(g0 + 8, bstart[(size_t)b + 1]);
                int mi = 0, me = 0;
                for (int32_t r = g0; r < g1; r++) {
                    mi = std::max<int>(mi, nint[(size_t)r]);
                    me = std::max<int>(me, next[(size_t)r]);
                }
                for (int32_t r = g0; r < g1; r++) {
                    gmi[(size_t)r] = (uint8_t)mi;
                    gme[(size_t)r] = (uint8_t)me;
                }
            }
        // room to pad: the group's largest internal count and the row's own
        // external entries must share the row's slots
        auto pads = [&](int W) {
            for (int64_t r = 0; r < du; r++)
                if (gmi[(size_t)r] + next[(size_t)r] > W)
                    return false;
            return true;
        };
        // one 128-byte line of 32 slots per row, or two (64 slots) for rows of
        // 33 to 64 hops or where one line has no room for the padding
        const int W = up.width <= 32 && pads(32) ? 32 : 64;
        const bool ipad = pads(W);
        std::vector<uint32_t> line((size_t)du * (size_t)W, 0u), cnt((size_t)du);
        for (int64_t r = 0; r < du; r++) {
            const size_t o = (size_t)r * (size_t)w;
            const int ni = nint[(size_t)r], ne = next[(size_t)r];
            const int b = blk_of[(size_t)r];
            for (int k = 0; k < ni; k++)
                line[(size_t)r * W + (size_t)k] = ent[o + (size_t)k];
            if (ipad)
                for (int k = ni; k < gmi[(size_t)r]; k++)
                    line[(size_t)r * W + (size_t)k] = (uint32_t)(bstart[(size_t)b + 1] - bstart[(size_t)b]);
            for (int k = 0; k < ne; k++)
                line[(size_t)r * W + (size_t)(W - 1 - k)] = ent[o + (size_t)(ni + k)];
            cnt[(size_t)r] = (uint32_t)ni | ((uint32_t)ne << 8) | ((uint32_t)gmi[(size_t)r] << 16) |
                             ((uint32_t)gme[(size_t)r] << 24);
        }
        d.up_line = upload<uint32_t>(line.data(), line.size() * 4, total);
        d.up_cnt = upload<uint32_t>(cnt.data(), cnt.size() * 4, total);
        d.up_line_w = W;
        d.up_line_ipad = ipad ? 1 : 0;
    }
    d.up_blk = upload<uint32_t>(ent.data(), ent.size() * 4, total);
    d.up_nint = upload<uint16_t>(nint.data(), nint.size() * 2, total);
    d.up_next = upload<uint16_t>(next.data(), next.size() * 2, total);
    d.up_bstart = upload<int32_t>(bstart.data(), bstart.size() * 4, total);
    d.up_nblocks = nb;
    d.up_max_block = longest;
}

static void upload_tables(hubbard *h)
{
    DeviceTables &d = h->dev;
    size_t total = 0;
    d.states_up = upload<uint32_t>(h->up.states.data(), h->up.states.size() * 4, total);
    d.states_dn = upload<uint32_t>(h->dn.states.data(), h->dn.states.size() * 4, total);
    // per-bond amplitudes: entries carry the amplitude class of their bond
    const bool gen = !h->tcls.empty();
    auto pack = [&](const SpinTable &tb, size_t src) {
        return gen ? pack_entry_class(tb.col[src], tb.sgn[src], h->bond_cls[tb.bond[src]])
                   : pack_entry(tb.col[src], tb.sgn[src]);
    };
    // up table row-major (one row's entries are read by a whole workgroup)
    std::vector<uint32_t> rows((size_t)h->up.dim * (size_t)std::max(1, h->up.width), 0u);
    for (int64_t r = 0; r < h->up.dim; r++)
        for (int k = 0; k < h->up.row_nnz[(size_t)r]; k++) {
            size_t src = (size_t)k * (size_t)h->up.dim + (size_t)r;
            rows[(size_t)r * (size_t)h->up.width + (size_t)k] = pack(h->up, src);
        }
    d.up_rows = upload<uint32_t>(rows.data(), rows.size() * 4, total);
    // down table column-major (lanes of a wave read consecutive rows d)
    std::vector<uint32_t> cols((size_t)h->dn.dim * (size_t)std::max(1, h->dn.width), 0u);
    for (int64_t r = 0; r < h->dn.dim; r++)
        for (int k = 0; k < h->dn.row_nnz[(size_t)r]; k++) {
            size_t src = (size_t)k * (size_t)h->dn.dim + (size_t)r;
            cols[src] = pack(h->dn, src);
        }
    d.dn_cols = upload<uint32_t>(cols.data(), cols.size() * 4, total);
    d.nnz_up = upload<uint16_t>(h->up.row_nnz.data(), h->up.row_nnz.size() * 2, total);
    d.nnz_dn = upload<uint16_t>(h->dn.row_nnz.data(), h->dn.row_nnz.size() * 2, total);
    if (gen) {
        d.tcls = upload<double>(h->tcls.data(), h->tcls.size() * 8, total);
        if ((int)h->tcls.size() > kTwoPassClasses) {
            // only the one-pass kernel reads this many classes
            d.bytes = total;
            return;
        }
    }
    // class bits of an entry of the down table (per-bond handles)
    auto dn_cls = [&](size_t src) -> uint32_t { return gen ? (uint32_t)h->bond_cls[h->dn.bond[src]] : 0u; };
    // row-pass groups: entry k of column d at ((k/4) * dim_dn + d) * 4 + k%4
    const int64_t ddn = h->dn.dim;
    const int ng = (h->dn.width + 3) / 4;
    d.dn_ngroups = ng;
    std::vector<uint8_t> nq((size_t)((ddn + 63) / 64), 0);
    for (int64_t r = 0; r < ddn; r++) {
        int need = (h->dn.row_nnz[(size_t)r] + 3) / 4;
        uint8_t &slot = nq[(size_t)(r / 64)];
        slot = (uint8_t)std::max<int>(slot, need);
    }
    for (int es : {8, 4}) {
        std::vector<uint32_t> g((size_t)std::max(ng, 1) * (size_t)ddn * 4, (uint32_t)(ddn * es));
        for (int64_t r = 0; r < ddn; r++)
            for (int k = 0; k < h->dn.row_nnz[(size_t)r]; k++) {
                size_t src = (size_t)k * (size_t)ddn + (size_t)r;
                uint32_t off = (uint32_t)h->dn.col[src] * (uint32_t)es;
                // classes sit above the offset (bits 18..19): offsets of the rows
                // the two-pass plan stages in LDS stay below 2^18
                if (gen && off < (1u << 18))
                    off |= dn_cls(src) << 18;
                g[((size_t)(k / 4) * (size_t)ddn + (size_t)r) * 4 + (size_t)(k % 4)] =
                    off | (h->dn.sgn[src] < 0 ? 0x80000000u : 0u);
            }
        uint32_t *dev = upload<uint32_t>(g.data(), g.size() * 4, total);
        (es == 8 ? d.dn_groups64 : d.dn_groups32) = dev;
    }
    d.dn_nq = upload<uint8_t>(nq.data(), nq.size(), total);
    if (ddn < 32768 && !gen) {
        // entry k of column d at ((k/8) * dim_dn + d) * 8 + k%8; padding = the zero slot's index
        const int ng8 = (h->dn.width + 7) / 8;
        std::vector<uint16_t> g((size_t)std::max(ng8, 1) * (size_t)ddn * 8, (uint16_t)ddn);
        // padded to whole 32-bit words (the FP64 row pass reads it by words)
        std::vector<uint8_t> nq8((size_t)((ddn + 255) / 256) * 4, 0);
        for (int64_t r = 0; r < ddn; r++) {
            const int nnz = h->dn.row_nnz[(size_t)r];
            for (int k = 0; k < nnz; k++) {
                size_t src = (size_t)k * (size_t)ddn + (size_t)r;
                g[((size_t)(k / 8) * (size_t)ddn + (size_t)r) * 8 + (size_t)(k % 8)] =
                    (uint16_t)((uint32_t)h->dn.col[src] | (h->dn.sgn[src] < 0 ? 0x8000u : 0u));
            }
            uint8_t &slot = nq8[(size_t)(r / 64)];
            slot = (uint8_t)std::max<int>(slot, (nnz + 7) / 8);
        }
        d.dn_groups16 = upload<uint16_t>(g.data(), g.size() * 2, total);
        d.dn_nq8 = upload<uint8_t>(nq8.data(), nq8.size(), total);
        if (ddn <= kRow64Max) {
            // the FP64 row pass: per column the + hops in groups of eight and
            // the - hops in groups of four (ascending column order within each)
            const int64_t nchunk = (ddn + 63) / 64;
            std::vector<int> np_col((size_t)ddn), nn_col((size_t)ddn);
            int npm = 1, nnm = 1;
            for (int64_t r = 0; r < ddn; r++) {
                int cp = 0, cn = 0;
                for (int k = 0; k < h->dn.row_nnz[(size_t)r]; k++)
                    (h->dn.sgn[(size_t)k * (size_t)ddn + (size_t)r] < 0 ? cn : cp)++;
                np_col[(size_t)r] = (cp + 7) / 8;
                nn_col[(size_t)r] = (cn + 3) / 4;
                npm = std::max(npm, np_col[(size_t)r]);
                nnm = std::max(nnm, nn_col[(size_t)r]);
            }
            std::vector<uint16_t> pi((size_t)npm * (size_t)ddn * 8, (uint16_t)ddn);
            std::vector<uint16_t> ni((size_t)nnm * (size_t)ddn * 4, (uint16_t)ddn);
            std::vector<uint8_t> pn((size_t)nchunk * 2, 0);
            for (int64_t r = 0; r < ddn; r++) {
                int cp = 0, cn = 0;
                for (int k = 0; k < h->dn.row_nnz[(size_t)r]; k++) {
                    const size_t src = (size_t)k * (size_t)ddn + (size_t)r;
                    const uint16_t c = (uint16_t)h->dn.col[src];
                    if (h->dn.sgn[src] < 0) {
                        ni[((size_t)(cn / 4) * (size_t)ddn + (size_t)r) * 4 + (size_t)(cn % 4)] = c;
                        cn++;
                    } else {
                        pi[((size_t)(cp / 8) * (size_t)ddn + (size_t)r) * 8 + (size_t)(cp % 8)] = c;
                        cp++;
                    }
                }
                uint8_t *slot = &pn[(size_t)(r / 64) * 2];
                slot[0] = (uint8_t)std::max<int>(slot[0], np_col[(size_t)r]);
                slot[1] = (uint8_t)std::max<int>(slot[1], nn_col[(size_t)r]);
            }
            d.dn_pidx = upload<uint16_t>(pi.data(), pi.size() * 2, total);
            d.dn_nidx = upload<uint16_t>(ni.data(), ni.size() * 2, total);
            d.dn_pn = upload<uint8_t>(pn.data(), pn.size(), total);
            d.dn_np = npm;
            d.dn_nn = nnm;
        }
    }
    upload_blocked_up(h, total);
    d.bytes = total;
}

static HvArgs hv_args(const hubbard *h)
{
    HvArgs a;
    // per-bond handles: the device amplitudes; without a device only the plan
    // reads this pointer, as the flag that selects the one-pass form
    a.tcls = h->dev.tcls ? h->dev.tcls : (h->tcls.empty() ? nullptr : h->tcls.data());
    a.ncls = (int)h->tcls.size();
    for (int c = 0; c < a.ncls && c < 4; c++)
        a.amp4[c] = h->tcls[(size_t)c];
    a.states_up = h->dev.states_up;
    a.states_dn = h->dev.states_dn;
    a.up_rows = h->dev.up_rows;
    a.dn_cols = h->dev.dn_cols;
    a.nnz_up = h->dev.nnz_up;
    a.nnz_dn = h->dev.nnz_dn;
    a.dn_groups64 = reinterpret_cast<const uint4 *>(h->dev.dn_groups64);
    a.dn_groups32 = reinterpret_cast<const uint4 *>(h->dev.dn_groups32);
    a.dn_nq = h->dev.dn_nq;
    a.dn_ngroups = h->dev.dn_ngroups;
    a.dn_groups16 = reinterpret_cast<const uint4 *>(h->dev.dn_groups16);
    a.dn_nq8 = h->dev.dn_nq8;
    a.dn_pidx = reinterpret_cast<const uint4 *>(h->dev.dn_pidx);
    a.dn_nidx = reinterpret_cast<const uint2 *>(h->dev.dn_nidx);
    a.dn_pn = h->dev.dn_pn;
    a.dn_np = h->dev.dn_np;
    a.dn_nn = h->dev.dn_nn;
    a.up_blk = h->dev.up_blk;
    a.up_nint = h->dev.up_nint;
    a.up_next = h->dev.up_next;
    a.up_bstart = h->dev.up_bstart;
    a.up_nblocks = h->dev.up_nblocks;
    a.up_max_block = h->dev.up_max_block;
    a.up_line = h->dev.up_line;
    a.up_line_w = h->dev.up_line_w;
    a.up_line_ipad = h->dev.up_line_ipad;
    a.up_cnt = h->dev.up_cnt;
    a.dim_up = h->up.dim;
    a.dim_dn = h->dn.dim;
    a.w_up = h->up.width;
    a.w_dn = h->dn.width;
    a.t = h->t;
    a.U = h->U;
    return a;
}

static void check_handle(hubbard_h h)
{
    if (!h)
        fail(HUBBARD_EINVAL, "null handle");
}

static void use_device(const hubbard *h)
{
    if (h->device < 0)
        fail(HUBBARD_EDEVICE, "no HIP device was present when the handle was built");
    HUB_HIP(hipSetDevice(h->device));
}

// ------------------------------------------------------------------ Lanczos

struct LanczosOut {
    std::vector<double> a, b, e;  // a_j, b_{j+1}, lowest eigenvalue of T_j
    int m = 0;
    int stop = HUBBARD_STOP_MAXITER;
    double e0 = 0, residual = -1, rayleigh = NAN;
    double seconds_first = 0;
    bool psi_resident = false;  // psi came from the resident vectors, not a replay
};

// sectors from this size on take the fused Lanczos step
constexpr int64_t kFusedMinDim = 1 << 16;

// Slots for a resident Lanczos basis, allocated in chunks of kBasisChunk
// vectors as a run needs them and reusable by the next run of the same call.
constexpr size_t kBasisChunk = 32;
struct BasisPool {
    std::vector<std::unique_ptr<DevBuf>> chunks;
    size_t vb = 0;  // bytes per vector
    // the padding of the rows (bytes pad_off..pitch of each row, rows per vector):
    // zeroed when a chunk is allocated, since the kernels write only the row
    // elements and the fix-up of a flagged fused step reads whole padded rows
    size_t pitch = 0, pad_off = 0;
    int64_t rows = 0;
    size_t capacity() const { return chunks.size() * kBasisChunk; }
    void *slot(size_t j) const { return static_cast<char *>(chunks[j / kBasisChunk]->p) + (j % kBasisChunk) * vb; }
    // room for vector j within budget (bytes the pool may hold in total); false when it cannot grow
    bool reserve(size_t j, size_t budget, hipStream_t s)
    {
        while (j >= capacity()) {
            if ((chunks.size() + 1) * kBasisChunk * vb > budget)
                return false;
            try {
                chunks.emplace_back(new DevBuf(kBasisChunk * vb));
            } catch (const Error &) {
                (void)hipGetLastError();
                return false;
            }
            if (pitch > pad_off)
                HUB_HIP(hipMemset2DAsync(static_cast<char *>(chunks.back()->p) + pad_off, pitch, 0, pitch - pad_off,
                                         (size_t)rows * kBasisChunk, s));
        }
        return true;
    }
};

// Lower eigenvectors to project out of every Lanczos vector (FP64, dense J
// order, vector l at psi + l * dim), nd of them.
struct Deflation {
    const double *psi = nullptr;
    int nd = 0;
};

template <typename T>
static void run_lanczos(hubbard *h, const hubbard_opts &o, LanczosOut &out, const Deflation &dfl = Deflation(),
                        BasisPool *pool_in = nullptr)
{
    const int64_t n = h->dim;
    const HvArgs args = hv_args(h);
    hipStream_t s = h->stream;
    const HvPlan plan = make_hv_plan(args, sizeof(T));
    const HvPlan plan64 = make_hv_plan(args, sizeof(double));
    const int64_t ld = plan.ld;                 // padded row stride of the two work vectors
    const int64_t npad = h->up.dim * ld;
    const int hb = plan.nparts;
    const int sb = stream_blocks(npad);
    const int max_iter = o.max_iter;

    // one allocation for both work vectors; after the replay it is reused as
    // the FP64 scratch of the residual (2 * npad * sizeof(T) >= npad * 8 bytes)
    // with psi requested it also holds the FP64 residual's two padded vectors
    DevBuf work(std::max(2 * sizeof(T), o.psi ? (size_t)16 : (size_t)0) * (size_t)npad);
    T *vecs[2] = {work.as<T>(), work.as<T>() + npad};
    const int nd = dfl.nd;
    const int db = defl_blocks(h->up.dim);
    DevBuf partials(sizeof(double) *
                    (size_t)(std::max((3 + 2 * kFusedDefl) * std::max(std::max(hb, plan64.nparts), sb), nd * db) + 64));
    DevBuf scal(sizeof(double) * (8 + kMaxDeflate + 1) + sizeof(double) * 2 * (size_t)(max_iter + 1));
    double *S = scal.as<double>();
    double *D = S + 8;  // projections psi_l . q of the deflated step
    PinnedBuf host(sizeof(double) * (2 * (size_t)(max_iter + 1) + 8));
    double *hh = host.as<double>();
    // the reductions write a_j, b_{j+1} straight to host memory (no copy per step)
    double *hist = static_cast<double *>(host.dev);
    const double *given = o.start;
    const uint64_t seed = o.seed;

    // f_1: generated (or given), normalised in FP64, rounded to T
    launch_start_norm2(given, seed, n, partials.as<double>(), sb, s);
    launch_reduce(partials.as<double>(), sb, 0, 1, S + 4, s);
    HUB_HIP(hipMemcpyAsync(hh, S + 4, sizeof(double), hipMemcpyDeviceToHost, s));
    HUB_HIP(hipStreamSynchronize(s));
    if (!(hh[0] > 0.0) || !std::isfinite(hh[0]))
        fail(HUBBARD_EINVAL, "start vector has zero or non-finite norm");
    const double inv_norm = 1.0 / std::sqrt(hh[0]);

    // q <- P q (P = 1 - sum_l psi_l psi_l^T), after q <- q - c v when v is
    // given; leaves the partial sums of |q|^2 (db of them) in `partials`.
    auto project = [&](T *q, const T *v, const double *coef, int64_t ldq) {
        const int nb = launch_defl_dots<T>(q, v, coef, dfl.psi, nd, n, h->up.dim, h->dn.dim, ldq,
                                           partials.as<double>(), s);
        launch_reduce(partials.as<double>(), nb, nb, nd, D, s);
        launch_defl_update<T>(q, dfl.psi, D, nd, n, h->up.dim, h->dn.dim, ldq, partials.as<double>(), s);
    };
    // the same projection of an FP64 vector in dense J order (the accumulated psi)
    auto project_psi = [&](double *q) {
        const int nb = launch_defl_dots<double>(q, nullptr, nullptr, dfl.psi, nd, n, h->up.dim, h->dn.dim, h->dn.dim,
                                                partials.as<double>(), s);
        launch_reduce(partials.as<double>(), nb, nb, nd, D, s);
        launch_defl_update<double>(q, dfl.psi, D, nd, n, h->up.dim, h->dn.dim, h->dn.dim, partials.as<double>(), s);
    };
    auto start_pass = [&](T *C, T *P) {
        launch_start_fill<T>(given, seed, inv_norm, C, P, h->up.dim, h->dn.dim, ld, s);
        if (nd > 0) {
            // f_1 = P f / |P f|: the stored vector keeps its norm, S[0] = 1/|P f|
            project(C, nullptr, nullptr, ld);
            launch_reduce_step(partials.as<double>(), db, RED_START, S, nullptr, 0, s);
        } else {
            launch_init_scalars(S, s);
        }
    };
    // Fused form (two-pass plans of large sectors): the update q - a_j f_j
    // is not a pass of its own.  The step leaves q = H v_j - b_j v_{j-1} in P,
    // the next step's row pass forms f_{j+1} from it while staging rows, and
    // b_{j+1} comes from the expanded norm (the reduction's RED_FUSED mode).
    // Small sectors, where a breakdown or an exhausted space is near, keep the
    // update pass and the norm of the stored vector.
    // With up to kFusedDefl lower states (one amplitude, line layout) the
    // deflated step is fused too: the up-spin pass also sums psi_l.q and
    // psi_l.f_j, the reduction forms g_l = psi_l.(q - a_j f_j) and takes
    // sum_l g_l^2 off the expanded norm, and the next row pass subtracts
    // sum_l g_l psi_l while it forms f_{j+1} (so P is applied to q - a_j f_j
    // as in the unfused step, with no pass of its own).
    const bool fused_defl = nd >= 1 && nd <= kFusedDefl && !args.tcls && args.up_line;
    const bool fused = (nd == 0 || fused_defl) && plan.two_pass && plan.blk_grid > 0 && n >= kFusedMinDim;
    HvDefl hdefl;
    hdefl.psi = dfl.psi;
    hdefl.nd = nd;
    hdefl.pdim = n;
    hdefl.g = S + 8;
    auto hv_step = [&](T *C, T *P) {
        if (fused && nd > 0)
            return launch_hv2<T>(args, plan, C, ld, P, ld, nullptr, 0, HV_FUSED_DEFL, 0.0, S, partials.as<double>(),
                                 s, nullptr, nullptr, &hdefl);
        return launch_hv2<T>(args, plan, C, ld, P, ld, nullptr, 0, fused ? HV_FUSED : HV_LANCZOS, 0.0,
                             fused ? S : S + 1, partials.as<double>(), s);
    };
    // the same step with f_j formed in place in C, f_{j-1} in Pm and the result in Q
    auto hv_step_slot = [&](T *C, T *Pm, T *Q) {
        return launch_hv2<T>(args, plan, C, ld, Pm, ld, nullptr, 0, nd > 0 ? HV_FUSED_DEFL : HV_FUSED, 0.0, S,
                             partials.as<double>(), s, nullptr, nullptr, nd > 0 ? &hdefl : nullptr, Q);
    };
    auto finish_step = [&](T *C, T *P, int np, int j0) {
        if (fused) {
            launch_reduce_step(partials.as<double>(), np, RED_FUSED, S, hist, j0, s, nd);
            // steps whose expanded norm lost its digits form X_{j+1} and its
            // norm explicitly; both launches return at once otherwise
            if (nd > 0) {
                const int nb = launch_fused_fix_defl<T>(P, C, S, dfl.psi, nd, n, h->up.dim, h->dn.dim, ld,
                                                        partials.as<double>(), s);
                launch_reduce_step(partials.as<double>(), nb, RED_FIX, S, hist, j0, s);
                return;
            }
            launch_fused_fix<T>(P, C, S, npad, partials.as<double>(), sb, s);
            launch_reduce_step(partials.as<double>(), sb, RED_FIX, S, hist, j0, s);
            return;
        }
        launch_reduce_step(partials.as<double>(), np, RED_DOT, S, hist, j0, s);
        if (nd > 0) {
            // deflated step: q = P (y - a_j f_j), then b_{j+1} = |q|
            project(P, C, S + 3, ld);
            launch_reduce_step(partials.as<double>(), db, RED_NORM, S, hist, j0, s);
            return;
        }
        launch_axpy_norm<T>(P, C, S + 3, npad, partials.as<double>(), sb, s);
        launch_reduce_step(partials.as<double>(), sb, RED_NORM, S, hist, j0, s);
    };
    auto step = [&](T *C, T *P, int j0) { finish_step(C, P, hv_step(C, P), j0); };

    // ---- first pass: run ahead of the host by `lookahead` steps
    const int lookahead = n >= (int64_t)4000000 ? 2 : 8;
    const int nev = lookahead + 2;
    std::vector<hipEvent_t> ev((size_t)nev);
    for (auto &e : ev)
        HUB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    struct EvGuard {
        std::vector<hipEvent_t> &v;
        ~EvGuard()
        {
            for (auto e : v)
                (void)hipEventDestroy(e);
        }
    } evguard{ev};

    // Resident basis: with psi requested, every stored Lanczos vector (and its
    // scale) is copied to a slot of its own while the device has room (and the
    // handle's basis limit allows), so psi is one combination pass over them
    // instead of a replay of the whole recurrence.  Running out of room frees
    // the slots and falls back to the replay.
    BasisPool local_pool;
    BasisPool &pool = pool_in ? *pool_in : local_pool;
    bool resident = o.psi != nullptr;
    size_t basis_budget = 0;
    if (resident) {
        const size_t vb = sizeof(T) * (size_t)npad;
        if (pool.vb != vb) {
            // slots of another size: the work that used them ran on this stream
            if (!pool.chunks.empty()) {
                HUB_HIP(hipStreamSynchronize(s));
                pool.chunks.clear();
            }
            pool.vb = vb;
            pool.pitch = sizeof(T) * (size_t)ld;
            pool.pad_off = sizeof(T) * (size_t)h->dn.dim;
            pool.rows = h->up.dim;
        }
        size_t fr = 0, tot = 0;
        HUB_HIP(hipMemGetInfo(&fr, &tot));
        const size_t reserve = (size_t)2 << 30;
        const size_t held = pool.chunks.size() * kBasisChunk * vb;
        basis_budget = std::min(held + (fr > reserve ? fr - reserve : 0), h->basis_limit);
    }
    DevBuf scales(o.psi ? sizeof(double) * (size_t)max_iter : 0);
    auto keep = [&](const T *C, int j0) {
        if (!resident)
            return;
        if (!pool.reserve((size_t)j0, basis_budget, s)) {
            resident = false;
            HUB_HIP(hipStreamSynchronize(s));
            pool.chunks.clear();
            return;
        }
        HUB_HIP(hipMemcpyAsync(pool.slot((size_t)j0), C, pool.vb, hipMemcpyDeviceToDevice, s));
        HUB_HIP(hipMemcpyAsync(scales.as<double>() + j0, S, sizeof(double), hipMemcpyDeviceToDevice, s));
    };
    // Fused steps with psi requested (line layout) form each Lanczos vector in
    // its slot: step j's row pass forms f_j in slot j from the q that step j-1
    // left there and the H.v result goes to slot j + 1, so keeping a vector
    // costs no copy.  When the pool cannot grow, the two live vectors move to
    // the work vectors and the run goes on as without psi (psi by replay).
    bool inslot = resident && fused && args.up_line && pool.reserve(1, basis_budget, s);
    auto slotp = [&](int j) { return static_cast<T *>(pool.slot((size_t)j)); };
    auto leave_slots = [&](int j0) {
        // step j0 is next: q in slot j0, f_{j0-1} in slot j0 - 1
        HUB_HIP(hipMemcpyAsync(vecs[j0 & 1], slotp(j0), pool.vb, hipMemcpyDeviceToDevice, s));
        HUB_HIP(hipMemcpyAsync(vecs[(j0 + 1) & 1], slotp(j0 - 1), pool.vb, hipMemcpyDeviceToDevice, s));
        HUB_HIP(hipStreamSynchronize(s));
        pool.chunks.clear();
        inslot = false;
        resident = false;
    };

    T *bufs[2] = {vecs[0], vecs[1]};
    auto t0 = std::chrono::steady_clock::now();
    if (inslot)
        start_pass(slotp(0), bufs[1]);  // bufs[1]: zeros, the vector before f_1
    else
        start_pass(bufs[0], bufs[1]);
    if (nd > 0) {
        HUB_HIP(hipMemcpyAsync(hh, S, sizeof(double), hipMemcpyDeviceToHost, s));
        HUB_HIP(hipStreamSynchronize(s));
        // 1/|P f| of the unit start vector
        if (!std::isfinite(hh[0]) || !(hh[0] > 0.0) || hh[0] > 1e8)
            fail(HUBBARD_EINVAL, "the start vector lies in the span of the lower states");
    }
    out.a.clear();
    out.b.clear();
    out.e.clear();
    int launched = 0, checked = 0;
    bool stop = false;
    double scale = 0.0;
    while (!stop) {
        if (launched < max_iter) {
            const int j0 = launched;  // 0-based step index
            T *C = bufs[j0 & 1], *P = bufs[(j0 + 1) & 1];
            if (inslot && !pool.reserve((size_t)j0 + 1, basis_budget, s))
                leave_slots(j0);
            if (inslot) {
                const int np = hv_step_slot(slotp(j0), j0 > 0 ? slotp(j0 - 1) : bufs[1], slotp(j0 + 1));
                HUB_HIP(hipMemcpyAsync(scales.as<double>() + j0, S, sizeof(double), hipMemcpyDeviceToDevice, s));
                // q is in slot j0 + 1, f_j0 in slot j0
                finish_step(slotp(j0), slotp(j0 + 1), np, j0);
            } else if (fused) {
                // f_j exists once the step's row pass has formed it; S[0] still holds 1/s_j
                const int np = hv_step(C, P);
                keep(C, j0);
                finish_step(C, P, np, j0);
            } else {
                keep(C, j0);
                step(C, P, j0);
            }
            HUB_HIP(hipEventRecord(ev[(size_t)(j0 % nev)], s));
            launched++;
        }
        while (checked < launched && (launched - checked > lookahead || launched == max_iter)) {
            const int j0 = checked;
            HUB_HIP(hipEventSynchronize(ev[(size_t)(j0 % nev)]));
            const double a = hh[2 * j0], b = hh[2 * j0 + 1];
            out.a.push_back(a);
            out.b.push_back(b);
            const int j = j0 + 1;
            const double e = tridiag_lowest(out.a.data(), out.b.data(), j);
            out.e.push_back(e);
            checked++;
            if (!std::isfinite(a) || !std::isfinite(b))
                fail(HUBBARD_EDEVICE, "non-finite Lanczos coefficient at step " + std::to_string(j));
            if (o.tol >= 0.0 && j >= 2 && std::fabs(e - out.e[(size_t)j0 - 1]) <= o.tol * std::fmax(1.0, std::fabs(e))) {
                out.stop = HUBBARD_STOP_CONVERGED;
                stop = true;
                break;
            }
            scale = std::fmax(scale, std::fabs(a) + (j0 > 0 ? out.b[(size_t)j0 - 1] : 0.0));
            if (b == 0.0 || b <= 1e-12 * scale) {
                out.stop = HUBBARD_STOP_BREAKDOWN;
                stop = true;
                break;
            }
            if ((int64_t)j >= n - nd) {
                out.stop = HUBBARD_STOP_EXHAUSTED;
                stop = true;
                break;
            }
            if (j == max_iter) {
                out.stop = HUBBARD_STOP_MAXITER;
                stop = true;
                break;
            }
        }
    }
    HUB_HIP(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    out.m = checked;
    out.a.resize((size_t)out.m);
    out.b.resize((size_t)out.m);
    out.e.resize((size_t)out.m);
    out.e0 = out.e.back();
    out.seconds_first = std::chrono::duration<double>(t1 - t0).count();

    if (!o.psi)
        return;
    const int m = out.m;
    std::vector<double> y((size_t)m);
    tridiag_lowest_vector(out.a.data(), out.b.data(), m, out.e0, y.data());
    out.psi_resident = resident && pool.capacity() >= (size_t)m;
    if (out.psi_resident) {
        // ---- psi = sum_j y_j f_j from the resident vectors
        std::vector<const T *> ptrs((size_t)m);
        for (int j = 0; j < m; j++)
            ptrs[(size_t)j] = static_cast<const T *>(pool.slot((size_t)j));
        DevBuf dptr(sizeof(const T *) * (size_t)m), dy(sizeof(double) * (size_t)m);
        HUB_HIP(hipMemcpyAsync(dptr.p, ptrs.data(), sizeof(const T *) * (size_t)m, hipMemcpyHostToDevice, s));
        HUB_HIP(hipMemcpyAsync(dy.p, y.data(), sizeof(double) * (size_t)m, hipMemcpyHostToDevice, s));
        launch_psi_combine<T>(o.psi, dptr.as<const T *>(), dy.as<double>(), scales.as<double>(), m, h->up.dim,
                              h->dn.dim, ld, s);
        HUB_HIP(hipStreamSynchronize(s));
    } else {
        // ---- second pass: replay the identical recurrence and accumulate psi
        if (!pool.chunks.empty()) {
            HUB_HIP(hipStreamSynchronize(s));
            pool.chunks.clear();
        }
        start_pass(bufs[0], bufs[1]);
        for (int j0 = 0; j0 < m; j0++) {
            T *C = bufs[j0 & 1], *P = bufs[(j0 + 1) & 1];
            if (fused) {
                // f_j exists once the step's row pass has formed it; S[0] still holds 1/s_j
                const int np = hv_step(C, P);
                launch_psi_acc<T>(o.psi, C, y[(size_t)j0], S, h->up.dim, h->dn.dim, ld, j0 == 0, s);
                if (j0 + 1 < m)
                    finish_step(C, P, np, j0);
                continue;
            }
            launch_psi_acc<T>(o.psi, C, y[(size_t)j0], S, h->up.dim, h->dn.dim, ld, j0 == 0, s);
            if (j0 + 1 < m)
                step(C, P, j0);
        }
    }
    // the accumulated vector is projected once more, so that it is orthogonal
    // to the lower states to rounding
    if (nd > 0)
        project_psi(o.psi);
    // normalise, sign so that <psi, f1> > 0
    launch_psi_stats(o.psi, given, seed, n, partials.as<double>(), sb, s);
    launch_reduce(partials.as<double>(), sb, sb, 2, S + 4, s);
    HUB_HIP(hipMemcpyAsync(hh, S + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HUB_HIP(hipStreamSynchronize(s));
    double c = 1.0 / std::sqrt(hh[0]);
    if (hh[1] * inv_norm < 0.0)
        c = -c;
    launch_scale(o.psi, c, n, s);
    // FP64 residual |H psi - E0 psi| and Rayleigh quotient <psi|H|psi>
    // rows of psi are dense: the row pass copies them to padded rows beside
    // its result, for the up-spin pass
    const int hb64 = launch_hv2<double>(args, plan64, o.psi, h->dn.dim, nullptr, 0, work.as<double>(), ld, HV_RESIDUAL,
                                        out.e0, nullptr, partials.as<double>(), s, work.as<double>() + npad);
    launch_reduce(partials.as<double>(), hb64, hb64, 2, S + 4, s);
    HUB_HIP(hipMemcpyAsync(hh, S + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HUB_HIP(hipStreamSynchronize(s));
    out.residual = std::sqrt(hh[0]);
    out.rayleigh = hh[1];
}

void validate_opts(const hubbard_opts &o)
{
    if (!(o.max_iter >= 1))
        fail(HUBBARD_EINVAL, "max_iter must be >= 1");
    if (std::isnan(o.tol))
        fail(HUBBARD_EINVAL, "tol is NaN");
    if (o.precision != HUBBARD_FP64 && o.precision != HUBBARD_MIXED)
        fail(HUBBARD_EINVAL, "unknown precision");
}

static hubbard_result make_result(const LanczosOut &out, const hubbard_opts &o, double seconds, int status)
{
    hubbard_result r;
    std::memset(&r, 0, sizeof(r));
    r.e0 = out.e0;
    r.residual = o.psi ? out.residual : -1.0;
    r.rayleigh = o.psi ? out.rayleigh : NAN;
    if (o.psi) {
        r.err_est = out.residual / std::fmax(1.0, std::fabs(out.e0));
    } else {
        // Lanczos estimate of |H psi - E0 psi| for the Ritz pair: b_{m+1} |y_m|
        std::vector<double> y((size_t)out.m);
        tridiag_lowest_vector(out.a.data(), out.b.data(), out.m, out.e0, y.data());
        r.err_est = std::fabs(out.b.back() * y.back()) / std::fmax(1.0, std::fabs(out.e0));
    }
    r.seconds = seconds;
    r.seconds_per_iter = out.m ? out.seconds_first / out.m : 0.0;
    r.n_iter = out.m;
    r.stop = out.stop;
    r.status = status;
    r.precision = o.precision;
    r.psi_resident = (o.psi && out.psi_resident) ? 1 : 0;
    return r;
}

static int status_of(const LanczosOut &out, const hubbard_opts &o)
{
    return (out.stop == HUBBARD_STOP_MAXITER && o.tol >= 0.0) ? HUBBARD_ENOCONV : HUBBARD_OK;
}

int lanczos_impl(hubbard *h, const hubbard_opts &o, hubbard_result *res)
{
    validate_opts(o);
    use_device(h);
    auto t0 = std::chrono::steady_clock::now();
    LanczosOut out;
    if (o.precision == HUBBARD_FP64)
        run_lanczos<double>(h, o, out);
    else
        run_lanczos<float>(h, o, out);
    auto t1 = std::chrono::steady_clock::now();
    if (o.a_out)
        std::memcpy(o.a_out, out.a.data(), sizeof(double) * (size_t)out.m);
    if (o.b_out)
        std::memcpy(o.b_out, out.b.data(), sizeof(double) * (size_t)out.m);
    if (o.e_out)
        std::memcpy(o.e_out, out.e.data(), sizeof(double) * (size_t)out.m);
    const int status = status_of(out, o);
    if (res)
        *res = make_result(out, o, std::chrono::duration<double>(t1 - t0).count(), status);
    return status;
}

// The k lowest eigenpairs one after another: state i is the ground state of
// P_i H P_i, P_i projecting out psi_0..psi_{i-1} (Sec. 2.2 names the lowest
// excited states as a goal of the method; the deflation by projection is this
// library's choice of how to reach them with the same recurrence).
int lowest_states_impl(hubbard *h, int k, const hubbard_opts &o, double *E, double *psi, hubbard_result *res)
{
    validate_opts(o);
    if (k < 1 || k > kMaxDeflate + 1)
        fail(HUBBARD_EINVAL, "k must lie in 1.." + std::to_string(kMaxDeflate + 1));
    if ((int64_t)k > h->dim)
        fail(HUBBARD_EINVAL, "k exceeds the sector dimension");
    if (!E)
        fail(HUBBARD_EINVAL, "E is NULL");
    if (o.psi || o.a_out || o.b_out || o.e_out)
        fail(HUBBARD_EINVAL, "opts.psi and the history arrays are not used by hubbard_lowest_states");
    use_device(h);
    std::unique_ptr<DevBuf> own;
    double *base = psi;
    if (!base) {
        own.reset(new DevBuf(sizeof(double) * (size_t)k * (size_t)h->dim));
        base = own->as<double>();
    }
    int worst = HUBBARD_OK;
    BasisPool pool;  // the resident basis slots, reused by every state
    for (int i = 0; i < k; i++) {
        auto t0 = std::chrono::steady_clock::now();
        // an independent start vector per state: a start shared by all of them
        // has, inside a degenerate level, only the component that the first
        // state of that level takes away, so the level's other vectors would be
        // missed
        hubbard_opts oi = o;
        oi.seed = o.seed + (uint64_t)i;
        if (i > 0)
            oi.start = nullptr;
        oi.psi = base + (size_t)i * (size_t)h->dim;
        Deflation d;
        d.psi = base;
        d.nd = i;
        LanczosOut out;
        if (o.precision == HUBBARD_FP64)
            run_lanczos<double>(h, oi, out, d, &pool);
        else
            run_lanczos<float>(h, oi, out, d, &pool);
        auto t1 = std::chrono::steady_clock::now();
        const int status = status_of(out, oi);
        E[i] = out.e0;
        if (res)
            res[i] = make_result(out, oi, std::chrono::duration<double>(t1 - t0).count(), status);
        worst = std::max(worst, status);
    }
    return worst;
}

// Krylov dimension limit of one propagation step
constexpr int kMaxKrylov = 64;

int propagate_impl(hubbard *h, double *re, double *im, double t, int n_steps, int m, double *energy,
                   hubbard_prop_result *res)
{
    if (!re || !im || re == im)
        fail(HUBBARD_EINVAL, "psi_re and psi_im must be two distinct device arrays");
    if (!std::isfinite(t))
        fail(HUBBARD_EINVAL, "t is not finite");
    if (n_steps < 1)
        fail(HUBBARD_EINVAL, "n_steps must be >= 1");
    if (m < 2 || m > kMaxKrylov)
        fail(HUBBARD_EINVAL, "krylov_dim must lie in 2.." + std::to_string(kMaxKrylov));
    use_device(h);
    auto t0 = std::chrono::steady_clock::now();
    const HvArgs args = hv_args(h);
    hipStream_t s = h->stream;
    const HvPlan plan = make_hv_plan(args, sizeof(double));
    const int64_t ld = plan.ld, npad = h->up.dim * ld, stride = 2 * npad;
    const int64_t du = h->up.dim, dd = h->dn.dim;
    // the Krylov basis, resident: slot m receives the last H.v of a step.  The
    // unfused H.v runs with beta = 0 on the old contents of a slot, so they start
    // as zeros.  The fused step reads slot 1 with weight 0 in step 0 and writes
    // only row elements, so there slot 1 and the rows' padding (which the
    // fix-up of a flagged step reads) are the parts cleared.
    const size_t bbytes = sizeof(double) * (size_t)stride * (size_t)(m + 1);
    DevBuf basis(bbytes);
    const bool fused = plan.two_pass && plan.blk_grid > 0 && args.up_line;
    if (fused) {
        HUB_HIP(hipMemsetAsync(static_cast<double *>(basis.p) + stride, 0, sizeof(double) * (size_t)stride, s));
        if (ld > dd)
            HUB_HIP(hipMemset2DAsync(static_cast<double *>(basis.p) + dd, sizeof(double) * (size_t)ld, 0,
                                     sizeof(double) * (size_t)(ld - dd), 2 * (size_t)du * (size_t)(m + 1), s));
    } else {
        HUB_HIP(hipMemsetAsync(basis.p, 0, bbytes, s));
    }
    DevBuf partials(sizeof(double) * (size_t)(std::max(6 * plan.nparts, 4096) + 64));
    DevBuf scal(sizeof(double) * 4 * (size_t)(m + 2));
    DevBuf gamd(sizeof(double) * 2 * (size_t)m);
    PinnedBuf host(sizeof(double) * (4 * (size_t)(m + 2) + 2 * (size_t)m));
    double *sh = host.as<double>(), *gh = sh + 4 * (m + 2);
    double *sc = scal.as<double>(), *B = basis.as<double>(), *part = partials.as<double>();
    auto slot = [&](int j) { return B + (size_t)j * (size_t)stride; };

    // Fused form (two-pass plans with the line layout of the up-spin
    // entries): step j's row pass forms w_j = q_{j-1} - c w_{j-1} in slot j
    // while it stages the rows, as the ground-state step does, and writes
    // s_j H w_j + beta w_{j-1} to slot j + 1; both halves run in the same
    // launches and one reduction gives a_j and b_{j+1} (expanded norm).  The
    // scalars then live in the ground-state layout S, the coefficients in
    // hist (a_j, b_{j+1}) and the scale of each w_j in scl.  Other plans keep
    // the separate update pass.
    const int sb = stream_blocks(stride);
    DevBuf fsc(sizeof(double) * (8 + kMaxDeflate + 1 + 2 * (size_t)m + (size_t)m + 8));
    double *S = fsc.as<double>(), *hist = S + 8 + kMaxDeflate + 1, *scl = hist + 2 * m;
    int nb = launch_prop_load(re, im, B, npad, du, dd, ld, part, s);
    if (fused)
        launch_reduce_step(part, nb, RED_START, S, nullptr, 0, s);
    else
        launch_prop_reduce(part, nb, PROP_START, sc, 0, s);
    const double dt = t / n_steps;
    double err = 0.0;
    int mmax = 0;
    for (int k = 0; k <= n_steps; k++) {
        // the round after the last step only measures <H> of the final state
        const int msteps = k < n_steps ? m : 1;
        for (int j = 0; j < msteps; j++) {
            if (fused) {
                // w_j is formed by this step's row pass; S[0] = 1/|w_j| until the reduction
                HUB_HIP(hipMemcpyAsync(scl + j, S, sizeof(double), hipMemcpyDeviceToDevice, s));
                // slot j - 1 feeds the beta and c terms (both 0 in step 0, any finite slot will do)
                const int np = launch_hv2<double>(args, plan, slot(j), ld, slot(j > 0 ? j - 1 : j + 1), ld, nullptr,
                                                  0, HV_FUSED, 0.0, S, part, s, nullptr, nullptr, nullptr,
                                                  slot(j + 1), npad);
                launch_reduce_step(part, np, RED_FUSED, S, hist, j, s);
                if (k == n_steps)
                    break;
                // steps whose expanded norm lost its digits form w_{j+1} explicitly
                launch_fused_fix<double>(slot(j + 1), slot(j), S, stride, part, sb, s);
                launch_reduce_step(part, sb, RED_FIX, S, hist, j, s);
                continue;
            }
            const int np = launch_hv2<double>(args, plan, slot(j), ld, slot(j + 1), ld, nullptr, 0, HV_LANCZOS, 0.0,
                                              sc + 4 * j, part, s);
            const int np2 = launch_hv2<double>(args, plan, slot(j) + npad, ld, slot(j + 1) + npad, ld, nullptr, 0,
                                               HV_LANCZOS, 0.0, sc + 4 * j, part + np, s);
            launch_prop_reduce(part, np + np2, PROP_DOT, sc, j, s);
            if (k == n_steps)
                break;
            nb = launch_prop_update(slot(j + 1), slot(j), j > 0 ? slot(j - 1) : nullptr, sc, j, stride, part, s);
            launch_prop_reduce(part, nb, PROP_NORM, sc, j, s);
        }
        if (fused) {
            // the same host view as the unfused form: {s_j, -, a_j, b_{j+1}} per step
            std::vector<double> fh(3 * (size_t)msteps);
            HUB_HIP(hipMemcpyAsync(fh.data(), hist, sizeof(double) * 2 * (size_t)msteps, hipMemcpyDeviceToHost, s));
            HUB_HIP(hipMemcpyAsync(fh.data() + 2 * msteps, scl, sizeof(double) * (size_t)msteps,
                                   hipMemcpyDeviceToHost, s));
            HUB_HIP(hipStreamSynchronize(s));
            for (int j = 0; j < msteps; j++) {
                sh[4 * j] = fh[2 * (size_t)msteps + (size_t)j];
                sh[4 * j + 1] = 0.0;
                sh[4 * j + 2] = fh[2 * (size_t)j];
                sh[4 * j + 3] = fh[2 * (size_t)j + 1];
            }
        } else {
            HUB_HIP(hipMemcpyAsync(sh, sc, sizeof(double) * 4 * (size_t)(msteps + 1), hipMemcpyDeviceToHost, s));
            HUB_HIP(hipStreamSynchronize(s));
        }
        if (!(sh[0] > 0.0) || !std::isfinite(sh[0]))
            fail(k == 0 ? HUBBARD_EINVAL : HUBBARD_EDEVICE, "psi has zero or non-finite norm");
        if (energy)
            energy[k] = sh[2];
        if (k == n_steps)
            break;
        // Krylov dimension: up to the first vanishing b_{j+1} (an invariant subspace, where the step is exact)
        int nv = m;
        double scale = 0.0;
        for (int j = 0; j < m; j++) {
            const double a = sh[4 * j + 2], b = sh[4 * j + 3];
            if (!std::isfinite(a) || !std::isfinite(b))
                fail(HUBBARD_EDEVICE, "non-finite Krylov coefficient in step " + std::to_string(k + 1));
            scale = std::fmax(scale, std::fabs(a) + (j > 0 ? sh[4 * (j - 1) + 3] : 0.0));
            if (!(b > 1e-12 * scale)) {
                nv = j + 1;
                break;
            }
        }
        std::vector<double> d((size_t)nv), e((size_t)nv), cr((size_t)nv), ci((size_t)nv);
        for (int j = 0; j < nv; j++) {
            d[(size_t)j] = sh[4 * j + 2];
            e[(size_t)j] = sh[4 * j + 3];
        }
        tridiag_expm_e1(d.data(), e.data(), nv, dt, cr.data(), ci.data());
        const double nrm = 1.0 / sh[0];  // |psi| at the start of the step
        if (nv == m)
            err += nrm * sh[4 * (m - 1) + 3] * std::hypot(cr[(size_t)m - 1], ci[(size_t)m - 1]);
        for (int j = 0; j < nv; j++) {
            gh[2 * j] = nrm * cr[(size_t)j] * sh[4 * j];
            gh[2 * j + 1] = nrm * ci[(size_t)j] * sh[4 * j];
        }
        HUB_HIP(hipMemcpyAsync(gamd.p, gh, sizeof(double) * 2 * (size_t)nv, hipMemcpyHostToDevice, s));
        // the caller's halves receive the state after the last step only
        const bool last = k == n_steps - 1;
        nb = launch_prop_combine(B, nv, stride, npad, gamd.as<double>(), last ? re : nullptr, last ? im : nullptr, du,
                                 dd, ld, part, s);
        if (fused)
            launch_reduce_step(part, nb, RED_START, S, nullptr, 0, s);
        else
            launch_prop_reduce(part, nb, PROP_START, sc, 0, s);
        mmax = std::max(mmax, nv);
    }
    auto t1 = std::chrono::steady_clock::now();
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->err_est = err;
        res->norm = 1.0 / sh[0];
        res->seconds = std::chrono::duration<double>(t1 - t0).count();
        res->n_steps = n_steps;
        res->krylov_dim_max = mmax;
    }
    return HUBBARD_OK;
}

}  // namespace hub

using namespace hub;

extern "C" {

// amp: NULL (every bond has amplitude t) or one amplitude per bond.
static int build_impl(int sites, const int32_t *edges, const double *amp, int n_edges, int n_up, int n_dn, double t,
                      double U, hubbard_h *out)
{
    return guarded([&]() -> int {
        if (!out)
            fail(HUBBARD_EINVAL, "out is NULL");
        *out = nullptr;
        if (sites < 1 || sites > 32)
            fail(HUBBARD_EINVAL, "sites must be in 1..32");
        if (n_edges < 0 || (n_edges > 0 && !edges))
            fail(HUBBARD_EINVAL, "bad edge list");
        if (n_up < 0 || n_up > sites || n_dn < 0 || n_dn > sites)
            fail(HUBBARD_EINVAL, "electron counts must be in 0..sites");
        if (!std::isfinite(t) || !std::isfinite(U))
            fail(HUBBARD_EINVAL, "t and U must be finite");
        std::vector<int32_t> e((size_t)2 * (size_t)n_edges);
        std::vector<char> seen((size_t)sites * (size_t)sites, 0);
        for (int k = 0; k < n_edges; k++) {
            int i = edges[2 * k], j = edges[2 * k + 1];
            if (i < 0 || j < 0 || i >= sites || j >= sites || i == j)
                fail(HUBBARD_EINVAL, "edge " + std::to_string(k) + " is not a pair of distinct sites");
            int lo = std::min(i, j), hi = std::max(i, j);
            if (seen[(size_t)lo * (size_t)sites + (size_t)hi])
                fail(HUBBARD_EINVAL, "edge " + std::to_string(k) + " repeats a bond");
            seen[(size_t)lo * (size_t)sites + (size_t)hi] = 1;
            e[(size_t)2 * k] = i;
            e[(size_t)2 * k + 1] = j;
        }
        // per-bond amplitudes: classes of equal value (all equal = the one-amplitude model)
        std::vector<double> tcls;
        std::vector<uint8_t> bond_cls;
        if (amp) {
            for (int k = 0; k < n_edges; k++)
                if (!std::isfinite(amp[k]))
                    fail(HUBBARD_EINVAL, "amplitude of edge " + std::to_string(k) + " is not finite");
            bool uniform = true;
            for (int k = 1; k < n_edges; k++)
                uniform = uniform && amp[k] == amp[0];
            if (uniform) {
                t = n_edges > 0 ? amp[0] : 0.0;
            } else {
                bond_cls.resize((size_t)n_edges);
                for (int k = 0; k < n_edges; k++) {
                    size_t c = 0;
                    while (c < tcls.size() && tcls[c] != amp[k])
                        c++;
                    if (c == tcls.size()) {
                        if ((int)tcls.size() == kMaxAmpClasses)
                            fail(HUBBARD_EINVAL, "more than " + std::to_string(kMaxAmpClasses) +
                                                     " distinct hopping amplitudes");
                        tcls.push_back(amp[k]);
                    }
                    bond_cls[(size_t)k] = (uint8_t)c;
                }
                t = NAN;
            }
        }
        const uint64_t du = binomial(sites, n_up), dd = binomial(sites, n_dn);
        // a spin dimension is at most C(32,16) < 2^31, so the sector size is the limit:
        // one vector of 2^40 elements would not fit the memory of any single device
        if ((long double)du * (long double)dd >= (long double)(1ull << 40))
            fail(HUBBARD_ERANGE, "sector dimension exceeds 2^40");
        if (!tcls.empty() && (du >= (1ull << 24) || dd >= (1ull << 24)))
            fail(HUBBARD_ERANGE, "per-bond amplitudes need spin dimensions below 2^24");
        std::unique_ptr<hubbard> h(new hubbard());
        h->sites = sites;
        h->n_up = n_up;
        h->n_dn = n_dn;
        h->t = t;
        h->U = U;
        h->edges = e;
        h->tcls = tcls;
        h->bond_cls = bond_cls;
        build_spin_table(sites, e, n_up, h->up);
        build_spin_table(sites, e, n_dn, h->dn);
        h->dim = h->up.dim * h->dn.dim;
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
            (void)hipGetLastError();
            h->device = -1;  // host tables only: info and export work, device calls fail
        } else {
            HUB_HIP(hipGetDevice(&h->device));
            try {
                upload_tables(h.get());
            } catch (...) {
                free_device(h.get());
                throw;
            }
        }
        *out = h.release();
        return HUBBARD_OK;
    });
}

int hubbard_build(int sites, const int32_t *edges, int n_edges, int n_up, int n_dn, double t, double U,
                  hubbard_h *out)
{
    return build_impl(sites, edges, nullptr, n_edges, n_up, n_dn, t, U, out);
}

int hubbard_build_bonds(int sites, const int32_t *edges, const double *t, int n_edges, int n_up, int n_dn, double U,
                        hubbard_h *out)
{
    if (n_edges > 0 && !t)
        return guarded([&]() -> int { fail(HUBBARD_EINVAL, "t is NULL"); });
    return build_impl(sites, edges, t, n_edges, n_up, n_dn, 0.0, U, out);
}

int hubbard_free(hubbard_h h)
{
    return guarded([&]() -> int {
        if (!h)
            return HUBBARD_OK;
        if (h->device >= 0) {
            (void)hipSetDevice(h->device);
            free_device(h);
        }
        delete h;
        return HUBBARD_OK;
    });
}

int hubbard_set_stream(hubbard_h h, void *hip_stream)
{
    return guarded([&]() -> int {
        check_handle(h);
        h->stream = static_cast<hipStream_t>(hip_stream);
        return HUBBARD_OK;
    });
}

int hubbard_set_precision(hubbard_h h, int precision)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (precision != HUBBARD_FP64 && precision != HUBBARD_MIXED)
            fail(HUBBARD_EINVAL, "unknown precision");
        h->precision = precision;
        return HUBBARD_OK;
    });
}

int hubbard_set_basis_limit(hubbard_h h, size_t bytes)
{
    return guarded([&]() -> int {
        check_handle(h);
        h->basis_limit = bytes;
        return HUBBARD_OK;
    });
}

int hubbard_set_seed(hubbard_h h, uint64_t seed)
{
    return guarded([&]() -> int {
        check_handle(h);
        h->seed = seed;
        return HUBBARD_OK;
    });
}

static int apply_impl(hubbard_h h, const void *x, int64_t ldx, void *y, int64_t ldy)
{
    check_handle(h);
    if (!x || !y)
        fail(HUBBARD_EINVAL, "x and y must be device pointers");
    const int64_t ddn = h->dn.dim;
    if (ldx < ddn || ldy < ddn)
        fail(HUBBARD_EINVAL, "row strides must be >= dim_dn");
    const size_t es = h->precision == HUBBARD_FP64 ? 8 : 4;
    const char *xb = static_cast<const char *>(x);
    const char *yb = static_cast<const char *>(y);
    const size_t xbytes = es * (size_t)((h->up.dim - 1) * ldx + ddn);
    const size_t ybytes = es * (size_t)((h->up.dim - 1) * ldy + ddn);
    if (xb < yb + ybytes && yb < xb + xbytes)
        fail(HUBBARD_EINVAL, "x and y overlap");
    use_device(h);
    const HvArgs a = hv_args(h);
    const HvPlan pl = make_hv_plan(a, (int)es);
    if (!pl.two_pass && (ldx != ddn || ldy != ddn))
        fail(HUBBARD_EINVAL, "rows too wide for the staged kernels: only dense rows (ld = dim_dn) are supported");
    // rows not on 128 bytes: the H.v routes through two padded work vectors
    // (the row pass writes them, the up-spin pass reads them and writes y)
    const int64_t slw = 128 / (int64_t)es;
    void *wx = nullptr, *wy = nullptr;
    if (pl.two_pass && pl.blk_grid > 0 && a.up_line && (ldx % slw != 0 || ldy % slw != 0)) {
        const size_t npad = (size_t)h->up.dim * (size_t)pl.ld;
        const size_t need = 2 * npad * es;
        if (h->apply_work_bytes < need) {
            if (h->apply_work) {
                HUB_HIP(hipStreamSynchronize(h->stream));
                HUB_HIP(hipFree(h->apply_work));
                h->apply_work = nullptr;
                h->apply_work_bytes = 0;
            }
            HUB_HIP(hipMalloc(&h->apply_work, need));
            h->apply_work_bytes = need;
        }
        if (!h->apply_ev)
            HUB_HIP(hipEventCreateWithFlags(&h->apply_ev, hipEventDisableTiming));
        else
            HUB_HIP(hipStreamWaitEvent(h->stream, h->apply_ev, 0));
        wx = h->apply_work;
        wy = static_cast<char *>(h->apply_work) + npad * es;
    }
    if (h->precision == HUBBARD_FP64)
        launch_hv2<double>(a, pl, static_cast<const double *>(x), ldx, static_cast<double *>(y), ldy, nullptr, 0,
                           HV_STORE, 0.0, nullptr, nullptr, h->stream, static_cast<double *>(wx),
                           static_cast<double *>(wy));
    else
        launch_hv2<float>(a, pl, static_cast<const float *>(x), ldx, static_cast<float *>(y), ldy, nullptr, 0,
                          HV_STORE, 0.0, nullptr, nullptr, h->stream, static_cast<float *>(wx),
                          static_cast<float *>(wy));
    if (wx)
        HUB_HIP(hipEventRecord(h->apply_ev, h->stream));
    return HUBBARD_OK;
}

int hubbard_apply(hubbard_h h, const void *x, void *y)
{
    return guarded([&]() -> int {
        check_handle(h);
        return apply_impl(h, x, h->dn.dim, y, h->dn.dim);
    });
}

int hubbard_apply_ld(hubbard_h h, const void *x, int64_t ldx, void *y, int64_t ldy)
{
    return guarded([&]() -> int { return apply_impl(h, x, ldx, y, ldy); });
}

int hubbard_lanczos(hubbard_h h, double tol, int max_iter, double *E0, double *psi)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (!E0)
            fail(HUBBARD_EINVAL, "E0 is NULL");
        if (!(tol > 0.0))
            fail(HUBBARD_EINVAL, "tol must be > 0");
        hubbard_opts o;
        std::memset(&o, 0, sizeof(o));
        o.tol = tol;
        o.max_iter = max_iter;
        o.precision = h->precision;
        o.seed = h->seed;
        o.psi = psi;
        hubbard_result r;
        int rc = lanczos_impl(h, o, &r);
        *E0 = r.e0;
        return rc;
    });
}

int hubbard_lanczos_ex(hubbard_h h, const hubbard_opts *opts, hubbard_result *res)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (!opts || !res)
            fail(HUBBARD_EINVAL, "opts and res must not be NULL");
        return lanczos_impl(h, *opts, res);
    });
}

int hubbard_lowest_states(hubbard_h h, int k, const hubbard_opts *opts, double *E, double *psi,
                          hubbard_result *res)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (!opts)
            fail(HUBBARD_EINVAL, "opts is NULL");
        return lowest_states_impl(h, k, *opts, E, psi, res);
    });
}

// The normalised observables from the unnormalised device sums r (host copy).
static void observables_out(const hubbard *h, const double *r, double *dens, double *corr, double *docc)
{
    const int NS = obs_ns_max(h->sites);
    const double norm = r[(size_t)3 * NS * NS];
    if (!(norm > 0.0) || !std::isfinite(norm))
        fail(HUBBARD_EINVAL, "psi has zero or non-finite norm");
    const int n = h->sites;
    auto at = [&](int block, int i, int j) { return r[(size_t)block * NS * NS + (size_t)i * NS + j] / norm; };
    if (dens)
        for (int i = 0; i < n; i++) {
            dens[i] = at(0, i, i);
            dens[n + i] = at(1, i, i);
        }
    if (corr)
        for (int b = 0; b < 3; b++)
            for (int i = 0; i < n; i++)
                for (int j = 0; j < n; j++)
                    corr[(size_t)b * n * n + (size_t)i * n + j] = at(b, i, j);
    if (docc) {
        double d = 0.0;
        for (int i = 0; i < n; i++)
            d += r[(size_t)2 * NS * NS + (size_t)i * NS + i];
        *docc = d / norm;
    }
}

int hubbard_observables_noalloc(hubbard_h h, const double *psi, double *dens, double *corr, double *docc)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (!psi)
            fail(HUBBARD_EINVAL, "psi is NULL");
        use_device(h);
        const int NS = obs_ns_max(h->sites);
        const int ps = 3 * NS * NS + 1;
        double *scr = obs_scratch(h->device);
        const int nb = obs_noalloc_blocks(h->sites, h->up.dim, h->dn.dim);
        const int np = obs_partial_count(h->sites, h->up.dim, h->dn.dim, nb);
        if ((size_t)(np + 1) * (size_t)ps * sizeof(double) > kObsScratchBytes)
            fail(HUBBARD_ERANGE, "the partial sums of this lattice exceed the " +
                                     std::to_string(kObsScratchBytes >> 20) + " MiB observables scratch");
        // partials first, the final sums after them; every value is written
        // by the kernels before it is read, so nothing is cleared
        double *part = scr, *sums = scr + (size_t)np * (size_t)ps;
        launch_observables(psi, h->dev.states_up, h->dev.states_dn, h->sites, h->up.dim, h->dn.dim, part, sums, nb,
                           h->stream);
        // host copy of the sums in a buffer of this thread (no allocation per call)
        thread_local double r[3 * 32 * 32 + 1];
        HUB_HIP(hipMemcpyAsync(r, sums, sizeof(double) * (size_t)ps, hipMemcpyDeviceToHost, h->stream));
        HUB_HIP(hipStreamSynchronize(h->stream));
        observables_out(h, r, dens, corr, docc);
        return HUBBARD_OK;
    });
}

int hubbard_observables(hubbard_h h, const double *psi, double *dens, double *corr, double *docc)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (!psi)
            fail(HUBBARD_EINVAL, "psi is NULL");
        use_device(h);
        const int NS = obs_ns_max(h->sites);
        const int ps = 3 * NS * NS + 1;
        const int np = obs_partial_count(h->sites, h->up.dim, h->dn.dim);
        DevBuf part(sizeof(double) * (size_t)np * (size_t)ps);
        DevBuf sums(sizeof(double) * (size_t)ps);
        launch_observables(psi, h->dev.states_up, h->dev.states_dn, h->sites, h->up.dim, h->dn.dim,
                           part.as<double>(), sums.as<double>(), kObsDefaultBlocks, h->stream);
        std::vector<double> r((size_t)ps);
        HUB_HIP(hipMemcpyAsync(r.data(), sums.p, sizeof(double) * (size_t)ps, hipMemcpyDeviceToHost, h->stream));
        HUB_HIP(hipStreamSynchronize(h->stream));
        observables_out(h, r.data(), dens, corr, docc);
        return HUBBARD_OK;
    });
}

int hubbard_propagate(hubbard_h h, double *psi_re, double *psi_im, double t, int n_steps, int krylov_dim,
                      double *energy, hubbard_prop_result *res)
{
    return guarded([&]() -> int {
        check_handle(h);
        return propagate_impl(h, psi_re, psi_im, t, n_steps, krylov_dim, energy, res);
    });
}

int hubbard_info(hubbard_h h, hubbard_info_t *info)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (!info)
            fail(HUBBARD_EINVAL, "info is NULL");
        hubbard_info_t r;
        std::memset(&r, 0, sizeof(r));
        r.sites = h->sites;
        r.n_up = h->n_up;
        r.n_dn = h->n_dn;
        r.n_edges = (int32_t)(h->edges.size() / 2);
        r.t = h->t;
        r.U = h->U;
        r.dim_up = h->up.dim;
        r.dim_dn = h->dn.dim;
        r.dim = h->dim;
        r.w_up = h->up.width;
        r.w_dn = h->dn.width;
        r.nnz_up = h->up.nnz;
        r.nnz_dn = h->dn.nnz;
        r.device_bytes = h->dev.bytes;
        const HvPlan pl = make_hv_plan(hv_args(h), h->precision == HUBBARD_FP64 ? 8 : 4);
        r.ld_pref = pl.ld;
        r.vector_bytes = (size_t)h->up.dim * (size_t)pl.ld * (h->precision == HUBBARD_FP64 ? 16 : 8);
        *info = r;
        return HUBBARD_OK;
    });
}

int hubbard_export_basis(hubbard_h h, int spin, uint32_t *states)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (spin != HUBBARD_SPIN_UP && spin != HUBBARD_SPIN_DN)
            fail(HUBBARD_EINVAL, "spin must be 0 (up) or 1 (down)");
        if (!states)
            fail(HUBBARD_EINVAL, "states is NULL");
        const SpinTable &tb = spin == HUBBARD_SPIN_UP ? h->up : h->dn;
        std::memcpy(states, tb.states.data(), tb.states.size() * 4);
        return HUBBARD_OK;
    });
}

int hubbard_export_table(hubbard_h h, int spin, int32_t *col, int8_t *sgn)
{
    return guarded([&]() -> int {
        check_handle(h);
        if (spin != HUBBARD_SPIN_UP && spin != HUBBARD_SPIN_DN)
            fail(HUBBARD_EINVAL, "spin must be 0 (up) or 1 (down)");
        if (!col || !sgn)
            fail(HUBBARD_EINVAL, "col and sgn must not be NULL");
        const SpinTable &tb = spin == HUBBARD_SPIN_UP ? h->up : h->dn;
        std::memcpy(col, tb.col.data(), tb.col.size() * 4);
        std::memcpy(sgn, tb.sgn.data(), tb.sgn.size());
        return HUBBARD_OK;
    });
}

int hubbard_start_raw(uint64_t seed, int64_t dim, double *f, void *hip_stream)
{
    return guarded([&]() -> int {
        if (dim < 0 || (dim > 0 && !f))
            fail(HUBBARD_EINVAL, "bad start-vector arguments");
        if (dim > 0)
            launch_start_raw(seed, f, dim, static_cast<hipStream_t>(hip_stream));
        return HUBBARD_OK;
    });
}

int hubbard_lanczos_batch(hubbard_h *hs, int n, const hubbard_opts *opts, hubbard_result *res)
{
    return guarded([&]() -> int {
        if (n < 0 || (n > 0 && (!hs || !opts || !res)))
            fail(HUBBARD_EINVAL, "bad batch arguments");
        // small sectors without a psi request share launches; the rest run one by one
        std::vector<hubbard *> bh;
        std::vector<hubbard_opts> bo;
        std::vector<int> bidx;
        for (int i = 0; i < n; i++) {
            check_handle(hs[i]);
            validate_opts(opts[i]);
            if (!opts[i].psi && batchable(hs[i], opts[i].precision)) {
                bh.push_back(hs[i]);
                bo.push_back(opts[i]);
                bidx.push_back(i);
            }
        }
        int worst = HUBBARD_OK;
        auto note = [&](int rc) {
            if (rc != HUBBARD_OK && (worst == HUBBARD_OK || rc < worst))
                worst = rc;
        };
        if (!bh.empty()) {
            use_device(bh[0]);
            std::vector<hubbard_result> br(bh.size());
            run_batch(bh.data(), bo.data(), br.data(), (int)bh.size(), bh[0]->stream);
            for (size_t k = 0; k < bidx.size(); k++) {
                res[bidx[k]] = br[k];
                note(br[k].status);
            }
        }
        for (int i = 0; i < n; i++) {
            if (!opts[i].psi && batchable(hs[i], opts[i].precision))
                continue;
            note(lanczos_impl(hs[i], opts[i], &res[i]));
        }
        return worst;
    });
}

const char *hubbard_strerror(int code)
{
    switch (code) {
    case HUBBARD_OK: return "success";
    case HUBBARD_ENOCONV: return "max_iter reached before convergence";
    case HUBBARD_EINVAL: return "invalid argument";
    case HUBBARD_ERANGE: return "sector too large";
    case HUBBARD_ENOMEM: return "out of memory";
    case HUBBARD_EDEVICE: return "device error";
    case HUBBARD_EBUSY: return "busy";
    default: return "unknown error code";
    }
}

const char *hubbard_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
