// libpic host runtime: the C ABI declared in include/libpic.h.  Validates
// arguments on the host, owns the context's device scratch (error flag, box
// and species tables, sort buffers, work-item queue, per-species x^n
// scratch), enqueues every kernel on the context's stream, and records
// whole steps into HIP graphs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "libpic.h"
#include "pic_aux.h"
#include "pic_dev.h"
#include "pic_math.h"

using namespace pic;

// Device memory of pic_energy_noalloc: the per-block partial sums of the
// energy reductions for up to ENERGY_MAX_SPECIES species (144 KiB), one copy
// per GPU, held until the process ends.  Host code never uses this name as
// an address: pic_init looks up each device's copy once
// (hipGetSymbolAddress) and keeps the pointer per device.
static __device__ __align__(256) double scratch[(2 + ENERGY_MAX_SPECIES) * ENERGY_MAX_GRID];

namespace {

thread_local std::string g_last_error;

pic_status fail(pic_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(PIC_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int LDS_BYTES_MAX = 160 * 1024 - 256;   // leave room for static LDS
constexpr int RANK_BITS = 4;                      // ranks of the rank-major order (0..15)

int halo_gl(int o) { return o == 1 ? 1 : (o == 2 ? 1 : 2); }
int halo_gh(int o) { return o == 1 ? 1 : 2; }
int halo_jl(int o) { return o == 1 ? 1 : 2; }
int halo_jh(int o) { return o == 1 ? 2 : 3; }

struct Slot {
    long long cap = 0;          // particles the scratch below can hold
    int prec_bytes = 0;
    double *xo[3] = {nullptr, nullptr, nullptr};
    int *cello = nullptr;
    float *offo[3] = {nullptr, nullptr, nullptr};
    int *carry = nullptr;
    int *strag = nullptr;       // straggler list of the tiled kernels (np entries)
    long long strag_cap = 0;
    int *tile_off = nullptr;
    int tile_cap = 0;
    // state of the last binding
    const void *key_ptr = nullptr;
    long long np = -1;
    int box = -1;
    bool sorted = false;
    bool pushed = false;
};

template <typename T> pic_status dalloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(PIC_ERR_OOM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    return PIC_OK;
}

template <typename T> void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

}  // namespace

struct pic_ctx {
    int nboxes = 0;
    int order = 1;
    pic_precision prec = PIC_FP64;
    hipStream_t stream = nullptr;
    pic_tuning tun{};
    int cus = 256;
    std::vector<DevBox> hbox;
    DevBox *dbox = nullptr;
    std::vector<long long> hfp;     // flat cell prefix over boxes
    long long *dfp = nullptr;
    long long total_cells = 0;
    int *derr = nullptr;
    size_t lds_field_bytes = 0, lds_bytes = 0;
    int margin[3] = {0, 0, 0};      // cells staged around each tile, per axis
    int jrow = 0;                   // padded row length of the LDS current tile (0 = none)
    int frow = 0;                   // padded row length of the LDS field tile (0 = none)
    int falign = 0;                 // field rows aligned to 16 bytes (16-byte copies)
    int lane_swz = 0;               // swap lane bits 4 and 5 (16-wide rows, padded FP32 field)
    // species
    std::vector<Slot> slots;
    std::vector<DevSpecies> hsp;    // last uploaded table
    DevSpecies *dsp = nullptr;
    int dsp_cap = 0;
    std::vector<int> hprefix;
    int *dprefix = nullptr;
    int nslots = 0;                 // (species, tile) slots of the tiled form
    // species of each box (CSR) and the boxes' tile-count prefix: the
    // box-tile slots the batched form builds its work items over
    std::vector<int> hbox_sp_off, hbox_sp;
    int *dbox_sp_off = nullptr, *dbox_sp = nullptr;
    int *dbprefix = nullptr;
    int nbslots = 0;
    // sort scratch
    long long sort_cap = 0;
    int *sort_tot = nullptr;        // 2 device ints of the quads-first pass
    int *keys[2] = {nullptr, nullptr};
    int *vals[2] = {nullptr, nullptr};
    void *tmp = nullptr;
    int *counts = nullptr;
    int *scan_scr = nullptr;
    size_t counts_cap = 0, scan_cap = 0;
    // batched work items
    Item *items = nullptr;
    long long items_cap = 0;
    int *item_counts = nullptr, *item_starts = nullptr;
    int item_slot_cap = 0;
    int *nitems = nullptr, *queue = nullptr;
    int *strag_count = nullptr;     // per species, capacity dsp_cap
    int dims = 0;                   // 3 or 2 if every box has it, else 0
    // graphs
    std::map<std::string, hipGraphExec_t> graphs;
    // optional timing of the tiled particle kernel (also inside graphs):
    // device wall-clock stamps written just before and after it
    bool timing = false, timed = false;
    long long *stamps = nullptr;    // 2 device values
    int clock_khz = 0;
    bool capturing = false;
    hipStream_t cap_stream = nullptr;   // private stream graphs are recorded on
    // partial sums of pic_energy; this device's copy of `scratch`
    double *energy_part = nullptr;
    double *noalloc_part = nullptr;
    size_t energy_cap = 0;
    // z-slab particle migration: direction flags and their prefixes (6 x
    // mig_cap ints), scan scratch, per-species totals (3 each) and per
    // species staging / send arrays
    int *mig_flags = nullptr;
    long long mig_cap = 0;
    int *mig_scan = nullptr;
    size_t mig_scan_cap = 0;
    int *mig_tot = nullptr;
    int mig_tot_cap = 0;
    struct MigStore {
        MigBuffers b{};
        long long cap[3] = {0, 0, 0};     // stay, down, up
        int na = 0, esize = 0;
    };
    std::vector<MigStore> mig_store;
    // electrostatic solve: rhs, r, p, Ap, ones (es_cap doubles each),
    // per-block partial sums and scalars
    double *es_vec = nullptr;
    long long es_cap = 0;
    double *es_part = nullptr, *es_sc = nullptr;
};

namespace {

int key_bits(int nkeys) {
    int b = 0;
    while ((1ll << b) < (long long)nkeys) ++b;
    return b < 1 ? 1 : b;
}

// Captured step graphs hold the addresses of the context's scratch buffers.
// Every site that frees or reallocates one of them (after waiting for the
// stream) drops the cached graphs, so none is ever replayed on freed memory;
// the next pic_step records afresh.
void drop_graphs(pic_ctx *c) {
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// Address of this device's copy of `scratch`; looked up once per device,
// with that device current.
pic_status noalloc_scratch(int dev, double **out) {
    *out = nullptr;
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PIC_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PIC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return PIC_OK;
}

pic_status check_box(const pic_box_desc &b, int i) {
    std::string w = "box " + std::to_string(i) + ": ";
    if (b.dim != 2 && b.dim != 3) return fail(PIC_ERR_ARG, w + "dim must be 2 or 3");
    if (b.order < 1 || b.order > 3) return fail(PIC_ERR_ARG, w + "order must be 1..3");
    long long nc = 1;
    for (int d = 0; d < 3; ++d) {
        if (b.n[d] < 1 || b.n[d] >= (1 << 20)) return fail(PIC_ERR_ARG, w + "n out of range");
        if (b.tile[d] < 1 || b.tile[d] > 16) return fail(PIC_ERR_ARG, w + "tile must be 1..16");
        if (!(b.dx[d] > 0.0) || !std::isfinite(b.dx[d])) return fail(PIC_ERR_ARG, w + "dx must be > 0");
        nc *= b.n[d];
    }
    if (nc >= (1ll << 31)) return fail(PIC_ERR_ARG, w + "more than 2^31-1 cells");
    if (b.dim == 2 && (b.n[1] != 1 || b.tile[1] != 1))
        return fail(PIC_ERR_ARG, w + "2D boxes need n[1] == 1 and tile[1] == 1");
    if (!(b.dt > 0.0) || !std::isfinite(b.dt)) return fail(PIC_ERR_ARG, w + "dt must be > 0");
    if (b.cell_base < 0) return fail(PIC_ERR_ARG, w + "cell_base < 0");
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (b.dim == 2 && d == 1) continue;
        s += 1.0 / (b.dx[d] * b.dx[d]);
    }
    if (b.dt * std::sqrt(s) > 1.0 + 1e-12)
        return fail(PIC_ERR_CFL, w + "dt above the Courant limit 1/sqrt(sum 1/dx^2)");
    return PIC_OK;
}

pic_status ensure_slot_scratch(pic_ctx *c, Slot &sl, long long np) {
    const int pb = c->prec == PIC_FP64 ? 8 : 4;
    if (sl.cap >= np && sl.prec_bytes == pb) return PIC_OK;
    drop_graphs(c);
    for (int d = 0; d < 3; ++d) { dfree(sl.xo[d]); dfree(sl.offo[d]); }
    dfree(sl.cello);
    dfree(sl.carry);
    pic_status s;
    if (c->prec == PIC_FP64) {
        for (int d = 0; d < 3; ++d)
            if ((s = dalloc(&sl.xo[d], (size_t)np)) != PIC_OK) return s;
    } else {
        for (int d = 0; d < 3; ++d)
            if ((s = dalloc(&sl.offo[d], (size_t)np)) != PIC_OK) return s;
        if ((s = dalloc(&sl.cello, (size_t)np)) != PIC_OK) return s;
        if ((s = dalloc(&sl.carry, (size_t)np)) != PIC_OK) return s;
    }
    sl.cap = np;
    sl.prec_bytes = pb;
    return PIC_OK;
}

pic_status validate_species(pic_ctx *c, const pic_species *sp, int nsp) {
    if (nsp < 0) return fail(PIC_ERR_ARG, "nsp < 0");
    if (nsp > 0 && !sp) return fail(PIC_ERR_ARG, "species array is NULL");
    for (int s = 0; s < nsp; ++s) {
        const pic_species &p = sp[s];
        std::string w = "species " + std::to_string(s) + ": ";
        if (p.box < 0 || p.box >= c->nboxes) return fail(PIC_ERR_ARG, w + "box index out of range");
        if (p.np < 0 || p.np >= (1ll << 31)) return fail(PIC_ERR_ARG, w + "np out of range");
        if (!(p.m > 0.0) || !std::isfinite(p.q) || !std::isfinite(p.m))
            return fail(PIC_ERR_ARG, w + "bad q or m");
        if (p.np == 0) continue;
        const bool two = c->hbox[p.box].dim == 2;
        for (int d = 0; d < 3; ++d)
            if (!p.u[d]) return fail(PIC_ERR_ARG, w + "u pointer is NULL");
        if (!p.w) return fail(PIC_ERR_ARG, w + "w pointer is NULL");
        if (c->prec == PIC_FP64) {
            for (int d = 0; d < 3; ++d)
                if (!(two && d == 1) && !p.x[d]) return fail(PIC_ERR_ARG, w + "x pointer is NULL");
        } else {
            if (!p.cell) return fail(PIC_ERR_ARG, w + "cell pointer is NULL");
            for (int d = 0; d < 3; ++d)
                if (!(two && d == 1) && !p.off[d]) return fail(PIC_ERR_ARG, w + "off pointer is NULL");
        }
    }
    return PIC_OK;
}

// Arguments of the energy reductions: validated on the host without any
// device call; species of other boxes get np = 0 (energy 0).
pic_status energy_args(pic_ctx *c, const pic_fields *f, const pic_species *sp, int nsp, int box,
                       const double *out, EnergySp *es) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (box < 0 || box >= c->nboxes || !out) return fail(PIC_ERR_ARG, "bad box or out");
    if (nsp > ENERGY_MAX_SPECIES)
        return fail(PIC_ERR_ARG, "energy reductions take at most " +
                                     std::to_string(ENERGY_MAX_SPECIES) + " species");
    if (!f) return fail(PIC_ERR_ARG, "fields is NULL");
    for (int d = 0; d < 3; ++d)
        if (!f->E[d] || !f->B[d]) return fail(PIC_ERR_ARG, "E/B pointer is NULL");
    pic_status st = validate_species(c, sp, nsp);
    if (st != PIC_OK) return st;
    for (int s = 0; s < nsp; ++s) {
        es[s].np = sp[s].box == box ? sp[s].np : 0;
        es[s].m = sp[s].m;
        for (int d = 0; d < 3; ++d) es[s].u[d] = sp[s].u[d];
        es[s].w = sp[s].w;
    }
    return PIC_OK;
}

// Upload the species table when the binding changed; (re)size per-species
// scratch.  need_push_scratch: also allocate the x^n scratch.
pic_status bind_species(pic_ctx *c, const pic_species *sp, int nsp, bool need_push_scratch) {
    pic_status st = validate_species(c, sp, nsp);
    if (st != PIC_OK) return st;
    if ((int)c->slots.size() < nsp) c->slots.resize(nsp);
    std::vector<DevSpecies> t(nsp);
    std::vector<int> prefix(nsp + 1, 0);
    for (int s = 0; s < nsp; ++s) {
        const pic_species &p = sp[s];
        Slot &sl = c->slots[s];
        const DevBox &b = c->hbox[p.box];
        const void *kp = c->prec == PIC_FP64 ? (const void *)p.x[0] : (const void *)p.cell;
        if (sl.key_ptr != kp || sl.np != p.np || sl.box != p.box) {
            sl.sorted = false;
            sl.pushed = false;
        }
        sl.key_ptr = kp;
        sl.np = p.np;
        sl.box = p.box;
        if (need_push_scratch && sl.cap < p.np) {
            if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
            (void)hipStreamSynchronize(c->stream);
            if ((st = ensure_slot_scratch(c, sl, p.np)) != PIC_OK) return st;
        }
        if (sl.tile_cap < b.ntiles + 2) {
            if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
            (void)hipStreamSynchronize(c->stream);
            drop_graphs(c);
            dfree(sl.tile_off);
            if ((st = dalloc(&sl.tile_off, (size_t)b.ntiles + 2)) != PIC_OK) return st;
            sl.tile_cap = b.ntiles + 2;
            sl.sorted = false;
        }
        if (c->tun.kernel != PIC_KERNEL_DIRECT && sl.strag_cap < p.np) {
            if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
            (void)hipStreamSynchronize(c->stream);
            drop_graphs(c);
            dfree(sl.strag);
            if ((st = dalloc(&sl.strag, (size_t)p.np)) != PIC_OK) return st;
            sl.strag_cap = p.np;
        }
        DevSpecies &d = t[s];
        std::memset(&d, 0, sizeof(d));
        d.np = p.np;
        d.q = p.q;
        d.m = p.m;
        d.box = p.box;
        d.tile_base = prefix[s];
        for (int k = 0; k < 3; ++k) {
            d.x[k] = p.x[k];
            d.off[k] = p.off[k];
            d.u[k] = p.u[k];
            d.xo[k] = sl.xo[k];
            d.offo[k] = sl.offo[k];
        }
        d.cell = p.cell;
        d.w = p.w;
        d.cello = sl.cello;
        d.carry = sl.carry;
        d.strag = sl.strag;
        d.tile_off = sl.tile_off;
        d.pusher = c->tun.pusher;
        d.galerkin = c->tun.gather;
        d.spread = c->tun.quad_spread > 0 ||
                   (c->tun.quad_spread == 0 && p.np >= 6 * c->hbox[p.box].ncells);
        prefix[s + 1] = prefix[s] + b.ntiles;
    }
    bool same = (int)c->hsp.size() == nsp &&
                (nsp == 0 || std::memcmp(c->hsp.data(), t.data(), nsp * sizeof(DevSpecies)) == 0);
    if (!same) {
        if (c->capturing) return fail(PIC_ERR_STATE, "species binding changed during graph capture");
        (void)hipStreamSynchronize(c->stream);
        if (c->dsp_cap < nsp + 1) {
            drop_graphs(c);
            dfree(c->dsp);
            dfree(c->dprefix);
            dfree(c->strag_count);
            dfree(c->dbox_sp);
            c->hbox_sp.clear();
            c->hbox_sp_off.clear();
            int cap = nsp + 8;
            if ((st = dalloc(&c->dsp, (size_t)cap)) != PIC_OK) return st;
            if ((st = dalloc(&c->dprefix, (size_t)cap + 1)) != PIC_OK) return st;
            if ((st = dalloc(&c->strag_count, (size_t)cap)) != PIC_OK) return st;
            if ((st = dalloc(&c->dbox_sp, (size_t)cap)) != PIC_OK) return st;
            c->dsp_cap = cap;
        }
        if (nsp > 0) {
            HIP_TRY(hipMemcpy(c->dsp, t.data(), nsp * sizeof(DevSpecies), hipMemcpyHostToDevice));
        }
        HIP_TRY(hipMemcpy(c->dprefix, prefix.data(), (nsp + 1) * sizeof(int), hipMemcpyHostToDevice));
        c->hsp = t;
        c->hprefix = prefix;
    }
    c->nslots = prefix[nsp];
    std::vector<int> bso(c->nboxes + 1, 0), bsl(std::max(nsp, 1), 0);
    for (int s = 0; s < nsp; ++s) ++bso[sp[s].box + 1];
    for (int b = 0; b < c->nboxes; ++b) bso[b + 1] += bso[b];
    {
        std::vector<int> fill(bso.begin(), bso.end() - 1);
        for (int s = 0; s < nsp; ++s) bsl[fill[sp[s].box]++] = s;
    }
    bsl.resize(nsp);
    if (bso != c->hbox_sp_off || bsl != c->hbox_sp) {
        if (c->capturing) return fail(PIC_ERR_STATE, "species binding changed during graph capture");
        (void)hipStreamSynchronize(c->stream);
        HIP_TRY(hipMemcpy(c->dbox_sp_off, bso.data(), (c->nboxes + 1) * sizeof(int), hipMemcpyHostToDevice));
        if (nsp > 0) HIP_TRY(hipMemcpy(c->dbox_sp, bsl.data(), nsp * sizeof(int), hipMemcpyHostToDevice));
        c->hbox_sp_off = bso;
        c->hbox_sp = bsl;
    }
    return PIC_OK;
}

KParams make_params(pic_ctx *c, const pic_fields *f, int nsp) {
    KParams k;
    std::memset(&k, 0, sizeof(k));
    k.boxes = c->dbox;
    k.species = c->dsp;
    k.nsp = nsp;
    if (f) {
        for (int d = 0; d < 3; ++d) {
            k.f.E[d] = f->E[d];
            k.f.B[d] = f->B[d];
            k.f.J[d] = f->J[d];
        }
    }
    k.err = c->derr;
    k.sp_tile_prefix = c->dprefix;
    k.items = c->items;
    k.nitems = c->nitems;
    k.queue = c->queue;
    k.lds_field_bytes = (int)c->lds_field_bytes;
    k.lane_stride = c->tun.lane_stride;
    // DPP quad pooling needs whole groups of four of one cell in a row
    k.quad = c->tun.lane_stride <= 1 && c->tun.cell_order == 2;
    for (int d = 0; d < 3; ++d) k.margin[d] = c->margin[d];
    k.jrow = c->jrow;
    k.frow = c->frow;
    k.falign = c->falign;
    k.lane_swz = c->lane_swz;
    k.strag_count = c->strag_count;
    k.box_sp_off = c->dbox_sp_off;
    k.box_sp = c->dbox_sp;
    return k;
}

#define PIC_UNITS(F, N) {{F##_o##N##_p0_t0, F##_o##N##_p0_t1, F##_o##N##_p0_t2}, \
                        {F##_o##N##_p1_t0, F##_o##N##_p1_t1, F##_o##N##_p1_t2}}
// [order - 1][precision][part] (parts as in pic_aux.h)
const ParticleLauncher k_launch[3][2][3] = {PIC_UNITS(launch_particles, 1),
                                            PIC_UNITS(launch_particles, 2),
                                            PIC_UNITS(launch_particles, 3)};
const LdsLimiter k_lds_limit[3][2][3] = {PIC_UNITS(particles_lds_limit, 1),
                                         PIC_UNITS(particles_lds_limit, 2),
                                         PIC_UNITS(particles_lds_limit, 3)};
#undef PIC_UNITS
const RhoLauncher k_rho_launch[3][2] = {{launch_rho_o1_p0_t0, launch_rho_o1_p1_t0},
                                        {launch_rho_o2_p0_t0, launch_rho_o2_p1_t0},
                                        {launch_rho_o3_p0_t0, launch_rho_o3_p1_t0}};

// form: 0 direct, 1 tiled, 2 batched (persistent), 3 stragglers of 1/2.
hipError_t launch_particles(pic_ctx *c, const KParams &k, int form, int mode, int grid,
                            int species) {
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    const int part = (mode == MODE_FUSED && (form == 1 || form == 2)) ? form : 0;
    return k_launch[c->order - 1][prec][part](k, form, mode, c->dims, grid, c->tun.block,
                                             c->lds_bytes, species, c->stream);
}

pic_status check_fields(pic_ctx *c, const pic_fields *f, bool need_eb) {
    if (!f) return fail(PIC_ERR_ARG, "fields is NULL");
    for (int d = 0; d < 3; ++d) {
        if (!f->J[d]) return fail(PIC_ERR_ARG, "J pointer is NULL");
        if (need_eb && (!f->E[d] || !f->B[d])) return fail(PIC_ERR_ARG, "E/B pointer is NULL");
    }
    (void)c;
    return PIC_OK;
}

pic_status run_particles(pic_ctx *c, pic_fields *f, pic_species *sp, int nsp, int mode) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    pic_status st = check_fields(c, f, (mode & MODE_PUSH) != 0);
    if (st != PIC_OK) return st;
    if ((st = bind_species(c, sp, nsp, mode == MODE_PUSH || mode == MODE_DEPOSIT)) != PIC_OK) return st;
    const int form = c->tun.kernel;
    for (int s = 0; s < nsp; ++s) {
        Slot &sl = c->slots[s];
        if (form != PIC_KERNEL_DIRECT && !sl.sorted && sp[s].np > 0)
            return fail(PIC_ERR_STATE, "tiled kernels need pic_sort_tiles first (species " +
                                           std::to_string(s) + ")");
        if (mode == MODE_DEPOSIT && !sl.pushed && sp[s].np > 0)
            return fail(PIC_ERR_STATE, "pic_deposit_J without a preceding pic_gather_push");
    }
    KParams k = make_params(c, f, nsp);
    if (mode & MODE_DEPOSIT)
        HIP_TRY(launch_zero_j(k.f, c->dbox, c->dfp, c->nboxes, c->total_cells, c->stream));
    if (form == PIC_KERNEL_DIRECT) {
        for (int s = 0; s < nsp; ++s) {
            if (sp[s].np == 0) continue;
            int grid = (int)((sp[s].np + 255) / 256);
            HIP_TRY(launch_particles(c, k, 0, mode, grid, s));
        }
    } else {
        HIP_TRY(launch_zero_ints(c->strag_count, nsp, c->stream));
        if (form == PIC_KERNEL_BATCHED) HIP_TRY(launch_set_int(c->queue, 0, c->stream));
        if (c->timing) HIP_TRY(launch_stamp(c->stamps, c->stream));
        if (form == PIC_KERNEL_TILED) {
            if (c->nslots > 0) HIP_TRY(launch_particles(c, k, 1, mode, c->nslots, 0));
        } else {
            int grid = c->cus * c->tun.wg_per_cu;
            HIP_TRY(launch_particles(c, k, 2, mode, grid, 0));
        }
        // particles that had left their tile plus margin since the sort
        HIP_TRY(launch_particles(c, k, 3, mode, c->cus * 2, 0));
        if (c->timing) {
            HIP_TRY(launch_stamp(c->stamps + 1, c->stream));
            c->timed = true;
        }
    }
    for (int s = 0; s < nsp; ++s) {
        if (mode == MODE_PUSH) c->slots[s].pushed = true;
        else c->slots[s].pushed = false;
    }
    return PIC_OK;
}

pic_status ensure_sort_scratch(pic_ctx *c, long long np, long long nitems_cap) {
    pic_status st;
    if (c->sort_cap < np) {
        if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
        (void)hipStreamSynchronize(c->stream);
        drop_graphs(c);
        for (int i = 0; i < 2; ++i) { dfree(c->keys[i]); dfree(c->vals[i]); }
        if (c->tmp) { (void)hipFree(c->tmp); c->tmp = nullptr; }
        for (int i = 0; i < 2; ++i) {
            if ((st = dalloc(&c->keys[i], (size_t)np)) != PIC_OK) return st;
            if ((st = dalloc(&c->vals[i], (size_t)np)) != PIC_OK) return st;
        }
        if (hipMalloc(&c->tmp, (size_t)std::max<long long>(np, 1) * PERM_GROUP_BYTES) != hipSuccess) {
            c->tmp = nullptr;
            return fail(PIC_ERR_OOM, "sort buffer allocation failed");
        }
        c->sort_cap = np;
    }
    size_t need_counts = (size_t)radix_blocks(np) * 256 + 256;
    size_t need_scan = std::max(scan_scratch_ints((long long)need_counts),
                                scan_scratch_ints((long long)c->nbslots + 1));
    if (c->tun.cell_order == 2 || c->tun.cell_order == 4)
        need_scan = std::max(need_scan, scan_scratch_ints(np));
    if (c->counts_cap < need_counts) {
        if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
        (void)hipStreamSynchronize(c->stream);
        drop_graphs(c);
        dfree(c->counts);
        if ((st = dalloc(&c->counts, need_counts)) != PIC_OK) return st;
        c->counts_cap = need_counts;
    }
    if (c->scan_cap < need_scan) {
        if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
        (void)hipStreamSynchronize(c->stream);
        drop_graphs(c);
        dfree(c->scan_scr);
        if ((st = dalloc(&c->scan_scr, need_scan)) != PIC_OK) return st;
        c->scan_cap = need_scan;
    }
    if (c->tun.kernel == PIC_KERNEL_BATCHED) {
        if (c->item_slot_cap < c->nbslots + 1) {
            if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
            (void)hipStreamSynchronize(c->stream);
            drop_graphs(c);
            dfree(c->item_counts);
            dfree(c->item_starts);
            int cap = c->nbslots + 64;
            if ((st = dalloc(&c->item_counts, (size_t)cap)) != PIC_OK) return st;
            if ((st = dalloc(&c->item_starts, (size_t)cap)) != PIC_OK) return st;
            c->item_slot_cap = cap;
        }
        if (c->items_cap < nitems_cap) {
            if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
            (void)hipStreamSynchronize(c->stream);
            drop_graphs(c);
            dfree(c->items);
            if ((st = dalloc(&c->items, (size_t)nitems_cap)) != PIC_OK) return st;
            c->items_cap = nitems_cap;
        }
    }
    return PIC_OK;
}

pic_status do_sort(pic_ctx *c, const pic_species *sp, int nsp, int32_t *const *perm_out,
                   int32_t *const *key_out, int32_t *const *off_out) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    pic_status st = bind_species(c, sp, nsp, false);
    if (st != PIC_OK) return st;
    long long maxnp = 0, nitems_cap = c->nslots + 1;
    for (int s = 0; s < nsp; ++s) {
        if (c->slots[s].pushed) return fail(PIC_ERR_STATE, "sort between pic_gather_push and pic_deposit_J");
        maxnp = std::max(maxnp, (long long)sp[s].np);
        nitems_cap += (sp[s].np + c->tun.chunk - 1) / c->tun.chunk;
    }
    if ((st = ensure_sort_scratch(c, maxnp, nitems_cap)) != PIC_OK) return st;
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    hipStream_t S = c->stream;
    for (int s = 0; s < nsp; ++s) {
        const pic_species &p = sp[s];
        const DevBox &b = c->hbox[p.box];
        const long long np = p.np;
        const int nkeys = b.ntiles + 1;
        Slot &sl = c->slots[s];
        // cell bits of the within-tile order (0: tile id only)
        // (cell_order 1/2 add two class bits; 3 orders by cell alone)
        int cb = 0;
        const int classes = (c->tun.cell_order == 3 || c->tun.cell_order == 4) ? 0 : 1;
        const int vol = b.tile[0] * (b.dim == 3 ? b.tile[1] : 1) * b.tile[2];
        if (c->tun.cell_order) {
            cb = key_bits(vol);
            if (key_bits(nkeys) + cb + 2 * classes > 31) cb = 0;
        }
        const int shift = cb ? cb + 2 * classes : 0;
        // rank-major with tiles of at most RM_MAXV cells: the radix passes
        // sort by tile only (from bit cb up) and one wave per tile orders
        // its particles
        const bool rm_tiles = cb && c->tun.cell_order == 4 && vol <= RM_MAXV;
        const int lo = rm_tiles ? cb : 0;
        HIP_TRY(launch_tile_keys(prec, c->dsp, s, np, c->dbox, cb, classes, c->keys[0], c->vals[0],
                                 c->derr, S));
        const int passes = (key_bits(nkeys) + shift - lo + 7) / 8;
        int cur = 0;
        for (int ps = 0; ps < passes; ++ps) {
            HIP_TRY(radix_pass(c->keys[cur], c->vals[cur], c->keys[1 - cur], c->vals[1 - cur], np,
                               lo + 8 * ps, c->counts, c->scan_scr, S));
            cur = 1 - cur;
        }
        const int *perm = c->vals[cur];
        int kshift = shift;
        if (rm_tiles) {
            HIP_TRY(launch_tile_offsets(c->keys[cur], np, nkeys, cb, sl.tile_off, S));
            HIP_TRY(rank_major_tiles(c->keys[cur], c->vals[cur], sl.tile_off, nkeys, cb, vol,
                                     c->keys[1 - cur], c->vals[1 - cur], S));
            perm = c->vals[1 - cur];
        } else if (cb && c->tun.cell_order == 4) {
            // rank-major: (tile, rank in cell) keys, then stable passes over
            // them (ties stay in cell order)
            int *heads = (int *)c->tmp, *starts = heads + np;
            HIP_TRY(rank_keys(c->keys[cur], np, cb, RANK_BITS, heads, starts, c->keys[1 - cur],
                              c->sort_tot, c->scan_scr, S));
            HIP_TRY(launch_copy4(c->vals[cur], c->vals[1 - cur], np, S));
            cur = 1 - cur;
            const int passes2 = (key_bits(nkeys) + RANK_BITS + 7) / 8;
            for (int ps = 0; ps < passes2; ++ps) {
                HIP_TRY(radix_pass(c->keys[cur], c->vals[cur], c->keys[1 - cur], c->vals[1 - cur], np,
                                   8 * ps, c->counts, c->scan_scr, S));
                cur = 1 - cur;
            }
            perm = c->vals[cur];
            kshift = RANK_BITS;
        }
        if (!rm_tiles) HIP_TRY(launch_tile_offsets(c->keys[cur], np, nkeys, kshift, sl.tile_off, S));
        if (cb && c->tun.cell_order == 2) {
            HIP_TRY(quads_first(c->keys[cur], c->vals[cur], np, shift, sl.tile_off, c->keys[1 - cur],
                                (int *)c->tmp, c->vals[1 - cur], c->sort_tot, c->scan_scr, S));
            perm = c->vals[1 - cur];
        }
        // permute the particle arrays in place, in groups that share one
        // read of perm, through the tmp buffer
        const bool two = b.dim == 2;
        if (np > 0) {
            void *arr[8];
            int na = 0;
            if (c->prec == PIC_FP64) {
                for (int d = 0; d < 3; ++d) if (!(two && d == 1)) arr[na++] = p.x[d];
            } else {
                arr[na++] = p.cell;
                for (int d = 0; d < 3; ++d) if (!(two && d == 1)) arr[na++] = p.off[d];
            }
            for (int d = 0; d < 3; ++d) arr[na++] = p.u[d];
            arr[na++] = p.w;
            HIP_TRY(launch_permute(c->prec == PIC_FP64 ? 8 : 4, arr, na, perm, c->tmp, np, S));
        }
        if (perm_out && perm_out[s]) HIP_TRY(launch_copy4(perm, perm_out[s], np, S));
        if (key_out && key_out[s]) HIP_TRY(launch_shift_copy(c->keys[cur], key_out[s], np, kshift, S));
        if (off_out && off_out[s]) HIP_TRY(launch_copy4(sl.tile_off, off_out[s], b.ntiles + 1, S));
        sl.sorted = true;
    }
    if (c->tun.kernel == PIC_KERNEL_BATCHED && c->nbslots > 0) {
        HIP_TRY(launch_items(c->dsp, c->dbprefix, c->nboxes, c->dbox_sp_off, c->dbox_sp, c->nbslots,
                             c->tun.chunk, c->item_counts,
                             c->item_starts, c->scan_scr, c->items, c->nitems, c->queue, S));
    }
    return PIC_OK;
}

pic_status do_fdtd(pic_ctx *c, pic_fields *f) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    pic_status st = check_fields(c, f, true);
    if (st != PIC_OK) return st;
    KParams k = make_params(c, f, 0);
    HIP_TRY(launch_fdtd(c->prec == PIC_FP64 ? 0 : 1, k.f, c->dbox, c->dfp, c->nboxes,
                        c->total_cells, c->stream));
    return PIC_OK;
}

// ---------------------------------------------------------------- z slabs

pic_status slab_check(pic_ctx *c, int g) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (g < 3) return fail(PIC_ERR_ARG, "slab guard must be >= 3 layers");
    const DevBox &b0 = c->hbox[0];
    for (int s = 0; s < c->nboxes; ++s) {
        const DevBox &b = c->hbox[s];
        if (b.dim != b0.dim || b.n[0] != b0.n[0] || b.n[1] != b0.n[1] || b.dt != b0.dt ||
            b.dx[0] != b0.dx[0] || b.dx[1] != b0.dx[1] || b.dx[2] != b0.dx[2])
            return fail(PIC_ERR_ARG, "slab boxes must share dim, nx, ny, dx and dt");
        if (b.n[2] - 2 * g < 2 * g)
            return fail(PIC_ERR_ARG, "slab " + std::to_string(s) + ": interior of " +
                                         std::to_string(b.n[2] - 2 * g) + " layers < 2 x guard");
    }
    return PIC_OK;
}

// Arrays of one species as migration sees them (NULL arrays of 2D left out).
MigSpecies mig_species(pic_ctx *c, const pic_species &p) {
    MigSpecies m{};
    m.np = p.np;
    m.zi = -1;
    auto add = [&](void *a) { if (a) m.a[m.na++] = a; };
    if (c->prec == PIC_FP64) {
        add(p.x[0]);
        add(p.x[1]);
        m.zi = m.na;
        add(p.x[2]);
    } else {
        add(p.cell);
        add(p.off[0]);
        add(p.off[1]);
        add(p.off[2]);
    }
    add(p.u[0]);
    add(p.u[1]);
    add(p.u[2]);
    add(p.w);
    return m;
}

pic_status mig_flags_and_scans(pic_ctx *c, const MigSpecies &m, int g, int nzs, int nxy, int *tot) {
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    const long long n = c->mig_cap;
    int *st = c->mig_flags, *dn = st + n, *up = dn + n;
    int *pst = up + n, *pdn = pst + n, *pup = pdn + n;
    HIP_TRY(launch_mig_flags(prec, m, g, nzs, nxy, st, dn, up, c->stream));
    HIP_TRY(scan_exclusive(st, pst, m.np, tot, c->mig_scan, c->stream));
    HIP_TRY(scan_exclusive(dn, pdn, m.np, tot + 1, c->mig_scan, c->stream));
    HIP_TRY(scan_exclusive(up, pup, m.np, tot + 2, c->mig_scan, c->stream));
    return PIC_OK;
}

pic_status grow_buffer(void **p, long long &cap, long long need, size_t esize) {
    if (cap >= need) return PIC_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    if (hipMalloc(p, (size_t)std::max<long long>(need, 1) * esize) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(PIC_ERR_OOM, "migration buffer allocation failed");
    }
    cap = need;
    return PIC_OK;
}

pic_status slab_migrate(pic_ctx *c, pic_species *sp, int nsp, int g, const int64_t *cap,
                        int64_t *np_out) {
    pic_status st = slab_check(c, g);
    if (st != PIC_OK) return st;
    if (c->capturing) return fail(PIC_ERR_STATE, "pic_slab_migrate cannot be captured");
    const int nslab = c->nboxes;
    if (nsp < 1 || nsp % nslab) return fail(PIC_ERR_ARG, "nsp must be a multiple of the slab count");
    if (!cap || !np_out) return fail(PIC_ERR_ARG, "cap or np_out is NULL");
    const int nkind = nsp / nslab;
    for (int i = 0; i < nsp; ++i) {
        if (sp[i].box != i / nkind) return fail(PIC_ERR_ARG, "species must be given slab-major (box == i / kinds)");
        if (sp[i].np > cap[i]) return fail(PIC_ERR_ARG, "species count above its capacity");
        if (cap[i] >= (1ll << 31)) return fail(PIC_ERR_ARG, "capacity out of range");
    }
    if ((st = validate_species(c, sp, nsp)) != PIC_OK) return st;
    const int nxy = c->hbox[0].n[0] * c->hbox[0].n[1];
    long long maxnp = 1;
    for (int i = 0; i < nsp; ++i) maxnp = std::max(maxnp, (long long)sp[i].np);
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->mig_cap < maxnp) {
        drop_graphs(c);
        dfree(c->mig_flags);
        c->mig_cap = 0;
        if ((st = dalloc(&c->mig_flags, (size_t)maxnp * 6)) != PIC_OK) return st;
        c->mig_cap = maxnp;
    }
    const size_t need_scan = scan_scratch_ints(maxnp);
    if (c->mig_scan_cap < need_scan) {
        dfree(c->mig_scan);
        c->mig_scan_cap = 0;
        if ((st = dalloc(&c->mig_scan, need_scan)) != PIC_OK) return st;
        c->mig_scan_cap = need_scan;
    }
    if (c->mig_tot_cap < 3 * nsp) {
        dfree(c->mig_tot);
        c->mig_tot_cap = 0;
        if ((st = dalloc(&c->mig_tot, (size_t)3 * nsp)) != PIC_OK) return st;
        c->mig_tot_cap = 3 * nsp;
    }
    if ((int)c->mig_store.size() < nsp) c->mig_store.resize(nsp);
    std::vector<MigSpecies> ms(nsp);
    const size_t esize = c->prec == PIC_FP64 ? 8 : 4;
    // counts of stayers and leavers of every species
    for (int i = 0; i < nsp; ++i) {
        ms[i] = mig_species(c, sp[i]);
        const int nzs = c->hbox[sp[i].box].n[2] - 2 * g;
        if ((st = mig_flags_and_scans(c, ms[i], g, nzs, nxy, c->mig_tot + 3 * i)) != PIC_OK) return st;
    }
    std::vector<int> tot(3 * nsp);
    HIP_TRY(hipMemcpyAsync(tot.data(), c->mig_tot, tot.size() * sizeof(int), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int i = 0; i < nsp; ++i)
        if (sp[i].np == 0) tot[3 * i] = tot[3 * i + 1] = tot[3 * i + 2] = 0;
    auto lower = [&](int i) { const int s = i / nkind; return ((s + nslab - 1) % nslab) * nkind + i % nkind; };
    auto upper = [&](int i) { const int s = i / nkind; return ((s + 1) % nslab) * nkind + i % nkind; };
    std::vector<long long> nnew(nsp);
    for (int i = 0; i < nsp; ++i) {
        nnew[i] = (long long)tot[3 * i] + tot[3 * lower(i) + 2] + tot[3 * upper(i) + 1];
        if (nnew[i] > cap[i])
            return fail(PIC_ERR_ARG, "species " + std::to_string(i) + ": " + std::to_string(nnew[i]) +
                                         " particles after migration exceed its capacity");
    }
    // staging / send arrays
    for (int i = 0; i < nsp; ++i) {
        auto &S = c->mig_store[i];
        if (S.na != ms[i].na || S.esize != (int)esize) {
            for (int a = 0; a < MIG_ARRAYS; ++a) {
                if (S.b.stay[a]) (void)hipFree(S.b.stay[a]);
                if (S.b.down[a]) (void)hipFree(S.b.down[a]);
                if (S.b.up[a]) (void)hipFree(S.b.up[a]);
            }
            S = pic_ctx::MigStore{};
            S.na = ms[i].na;
            S.esize = (int)esize;
        }
        for (int k = 0; k < 3; ++k) {
            const long long need = tot[3 * i + k];
            if (S.cap[k] >= need) continue;
            for (int a = 0; a < S.na; ++a) {
                void **bp = k == 0 ? &S.b.stay[a] : (k == 1 ? &S.b.down[a] : &S.b.up[a]);
                long long cp = S.cap[k];
                if ((st = grow_buffer(bp, cp, need, esize)) != PIC_OK) return st;
            }
            S.cap[k] = need;
        }
    }
    // leavers out, stayers compacted
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    for (int i = 0; i < nsp; ++i) {
        if (sp[i].np == 0) continue;
        const int nzs = c->hbox[sp[i].box].n[2] - 2 * g;
        const int nzp = c->hbox[sp[lower(i)].box].n[2] - 2 * g;
        if ((st = mig_flags_and_scans(c, ms[i], g, nzs, nxy, c->mig_tot + 3 * i)) != PIC_OK) return st;
        const long long n = c->mig_cap;
        const int *fs = c->mig_flags;
        HIP_TRY(launch_mig_scatter(prec, ms[i], fs, fs + n, fs + 2 * n, fs + 3 * n, fs + 4 * n,
                                   fs + 5 * n, c->mig_store[i].b, nzp, nzs, nxy, c->stream));
    }
    // stayers, then arrivals from below and from above
    for (int i = 0; i < nsp; ++i) {
        MigSpecies m = ms[i];
        m.np = nnew[i];
        HIP_TRY(launch_mig_gather(prec, m, tot[3 * i], c->mig_store[i].b, tot[3 * lower(i) + 2],
                                  c->mig_store[lower(i)].b, tot[3 * upper(i) + 1],
                                  c->mig_store[upper(i)].b, c->stream));
        np_out[i] = nnew[i];
    }
    return PIC_OK;
}

// ---------------------------------------------------------------- boundaries

pic_status ensure_mig_scratch(pic_ctx *c, long long maxnp, int nsp) {
    pic_status st;
    if (c->mig_cap < maxnp) {
        drop_graphs(c);
        dfree(c->mig_flags);
        c->mig_cap = 0;
        if ((st = dalloc(&c->mig_flags, (size_t)maxnp * 6)) != PIC_OK) return st;
        c->mig_cap = maxnp;
    }
    const size_t need_scan = scan_scratch_ints(maxnp);
    if (c->mig_scan_cap < need_scan) {
        dfree(c->mig_scan);
        c->mig_scan_cap = 0;
        if ((st = dalloc(&c->mig_scan, need_scan)) != PIC_OK) return st;
        c->mig_scan_cap = need_scan;
    }
    if (c->mig_tot_cap < 3 * nsp) {
        dfree(c->mig_tot);
        c->mig_tot_cap = 0;
        if ((st = dalloc(&c->mig_tot, (size_t)3 * nsp)) != PIC_OK) return st;
        c->mig_tot_cap = 3 * nsp;
    }
    if ((int)c->mig_store.size() < nsp) c->mig_store.resize(nsp);
    return PIC_OK;
}

pic_status ensure_mig_store(pic_ctx *c, int i, int na, size_t esize, int kind, long long need) {
    auto &S = c->mig_store[i];
    if (S.na != na || S.esize != (int)esize) {
        for (int a = 0; a < MIG_ARRAYS; ++a) {
            if (S.b.stay[a]) (void)hipFree(S.b.stay[a]);
            if (S.b.down[a]) (void)hipFree(S.b.down[a]);
            if (S.b.up[a]) (void)hipFree(S.b.up[a]);
        }
        S = pic_ctx::MigStore{};
        S.na = na;
        S.esize = (int)esize;
    }
    if (S.cap[kind] >= need) return PIC_OK;
    for (int a = 0; a < S.na; ++a) {
        void **bp = kind == 0 ? &S.b.stay[a] : (kind == 1 ? &S.b.down[a] : &S.b.up[a]);
        long long cp = S.cap[kind];
        pic_status st = grow_buffer(bp, cp, need, esize);
        if (st != PIC_OK) return st;
    }
    S.cap[kind] = need;
    return PIC_OK;
}

pic_status window_shift(pic_ctx *c, pic_fields *f, pic_species *sp, int nsp, int box,
                        const pic_species *inj, const int64_t *cap, int64_t *np_out) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (c->capturing) return fail(PIC_ERR_STATE, "pic_window_shift cannot be captured");
    if (box < 0 || box >= c->nboxes) return fail(PIC_ERR_ARG, "bad box");
    if (!cap || !np_out || (nsp > 0 && !inj)) return fail(PIC_ERR_ARG, "cap, np_out or inject is NULL");
    pic_status st = check_fields(c, f, true);
    if (st != PIC_OK) return st;
    if ((st = validate_species(c, sp, nsp)) != PIC_OK) return st;
    for (int i = 0; i < nsp; ++i) {
        if (sp[i].box != box) continue;
        if (inj[i].np < 0 || sp[i].np > cap[i] || cap[i] >= (1ll << 31))
            return fail(PIC_ERR_ARG, "bad count or capacity (species " + std::to_string(i) + ")");
        if (inj[i].np > 0) {
            pic_species t = inj[i];
            t.box = box;
            if ((st = validate_species(c, &t, 1)) != PIC_OK) return st;
        }
    }
    DevBox &hb = c->hbox[box];
    const int nz = hb.n[2], nxy = hb.n[0] * hb.n[1];
    const int k = ((hb.zoff % nz) + nz) % nz;       // array layer leaving the frame
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    long long maxnp = 1;
    for (int i = 0; i < nsp; ++i) maxnp = std::max(maxnp, (long long)sp[i].np);
    HIP_TRY(hipStreamSynchronize(c->stream));
    if ((st = ensure_mig_scratch(c, maxnp, std::max(nsp, 1))) != PIC_OK) return st;
    void *comps[6] = {f->E[0], f->E[1], f->E[2], f->B[0], f->B[1], f->B[2]};
    HIP_TRY(launch_zero_layer(prec, comps, c->dbox, box, nxy, k, c->stream));
    hb.zoff = (k + 1) % nz;
    HIP_TRY(launch_box_zoff(c->dbox, box, hb.zoff, c->stream));
    std::vector<MigSpecies> ms(std::max(nsp, 1));
    for (int i = 0; i < nsp; ++i) {
        np_out[i] = sp[i].np;
        if (sp[i].box != box) continue;
        ms[i] = mig_species(c, sp[i]);
        HIP_TRY(launch_win_flags(prec, ms[i], k, nxy, c->mig_flags, c->stream));
        HIP_TRY(scan_exclusive(c->mig_flags, c->mig_flags + c->mig_cap, sp[i].np, c->mig_tot + 3 * i,
                               c->mig_scan, c->stream));
        if (sp[i].np == 0) continue;
        // the compaction needs this species' flags and positions now
        std::vector<int> one(1);
        HIP_TRY(hipMemcpyAsync(one.data(), c->mig_tot + 3 * i, sizeof(int), hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        const long long nstay = one[0];
        const long long n = nstay + inj[i].np;
        if (n > cap[i])
            return fail(PIC_ERR_ARG, "species " + std::to_string(i) + ": " + std::to_string(n) +
                                         " particles after the shift exceed its capacity");
        const size_t esize = c->prec == PIC_FP64 ? 8 : 4;
        if ((st = ensure_mig_store(c, i, ms[i].na, esize, 0, std::max(nstay, 1ll))) != PIC_OK) return st;
        HIP_TRY(launch_win_compact(prec, ms[i], c->mig_flags, c->mig_flags + c->mig_cap,
                                   c->mig_store[i].b, c->stream));
        MigSpecies in = mig_species(c, inj[i]);
        in.np = inj[i].np;
        MigSpecies out = ms[i];
        out.np = n;
        HIP_TRY(launch_win_fill(prec, out, nstay, c->mig_store[i].b, in, hb.zoff, nz, nxy,
                                c->stream));
        np_out[i] = n;
    }
    // species with np == 0 before the shift: only the injected particles
    for (int i = 0; i < nsp; ++i) {
        if (sp[i].box != box || sp[i].np != 0 || inj[i].np == 0) continue;
        if (inj[i].np > cap[i]) return fail(PIC_ERR_ARG, "injected particles exceed the capacity");
        MigSpecies in = mig_species(c, inj[i]);
        in.np = inj[i].np;
        MigSpecies out = mig_species(c, sp[i]);
        out.np = inj[i].np;
        HIP_TRY(launch_win_fill(prec, out, 0, c->mig_store[0].b, in, hb.zoff, nz, nxy, c->stream));
        np_out[i] = inj[i].np;
    }
    return PIC_OK;
}

// ---------------------------------------------------------------- electrostatic

pic_status es_solve(pic_ctx *c, const pic_species *sp, int nsp, int box, pic_fields *f, double *phi,
                    double tol, int max_iter, int32_t *iters_out, double *res_out) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (c->capturing) return fail(PIC_ERR_STATE, "pic_es_solve cannot be captured");
    if (box < 0 || box >= c->nboxes || !phi) return fail(PIC_ERR_ARG, "bad box or phi");
    if (!(tol > 0.0) || max_iter < 1) return fail(PIC_ERR_ARG, "tol must be > 0 and max_iter >= 1");
    pic_status st = check_fields(c, f, true);
    if (st != PIC_OK) return st;
    if ((st = bind_species(c, sp, nsp, false)) != PIC_OK) return st;
    const long long n = c->hbox[box].ncells;
    if (c->es_cap < n) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        dfree(c->es_vec);
        c->es_cap = 0;
        if ((st = dalloc(&c->es_vec, (size_t)n * 5)) != PIC_OK) return st;
        c->es_cap = n;
        std::vector<double> one(n, 1.0);
        HIP_TRY(hipMemcpy(c->es_vec + 4 * n, one.data(), n * sizeof(double), hipMemcpyHostToDevice));
    }
    if (!c->es_part) {
        if ((st = dalloc(&c->es_part, (size_t)ES_DOT_GRID)) != PIC_OK) return st;
        if ((st = dalloc(&c->es_sc, 8)) != PIC_OK) return st;
    }
    const long long cap = c->es_cap;
    double *b = c->es_vec, *r = b + cap, *p = r + cap, *ap = p + cap, *ones = ap + cap;
    double *part = c->es_part, *sc = c->es_sc;
    hipStream_t S = c->stream;
    // rhs: rho of the box's species, mean removed
    HIP_TRY(launch_zero_d(b, n, S));
    KParams k = make_params(c, f, nsp);
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    for (int s = 0; s < nsp; ++s) {
        if (sp[s].box != box || sp[s].np == 0) continue;
        HIP_TRY(k_rho_launch[c->order - 1][prec](k, s, sp[s].np, b, S));
    }
    HIP_TRY(launch_remove_mean(b, n, part, sc + 4, ones, S));
    // conjugate gradients on -lap phi = b from phi = 0
    HIP_TRY(launch_zero_d(phi, n, S));
    HIP_TRY(launch_copy_d(b, r, n, S));
    HIP_TRY(launch_copy_d(b, p, n, S));
    HIP_TRY(launch_dot(r, r, n, part, sc, S));
    double bb = 0.0;
    HIP_TRY(hipMemcpyAsync(&bb, sc, sizeof(double), hipMemcpyDeviceToHost, S));
    HIP_TRY(hipStreamSynchronize(S));
    int it = 0;
    double rr = bb;
    if (bb > 0.0) {
        while (it < max_iter) {
            HIP_TRY(launch_neg_lap(c->dbox, box, n, p, ap, S));
            HIP_TRY(launch_dot(p, ap, n, part, sc + 1, S));
            HIP_TRY(launch_cg_xr(phi, r, p, ap, n, sc, S));
            HIP_TRY(launch_dot(r, r, n, part, sc + 2, S));
            HIP_TRY(launch_cg_p(p, r, n, sc, S));
            HIP_TRY(launch_copy_scalar(sc, 0, 2, S));
            ++it;
            if (it % 16 == 0 || it == max_iter) {
                HIP_TRY(hipMemcpyAsync(&rr, sc, sizeof(double), hipMemcpyDeviceToHost, S));
                HIP_TRY(hipStreamSynchronize(S));
                if (std::sqrt(rr / bb) <= tol) break;
            }
        }
    }
    HIP_TRY(launch_remove_mean(phi, n, part, sc + 4, ones, S));
    HIP_TRY(launch_es_field(prec, c->dbox, box, n, phi, k.f, S));
    if (iters_out) *iters_out = it;
    if (res_out) *res_out = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    if (bb > 0.0 && std::sqrt(rr / bb) > tol)
        return fail(PIC_ERR_STATE, "Poisson solve did not reach the tolerance in max_iter iterations");
    return PIC_OK;
}

pic_status es_push(pic_ctx *c, const pic_fields *f, pic_species *sp, int nsp) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    pic_status st = check_fields(c, f, true);
    if (st != PIC_OK) return st;
    if ((st = bind_species(c, sp, nsp, false)) != PIC_OK) return st;
    for (int s = 0; s < nsp; ++s) c->slots[s].sorted = false;     // positions change
    KParams k = make_params(c, f, nsp);
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    for (int s = 0; s < nsp; ++s)
        HIP_TRY(launch_es_push(c->order, prec, c->dsp, s, sp[s].np, c->dbox, k.f, c->derr, c->stream));
    return PIC_OK;
}

}  // namespace

extern "C" {

const char *pic_status_str(pic_status s) {
    switch (s) {
        case PIC_OK: return "ok";
        case PIC_ERR_ARG: return "invalid argument";
        case PIC_ERR_CFL: return "time step above the Courant limit";
        case PIC_ERR_OOM: return "device out of memory";
        case PIC_ERR_DEVICE: return "HIP runtime error";
        case PIC_ERR_RANGE: return "particle displacement >= 1 cell, or non-finite value";
        case PIC_ERR_STATE: return "call order violated";
    }
    return "unknown status";
}

const char *pic_last_error(void) { return g_last_error.c_str(); }

pic_status pic_init(pic_ctx **out, const pic_box_desc *boxes, int32_t nboxes, pic_precision prec,
                    void *stream, const pic_tuning *tuning) {
    if (!out) return fail(PIC_ERR_ARG, "ctx out-pointer is NULL");
    *out = nullptr;
    if (!boxes || nboxes < 1) return fail(PIC_ERR_ARG, "need at least one box");
    if (prec != PIC_FP64 && prec != PIC_FP32_SPLIT) return fail(PIC_ERR_ARG, "bad precision");
    pic_status st;
    for (int i = 0; i < nboxes; ++i)
        if ((st = check_box(boxes[i], i)) != PIC_OK) return st;
    for (int i = 1; i < nboxes; ++i)
        if (boxes[i].order != boxes[0].order)
            return fail(PIC_ERR_ARG, "all boxes of a context must share one shape order");
    pic_tuning t{};
    t.kernel = prec == PIC_FP64 ? PIC_KERNEL_TILED : PIC_KERNEL_BATCHED;
    t.block = 256;
    t.chunk = 4096;
    t.wg_per_cu = 2;
    t.lane_stride = 1;
    t.pad = 0;
    t.cell_order = 0;
    t.quad_spread = 0;
    t.margin = 0;
    t.pusher = 0;
    t.gather = 0;
    if (tuning) {
        t.kernel = tuning->kernel;
        if (tuning->block) t.block = tuning->block;
        if (tuning->chunk) t.chunk = tuning->chunk;
        if (tuning->wg_per_cu) t.wg_per_cu = tuning->wg_per_cu;
        if (tuning->lane_stride) t.lane_stride = tuning->lane_stride;
        t.pad = tuning->pad;
        t.cell_order = tuning->cell_order;
        t.quad_spread = tuning->quad_spread;
        t.margin = tuning->margin;
        t.pusher = tuning->pusher;
        t.gather = tuning->gather;
    }
    if (t.kernel < 0 || t.kernel > 2) return fail(PIC_ERR_ARG, "bad kernel form");
    const int max_block = prec == PIC_FP64 ? 512 : 1024;
    if (t.block < 64 || t.block > max_block || t.block % 64)
        return fail(PIC_ERR_ARG, "block must be a multiple of 64 in 64..512 (FP64) or 64..1024 (split)");
    if (t.chunk < 1) return fail(PIC_ERR_ARG, "chunk must be >= 1");
    if (t.wg_per_cu < 1 || t.wg_per_cu > 64) return fail(PIC_ERR_ARG, "wg_per_cu must be 1..64");
    if (t.lane_stride < 1 || t.lane_stride > 64) return fail(PIC_ERR_ARG, "lane_stride must be 1..64");
    if (t.cell_order < -1 || t.cell_order > 4) return fail(PIC_ERR_ARG, "cell_order must be -1..4");
    if (t.pad < -1 || t.pad > 2) return fail(PIC_ERR_ARG, "pad must be -1..2");
    if (t.quad_spread < -1 || t.quad_spread > 1) return fail(PIC_ERR_ARG, "quad_spread must be -1..1");
    if (t.margin < -1 || t.margin > 0) return fail(PIC_ERR_ARG, "margin must be -1 or 0");
    if (t.pusher < 0 || t.pusher > 1) return fail(PIC_ERR_ARG, "pusher must be 0 (Boris) or 1 (Vay)");
    if (t.gather < 0 || t.gather > 1) return fail(PIC_ERR_ARG, "gather must be 0 or 1 (Galerkin)");
    t.cell_order = t.cell_order == 0 ? (t.kernel == PIC_KERNEL_BATCHED ? 2 : 0) : std::max(t.cell_order, 0);

    pic_ctx *c = new pic_ctx();
    c->nboxes = nboxes;
    c->order = boxes[0].order;
    c->prec = prec;
    c->stream = (hipStream_t)stream;
    c->tun = t;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete c;
        return fail(PIC_ERR_DEVICE, "no HIP device");
    }
    if ((st = noalloc_scratch(dev, &c->noalloc_part)) != PIC_OK) {
        delete c;
        return st;
    }
    const int o = c->order;
    const size_t fb = prec == PIC_FP64 ? 8 : 4;
    c->hfp.assign(nboxes + 1, 0);
    for (int i = 0; i < nboxes; ++i) {
        const pic_box_desc &b = boxes[i];
        DevBox d;
        std::memset(&d, 0, sizeof(d));
        d.dim = b.dim;
        d.order = b.order;
        d.ncells = 1;
        d.small = 0;
        for (int k = 0; k < 3; ++k) {
            d.n[k] = b.n[k];
            d.tile[k] = b.tile[k];
            d.nt[k] = (b.n[k] + b.tile[k] - 1) / b.tile[k];
            d.dx[k] = b.dx[k];
            d.ncells *= b.n[k];
            const bool active = !(b.dim == 2 && k == 1);
            if (active && b.n[k] < 8) d.small = 1;
        }
        d.ntiles = d.nt[0] * d.nt[1] * d.nt[2];
        d.cell_base = b.cell_base;
        d.dt = b.dt;
        d.inv_nx = 1.0 / (double)b.n[0];
        d.inv_nxy = 1.0 / ((double)b.n[0] * (double)b.n[1]);
        c->hbox.push_back(d);
        c->hfp[i + 1] = c->hfp[i] + d.ncells;
    }
    c->total_cells = c->hfp[nboxes];
    {
        int n3 = 0;
        for (int i = 0; i < nboxes; ++i) n3 += boxes[i].dim == 3;
        c->dims = n3 == nboxes ? 3 : (n3 == 0 ? 2 : 0);
    }
    // LDS layout: a 1-cell margin around every tile (on the axes where it
    // fits), and rows
    // padded (t.pad) so that a wave's lanes, which sit on a block of tile
    // rows, hit distinct LDS banks.
    int tx = 0;
    for (int i = 0; i < nboxes; ++i) tx = std::max(tx, std::min(boxes[i].tile[0], boxes[i].n[0]));
    // LDS serves a wave's access in passes of 128 bytes over 32 banks: 32
    // lanes of a 4-byte access, 16 of an 8-byte one (measured: a 16 x 4
    // block of FP64 slots is conflict-free with rows 23 long, an 8 x 8 one
    // only with rows an odd multiple of 8 modulo 16).  Smallest row >= need
    // that is an odd multiple of w modulo the elements of one pass
    // (per_pass), so that the w-wide rows of a pass fall on distinct banks;
    // need itself when a pass holds one row; 0 if none within 2x need.
    // w = tx for the rows r, r + 1, ... of a pass; a pass of 32 FP32 holds
    // two 16-wide rows, and with the lanes' bits 4 and 5 swapped (lane_swz)
    // these are rows r and r + 2, which w = 8 keeps apart with rows of 24
    // where rows r and r + 1 would need 48.
    auto pad_row = [&](int need, int per_pass, int w) {
        if (w >= per_pass) return need;
        if (w <= 0 || per_pass % w) return 0;
        int row = need;
        while (!((row % per_pass) % w == 0 && ((row % per_pass) / w) % 2 == 1)) ++row;
        return row <= 2 * need ? row : 0;
    };
    // LDS bytes of the field (F) or current (J) stage for a margin per axis
    // and a padded row length (0 = unpadded), max over the boxes.
    // (each field component spans only its own stencil's nodes, by stagger)
    // Field rows from and to multiples of 16 bytes (al = 4 FP32 or 2 FP64
    // nodes), so that the stage is copied 16 bytes a lane: every box's x
    // tile and x size a multiple of al cells and its first cell at a
    // multiple of al in the arrays; the rows are not padded further.
    const int al = 16 / fb;
    bool falign_ok = t.pad == 0;
    for (int i = 0; i < nboxes; ++i)
        falign_ok = falign_ok && boxes[i].tile[0] % al == 0 && boxes[i].n[0] % al == 0 &&
                    boxes[i].cell_base % al == 0;
    bool falign = falign_ok;
    auto stage_bytes = [&](bool field, const int *mg, int row) {
        size_t mx = 0;
        for (int i = 0; i < nboxes; ++i) {
            const pic_box_desc &b = boxes[i];
            size_t by = 0;
            for (int c = 0; c < (field ? 6 : 3); ++c) {
                size_t n = field ? fb : 8;         // FP64 or 64-bit fixed point
                for (int k = 0; k < 3; ++k) {
                    if (b.dim == 2 && k == 1) continue;
                    const int st = comp_stagger(c, k);
                    const int lo = field ? gather_lo(o, st) : halo_jl(o);
                    const int hi = field ? gather_hi(o, st) : halo_jh(o);
                    size_t w = (size_t)(std::min(b.tile[k], b.n[k]) + lo + hi + 2 * mg[k]);
                    if (field && k == 0 && falign)   // [t0 - lo, t0 + te + hi) to multiples of al
                        w = (size_t)(((std::min(b.tile[k], b.n[k]) + hi + mg[k] + al - 1) & -al) +
                                     ((lo + mg[k] + al - 1) & -al));
                    if (k == 0 && row > 0) w = std::max(w, (size_t)row);
                    // J_z's edges along z end one node before the region
                    if (!field && c == 2 && k == 2) w -= 1;
                    n *= w;
                }
                by += n;
            }
            mx = std::max(mx, by);
        }
        return field ? (mx + 15) / 16 * 16 : mx;
    };
    const int fpass = fb == 4 ? 32 : 16;
    auto layout = [&](const int *mg, bool padf, bool padj, int &frow, int &jrow) {
        frow = padf ? pad_row(tx + halo_gl(o) + halo_gh(o) + 2 * mg[0], fpass,
                              tx == 16 && fb == 4 ? 8 : tx) : 0;
        jrow = padj ? pad_row(tx + halo_jl(o) + halo_jh(o) + 2 * mg[0], 16, tx) : 0;
        return stage_bytes(true, mg, frow) + stage_bytes(false, mg, jrow);
    };
    {
        const size_t cap = (size_t)LDS_BYTES_MAX;
        int fr = 0, jr = 0;
        // Margin axes are given up widest tile edge first (a particle leaves
        // a wide tile through that axis least often).
        int ext[3] = {0, 0, 0}, drop[3] = {0, 1, 2};
        for (int i = 0; i < nboxes; ++i)
            for (int k = 0; k < 3; ++k) ext[k] = std::max(ext[k], std::min(boxes[i].tile[k], boxes[i].n[k]));
        std::stable_sort(drop, drop + 3, [&](int a, int b) { return ext[a] > ext[b]; });
        const int m0 = t.margin < 0 ? 0 : 1;
        int mg[3] = {m0, m0, m0};
        // FP32: aligned rows only where they fit with the full margin.
        // FP64 (whose stage rarely holds the margin): the margin axes are
        // given up first without them, then aligned rows where they fit.
        if (falign && (fb == 8 || layout(mg, false, false, fr, jr) > cap)) falign = false;
        for (int i = 0; i < 3 && layout(mg, false, false, fr, jr) > cap; ++i) mg[drop[i]] = 0;
        if (falign_ok && fb == 8) {
            falign = true;
            if (layout(mg, false, false, fr, jr) > cap) falign = false;
        }
        bool padf = false, padj = false;
        if (t.pad >= 0) {
            // pad 0: current rows; 1: field rows, then current rows, each
            // where it fits; 2: both, giving up margin axes if need be
            padj = layout(mg, false, true, fr, jr) <= cap && jr > 0;
            if (t.pad >= 1) {
                if (layout(mg, true, padj, fr, jr) <= cap && fr > 0) padf = true;
                else if (layout(mg, true, false, fr, jr) <= cap && fr > 0) { padf = true; padj = false; }
                if (t.pad == 2 && !(padf && padj)) {
                    int m2[3] = {mg[0], mg[1], mg[2]};
                    for (int i = 0; i < 3; ++i) {
                        m2[drop[i]] = 0;
                        if (layout(m2, true, true, fr, jr) <= cap && fr > 0 && jr > 0) {
                            for (int k = 0; k < 3; ++k) mg[k] = m2[k];
                            padf = padj = true;
                            break;
                        }
                    }
                }
            }
        }
        c->lds_bytes = layout(mg, padf, padj, fr, jr);
        c->frow = fr;
        c->jrow = jr;
        c->falign = falign && fr == 0;
        // FP32 rows of 24 (padded, or aligned to 4 nodes around a 16-wide
        // tile): a half-wave on rows r and r + 2 of a pass is conflict-free
        c->lane_swz = tx == 16 && fb == 4 && (fr > 0 || c->falign);
        for (int k = 0; k < 3; ++k) c->margin[k] = mg[k];
        c->lds_field_bytes = stage_bytes(true, mg, fr);
    }
    if (t.kernel != PIC_KERNEL_DIRECT && c->lds_bytes > (size_t)LDS_BYTES_MAX) {
        delete c;
        return fail(PIC_ERR_ARG, "tile too large: LDS need " + std::to_string(c->lds_bytes) + " bytes");
    }
    if ((st = dalloc(&c->dbox, (size_t)nboxes)) != PIC_OK ||
        (st = dalloc(&c->dfp, (size_t)nboxes + 1)) != PIC_OK ||
        (st = dalloc(&c->derr, 4)) != PIC_OK || (st = dalloc(&c->nitems, 4)) != PIC_OK ||
        (st = dalloc(&c->queue, 4)) != PIC_OK ||
        (st = dalloc(&c->dbox_sp_off, (size_t)nboxes + 1)) != PIC_OK ||
        (st = dalloc(&c->dbprefix, (size_t)nboxes + 1)) != PIC_OK ||
        (st = dalloc(&c->sort_tot, 4)) != PIC_OK) {
        pic_free(c);
        return st;
    }
    {
        std::vector<int> bp(nboxes + 1, 0);
        for (int i = 0; i < nboxes; ++i) bp[i + 1] = bp[i] + c->hbox[i].ntiles;
        c->nbslots = bp[nboxes];
        if (hipMemcpy(c->dbprefix, bp.data(), (nboxes + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
            pic_free(c);
            return fail(PIC_ERR_DEVICE, "upload of box tables failed");
        }
    }
    if (hipMemcpy(c->dbox, c->hbox.data(), nboxes * sizeof(DevBox), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->dfp, c->hfp.data(), (nboxes + 1) * sizeof(long long), hipMemcpyHostToDevice) != hipSuccess) {
        pic_free(c);
        return fail(PIC_ERR_DEVICE, "upload of box tables failed");
    }
    int zero[4] = {0, 0, 0, 0};
    if (hipMemcpy(c->derr, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->nitems, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->queue, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) {
        pic_free(c);
        return fail(PIC_ERR_DEVICE, "init of device flags failed");
    }
    if (t.kernel != PIC_KERNEL_DIRECT) {
        const int precb = prec == PIC_FP64 ? 0 : 1;
        // The limit is per kernel and shared by every context of the process:
        // set it to the largest stage any context may use, so a later context
        // with a smaller stage cannot lower it below an earlier one's need.
        hipError_t e = hipSuccess;
        for (int part = 0; part < 3 && e == hipSuccess; ++part)
            e = k_lds_limit[o - 1][precb][part](LDS_BYTES_MAX);
        if (e != hipSuccess) {
            pic_free(c);
            return fail(PIC_ERR_DEVICE, std::string("LDS limit: ") + hipGetErrorString(e));
        }
    }
    *out = c;
    return PIC_OK;
}

pic_status pic_sort_tiles(pic_ctx *c, const pic_species *sp, int32_t nsp, int32_t *const *perm_out,
                          int32_t *const *key_out, int32_t *const *tile_offset_out) {
    return do_sort(c, sp, nsp, perm_out, key_out, tile_offset_out);
}

pic_status pic_gather_push(pic_ctx *c, const pic_fields *f, pic_species *sp, int32_t nsp) {
    return run_particles(c, const_cast<pic_fields *>(f), sp, nsp, MODE_PUSH);
}

pic_status pic_deposit_J(pic_ctx *c, pic_fields *f, pic_species *sp, int32_t nsp) {
    return run_particles(c, f, sp, nsp, MODE_DEPOSIT);
}

pic_status pic_advance(pic_ctx *c, pic_fields *f, pic_species *sp, int32_t nsp) {
    return run_particles(c, f, sp, nsp, MODE_FUSED);
}

pic_status pic_fdtd_step(pic_ctx *c, pic_fields *f) { return do_fdtd(c, f); }

pic_status pic_step(pic_ctx *c, pic_fields *f, pic_species *sp, int32_t nsp, int32_t sort) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    pic_status st = check_fields(c, f, true);
    if (st != PIC_OK) return st;
    if ((st = bind_species(c, sp, nsp, false)) != PIC_OK) return st;
    if (c->tun.kernel != PIC_KERNEL_DIRECT && !sort) {
        for (int s = 0; s < nsp; ++s)
            if (!c->slots[s].sorted && sp[s].np > 0)
                return fail(PIC_ERR_STATE, "tiled kernels need a sort before the first step");
    }
    // key: fields, species table, sort flag
    std::string key((const char *)f, sizeof(pic_fields));
    key.append((const char *)c->hsp.data(), c->hsp.size() * sizeof(DevSpecies));
    key.push_back(sort ? 'S' : 'N');
    key.push_back(c->timing ? 'T' : 'U');
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        // size every scratch buffer before capture starts
        long long maxnp = 0, nitems_cap = c->nslots + 1;
        for (int s = 0; s < nsp; ++s) {
            maxnp = std::max(maxnp, (long long)sp[s].np);
            nitems_cap += (sp[s].np + c->tun.chunk - 1) / c->tun.chunk;
        }
        if (sort && (st = ensure_sort_scratch(c, maxnp, nitems_cap)) != PIC_OK) return st;
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipGraphExec_t ex = nullptr;
        hipGraph_t g = nullptr;
        hipStream_t user = c->stream;
        HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        c->stream = c->cap_stream;
        c->capturing = true;
        const bool prev_timed = c->timed;
        pic_status s1 = PIC_OK;
        if (sort) s1 = do_sort(c, sp, nsp, nullptr, nullptr, nullptr);
        if (s1 == PIC_OK) s1 = run_particles(c, f, sp, nsp, MODE_FUSED);
        if (s1 == PIC_OK) s1 = do_fdtd(c, f);
        c->capturing = false;
        c->stream = user;
        c->timed = prev_timed;       // nothing has run yet
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (s1 != PIC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s1;
        }
        if (e != hipSuccess) return fail(PIC_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(PIC_ERR_DEVICE, std::string("instantiate: ") + hipGetErrorString(e));
        it = c->graphs.emplace(key, ex).first;
    } else {
        // capture bookkeeping done at record time; mirror its effect
        for (int s = 0; s < nsp; ++s) {
            if (sort) c->slots[s].sorted = true;
            c->slots[s].pushed = false;
        }
    }
    HIP_TRY(hipGraphLaunch(it->second, c->stream));
    if (c->timing) c->timed = true;
    return PIC_OK;
}

pic_status pic_deposit_rho(pic_ctx *c, const pic_species *sp, int32_t nsp, int32_t box, double *rho) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (box < 0 || box >= c->nboxes || !rho) return fail(PIC_ERR_ARG, "bad box or rho");
    pic_status st = bind_species(c, sp, nsp, false);
    if (st != PIC_OK) return st;
    KParams k = make_params(c, nullptr, nsp);
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    for (int s = 0; s < nsp; ++s) {
        if (sp[s].box != box || sp[s].np == 0) continue;
        hipError_t e = k_rho_launch[c->order - 1][prec](k, s, sp[s].np, rho, c->stream);
        HIP_TRY(e);
    }
    return PIC_OK;
}

pic_status pic_div_edge(pic_ctx *c, int32_t box, double *const v[3], double *out) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (box < 0 || box >= c->nboxes || !v || !out || !v[0] || !v[1] || !v[2])
        return fail(PIC_ERR_ARG, "bad box or pointers");
    HIP_TRY(launch_div_edge(c->dbox, box, c->hbox[box].ncells, v, out, c->stream));
    return PIC_OK;
}

pic_status pic_energy(pic_ctx *c, const pic_fields *f, const pic_species *sp, int32_t nsp,
                      int32_t box, double *out) {
    EnergySp es[ENERGY_MAX_SPECIES];
    pic_status st = energy_args(c, f, sp, nsp, box, out, es);
    if (st != PIC_OK) return st;
    const size_t need = energy_scratch_doubles(nsp);
    if (c->energy_cap < need) {
        if (c->capturing) return fail(PIC_ERR_STATE, "scratch growth during graph capture");
        HIP_TRY(hipStreamSynchronize(c->stream));
        dfree(c->energy_part);
        if ((st = dalloc(&c->energy_part, need)) != PIC_OK) return st;
        c->energy_cap = need;
    }
    KParams k = make_params(c, f, 0);
    HIP_TRY(launch_energy(c->prec == PIC_FP64 ? 0 : 1, k.f, c->dbox, box, c->hbox[box].ncells, es,
                          nsp, c->energy_part, out, c->stream));
    return PIC_OK;
}

pic_status pic_energy_noalloc(pic_ctx *c, const pic_fields *f, const pic_species *sp,
                              int32_t nsp, int32_t box, double *out) {
    EnergySp es[ENERGY_MAX_SPECIES];
    pic_status st = energy_args(c, f, sp, nsp, box, out, es);
    if (st != PIC_OK) return st;
    if (!c->noalloc_part) return fail(PIC_ERR_STATE, "no device scratch for this context");
    DevFields df;
    for (int d = 0; d < 3; ++d) {
        df.E[d] = f->E[d];
        df.B[d] = f->B[d];
        df.J[d] = f->J[d];
    }
    HIP_TRY(launch_energy(c->prec == PIC_FP64 ? 0 : 1, df, c->dbox, box, c->hbox[box].ncells, es,
                          nsp, c->noalloc_part, out, c->stream));
    return PIC_OK;
}

pic_status pic_slab_fill_guards(pic_ctx *c, pic_fields *f, int32_t guard) {
    pic_status st = slab_check(c, guard);
    if (st != PIC_OK) return st;
    if ((st = check_fields(c, f, true)) != PIC_OK) return st;
    void *comps[6] = {f->E[0], f->E[1], f->E[2], f->B[0], f->B[1], f->B[2]};
    const long long nxy = (long long)c->hbox[0].n[0] * c->hbox[0].n[1];
    HIP_TRY(launch_slab_fill(c->prec == PIC_FP64 ? 0 : 1, comps, 6, c->dbox, c->nboxes, guard, nxy,
                             c->stream));
    return PIC_OK;
}

pic_status pic_slab_reduce_j(pic_ctx *c, pic_fields *f, int32_t guard) {
    pic_status st = slab_check(c, guard);
    if (st != PIC_OK) return st;
    if ((st = check_fields(c, f, false)) != PIC_OK) return st;
    const long long nxy = (long long)c->hbox[0].n[0] * c->hbox[0].n[1];
    HIP_TRY(launch_slab_sum_j(f->J, c->dbox, c->nboxes, guard, nxy, c->stream));
    void *comps[3] = {f->J[0], f->J[1], f->J[2]};
    HIP_TRY(launch_slab_fill(0, comps, 3, c->dbox, c->nboxes, guard, nxy, c->stream));
    return PIC_OK;
}

pic_status pic_slab_migrate(pic_ctx *c, pic_species *sp, int32_t nsp, int32_t guard,
                            const int64_t *cap, int64_t *np_out) {
    return slab_migrate(c, sp, nsp, guard, cap, np_out);
}

pic_status pic_set_absorber(pic_ctx *c, int32_t box, int32_t cells, double sigma_max,
                            int32_t power) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (box < 0 || box >= c->nboxes) return fail(PIC_ERR_ARG, "bad box");
    DevBox &b = c->hbox[box];
    if (cells < 0 || 2 * cells > b.n[2]) return fail(PIC_ERR_ARG, "absorber cells must be 0..n_z/2");
    if (!(sigma_max >= 0.0) || !std::isfinite(sigma_max)) return fail(PIC_ERR_ARG, "bad sigma_max");
    if (power < 0 || power > 8) return fail(PIC_ERR_ARG, "absorber power must be 0..8");
    if (c->capturing) return fail(PIC_ERR_STATE, "pic_set_absorber cannot be captured");
    b.abs_cells = cells;
    b.abs_sigma = sigma_max;
    b.abs_power = power;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->dbox + box, &b, sizeof(DevBox), hipMemcpyHostToDevice));
    return PIC_OK;
}

pic_status pic_antenna_add(pic_ctx *c, pic_fields *f, int32_t box, const pic_antenna *an, double t) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (box < 0 || box >= c->nboxes || !an) return fail(PIC_ERR_ARG, "bad box or antenna");
    pic_status st = check_fields(c, f, false);
    if (st != PIC_OK) return st;
    const DevBox &b = c->hbox[box];
    if (an->k < 0 || an->k >= b.n[2]) return fail(PIC_ERR_ARG, "antenna layer outside the box");
    if (!(an->tau > 0.0) || !(an->waist > 0.0)) return fail(PIC_ERR_ARG, "antenna tau and waist must be > 0");
    AntennaArgs a;
    a.k = an->k; a.E0 = an->E0; a.omega = an->omega; a.waist = an->waist;
    a.x0 = an->x0; a.y0 = an->y0; a.t0 = an->t0; a.tau = an->tau;
    HIP_TRY(launch_antenna(f->J[0], c->dbox, box, (long long)b.n[0] * b.n[1], a, t, c->stream));
    return PIC_OK;
}

pic_status pic_window_shift(pic_ctx *c, pic_fields *f, pic_species *sp, int32_t nsp, int32_t box,
                            const pic_species *inject, const int64_t *cap, int64_t *np_out) {
    return window_shift(c, f, sp, nsp, box, inject, cap, np_out);
}

pic_status pic_window_offset(pic_ctx *c, int32_t box, int32_t *zoff) {
    if (!c || !zoff) return fail(PIC_ERR_ARG, "ctx or zoff is NULL");
    if (box < 0 || box >= c->nboxes) return fail(PIC_ERR_ARG, "bad box");
    *zoff = c->hbox[box].zoff;
    return PIC_OK;
}

pic_status pic_es_solve(pic_ctx *c, const pic_species *sp, int32_t nsp, int32_t box, pic_fields *f,
                        double *phi, double tol, int32_t max_iter, int32_t *iters_out,
                        double *res_out) {
    return es_solve(c, sp, nsp, box, f, phi, tol, max_iter, iters_out, res_out);
}

pic_status pic_es_push(pic_ctx *c, const pic_fields *f, pic_species *sp, int32_t nsp) {
    return es_push(c, f, sp, nsp);
}

pic_status pic_slice_moments(pic_ctx *c, const pic_species *sp, int32_t nsp, int32_t box,
                             double *out) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (box < 0 || box >= c->nboxes || !out) return fail(PIC_ERR_ARG, "bad box or out");
    pic_status st = bind_species(c, sp, nsp, false);
    if (st != PIC_OK) return st;
    const long long nz = c->hbox[box].n[2];
    HIP_TRY(launch_zero_doubles(out, 5 * nz * nsp, c->stream));
    const int prec = c->prec == PIC_FP64 ? 0 : 1;
    for (int s = 0; s < nsp; ++s) {
        if (sp[s].box != box) continue;
        HIP_TRY(launch_slice_moments(prec, c->dsp, s, sp[s].np, c->dbox, out + 5 * nz * s, c->stream));
    }
    return PIC_OK;
}

pic_status pic_check(pic_ctx *c) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, c->derr, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        HIP_TRY(launch_set_int(c->derr, 0, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return fail(PIC_ERR_RANGE, "a particle moved >= 1 cell in a step, or a value was not finite");
    }
    return PIC_OK;
}

pic_status pic_free(pic_ctx *c) {
    if (!c) return PIC_OK;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    dfree(c->stamps);
    dfree(c->energy_part);
    dfree(c->mig_flags);
    dfree(c->mig_scan);
    dfree(c->mig_tot);
    dfree(c->es_vec);
    dfree(c->es_part);
    dfree(c->es_sc);
    for (auto &ms : c->mig_store)
        for (int a = 0; a < MIG_ARRAYS; ++a) {
            if (ms.b.stay[a]) (void)hipFree(ms.b.stay[a]);
            if (ms.b.down[a]) (void)hipFree(ms.b.down[a]);
            if (ms.b.up[a]) (void)hipFree(ms.b.up[a]);
        }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto &sl : c->slots) {
        for (int d = 0; d < 3; ++d) { dfree(sl.xo[d]); dfree(sl.offo[d]); }
        dfree(sl.cello);
        dfree(sl.carry);
        dfree(sl.tile_off);
        dfree(sl.strag);
    }
    for (int i = 0; i < 2; ++i) { dfree(c->keys[i]); dfree(c->vals[i]); }
    dfree(c->strag_count);
    if (c->tmp) (void)hipFree(c->tmp);
    dfree(c->counts);
    dfree(c->scan_scr);
    dfree(c->items);
    dfree(c->item_counts);
    dfree(c->item_starts);
    dfree(c->nitems);
    dfree(c->queue);
    dfree(c->dsp);
    dfree(c->dprefix);
    dfree(c->dbox_sp);
    dfree(c->dbox_sp_off);
    dfree(c->dbprefix);
    dfree(c->sort_tot);
    dfree(c->dbox);
    dfree(c->dfp);
    dfree(c->derr);
    delete c;
    return PIC_OK;
}

int32_t pic_device_cus(pic_ctx *c) { return c ? c->cus : 0; }

pic_status pic_set_timing(pic_ctx *c, int32_t on) {
    if (!c) return fail(PIC_ERR_ARG, "ctx is NULL");
    if (on && !c->stamps) {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&c->clock_khz, hipDeviceAttributeWallClockRate, dev));
        if (c->clock_khz <= 0) return fail(PIC_ERR_DEVICE, "no device wall clock rate");
        pic_status st = dalloc(&c->stamps, 2);
        if (st != PIC_OK) return st;
    }
    c->timing = on != 0;
    c->timed = false;
    return PIC_OK;
}

pic_status pic_kernel_ms(pic_ctx *c, float *ms) {
    if (!c || !ms) return fail(PIC_ERR_ARG, "ctx or ms is NULL");
    if (!c->timed) return fail(PIC_ERR_STATE, "no timed particle kernel since pic_set_timing");
    long long t[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(t, c->stamps, sizeof(t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *ms = (float)((double)(t[1] - t[0]) / (double)c->clock_khz);
    return PIC_OK;
}

}  // extern "C"
