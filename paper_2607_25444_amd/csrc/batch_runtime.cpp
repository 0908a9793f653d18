// batch_runtime.cpp -- host side of the batched step (cac_batch_* in
// include/cac.h): packing of many domains into shared arrays, per-domain
// geometry, work lists and block schedules for the persistent kernels, graph
// replay, per-domain FP64 volumes and the schedule autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "batch_r1.hpp"
#include "../../include/cac.h"
#include "cac_internal.hpp"

namespace cac {
DevParams make_dev_params(const cac_params &p);
Tiling make_tiling(const Grid &g, int bx, int by, int bz);
void build_geometry(const Grid &g, const uint8_t *solid, std::vector<uint32_t> &nbr, std::vector<int32_t> &widx,
                    std::vector<int32_t> &wn6, std::vector<int32_t> &wdonor, int &nskip);
bool valid_params(const cac_params &p);
}  // namespace cac

using namespace cac;

namespace {

struct Schedule {
    int bx = 0, by = 256, bz = 0;  // hydrodynamic tile (bx = 0: per-domain fitted tiles of `by` nodes)
    int phase = 3;                // phase column tile code
    int mult = 2;                 // persistent grid = mult x resident capacity; 0 = one workgroup per item
    int order = 0;                // 0: domains in input order; 1: largest domains first
};

}  // namespace

struct cac_batch {
    int dev = 0, ncu = 0;
    hipStream_t stream = nullptr, cap_stream = nullptr;
    cac_alloc_fn alloc = nullptr;
    void *alloc_user = nullptr;
    std::vector<void *> owned;
    int ndom = 0;
    std::vector<BatchDomain> dom;  // host copy of the descriptors
    std::vector<cac_params> prm;
    uint32_t Ntot = 0, nwall = 0, nptot = 0;
    BatchPtrs B{};
    BatchDomain *d_dom = nullptr;
    float *pstar0 = nullptr;
    double2 *mass_partial = nullptr;
    size_t dom_cap = 0;
    Schedule sch;
    bool use_graph = true;
    uint2 *d_hitems = nullptr, *d_pitems = nullptr;
    size_t hcap = 0, pcap = 0;
    uint32_t nh = 0, np = 0, hgrid = 0, pgrid = 0;
    uint32_t hlds = 0;            // LDS each collide-stream workgroup reserves (occupancy cap)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int cur = 0;
    long long steps = 0;
    int coll = 0;  // collision reading of every domain (cac_params.collision)
    std::string err;
};

namespace {

cac_status bfail(cac_batch *b, cac_status s, const char *fmt, ...)
{
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return s;
}

#define BCHK(b, call)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return bfail(b, CAC_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

void *balloc(cac_batch *b, size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    if (b->alloc) return b->alloc(bytes, b->alloc_user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    b->owned.push_back(p);
    return p;
}

void drop_graphs(cac_batch *b)
{
    for (auto &e : b->gexec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Tile of bx*by*bz = nt nodes fitted to a domain: bx the largest power of two
// (16..128) dividing nx (or the smallest covering it), then y, then z.
void fit_tile(const Grid &g, int nt, int &bx, int &by, int &bz)
{
    bx = 16;
    for (int c = 128; c >= 16; c /= 2)
        if (g.nx % c == 0 && c <= nt) {
            bx = c;
            break;
        }
    if (g.nx % bx != 0)
        while (bx < 64 && bx < g.nx) bx *= 2;
    by = 1;
    while (bx * by * 2 <= nt && by < 4) by *= 2;
    bz = nt / (bx * by);
}

int sched_nt(const Schedule &s) { return s.bx == 0 ? s.by : s.bx * s.by * s.bz; }

// Descriptors and work lists for a schedule; uploads them (synchronously).
// bx = 0 selects per-domain fitted tiles of by nodes ("fit" mode).
cac_status apply_schedule(cac_batch *b, const Schedule &s)
{
    const int nt = sched_nt(s);
    const bool fit = s.bx == 0;
    if (fit ? (nt != 128 && nt != 256 && nt != 512)
            : (!pow2(s.bx) || !pow2(s.by) || !pow2(s.bz) || s.bx < 16 || (nt != 128 && nt != 256 && nt != 512)))
        return bfail(b, CAC_ERR_ARG, "unsupported hydro tile %dx%dx%d", s.bx, s.by, s.bz);
    if (s.phase < 1 || s.phase > 6) return bfail(b, CAC_ERR_ARG, "unsupported phase tile %d", s.phase);
    if (s.mult < 0 || s.mult > 64) return bfail(b, CAC_ERR_ARG, "grid multiplier %d", s.mult);
    int pbx, pby;
    phase_shape_of(s.phase, pbx, pby);
    uint32_t p0 = 0;
    for (int k = 0; k < b->ndom; ++k) {
        BatchDomain &d = b->dom[k];
        int tx = s.bx, ty = s.by, tz = s.bz;
        if (fit) fit_tile(d.g, nt, tx, ty, tz);
        d.t = make_tiling(d.g, tx, ty, tz);
        d.t.phase = s.phase;
        d.pt = phase_tiling(d.g, pbx, pby);
        // the batch supplies the parallelism: whole chunks of up to 32 planes
        // pay the phase kernel's per-chunk prologue least often
        d.pt.zc = std::min(32, d.g.nz);
        d.pt.nzc = (d.g.nz + d.pt.zc - 1) / d.pt.zc;
        d.pt.ntiles = (uint32_t)d.pt.ntx * (uint32_t)d.pt.nty * (uint32_t)d.pt.nzc;
        d.p_item0 = p0;
        p0 += d.pt.ntiles;
    }
    if (p0 > b->nptot) return bfail(b, CAC_ERR_ARG, "phase tiles exceed the partial buffer");
    // item order
    std::vector<int> order(b->ndom);
    std::iota(order.begin(), order.end(), 0);
    if (s.order == 1)
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->dom[a].g.N > b->dom[c].g.N; });
    std::vector<uint2> hi, pi;
    for (int k : order) {
        for (uint32_t t = 0; t < b->dom[k].t.ntiles; ++t) hi.push_back(make_uint2((uint32_t)k, t));
        for (uint32_t t = 0; t < b->dom[k].pt.ntiles; ++t) pi.push_back(make_uint2((uint32_t)k, t));
    }
    if (hi.size() > b->hcap) {
        b->hcap = hi.size() + 1024;
        b->d_hitems = (uint2 *)balloc(b, b->hcap * sizeof(uint2));
        if (!b->d_hitems) return bfail(b, CAC_ERR_ALLOC, "hydro items");
    }
    if (pi.size() > b->pcap) {
        b->pcap = pi.size() + 256;
        b->d_pitems = (uint2 *)balloc(b, b->pcap * sizeof(uint2));
        if (!b->d_pitems) return bfail(b, CAC_ERR_ALLOC, "phase items");
    }
    b->nh = (uint32_t)hi.size();
    b->np = (uint32_t)pi.size();
    b->hlds = hydro_lds_reserve(b->dev, nt);
    const int hb = std::max(1, batch_blocks_per_cu(0, nt, b->hlds));
    const int pb = std::max(1, batch_blocks_per_cu(1, s.phase));
    if (s.mult == 0) {
        b->hgrid = b->nh;
        b->pgrid = b->np;
    } else {
        b->hgrid = std::min<uint32_t>(b->nh, (uint32_t)(s.mult * hb * b->ncu));
        b->pgrid = std::min<uint32_t>(b->np, (uint32_t)(s.mult * pb * b->ncu));
    }
    // persistent grids are multiples of 8 (one share per XCD)
    if (b->hgrid < b->nh) b->hgrid = std::max<uint32_t>(8, b->hgrid & ~7u);
    if (b->pgrid < b->np) b->pgrid = std::max<uint32_t>(8, b->pgrid & ~7u);
    b->hgrid = std::max<uint32_t>(b->hgrid, 1);
    b->pgrid = std::max<uint32_t>(b->pgrid, 1);
    BCHK(b, hipMemcpyAsync(b->d_dom, b->dom.data(), b->ndom * sizeof(BatchDomain), hipMemcpyHostToDevice, b->stream));
    if (b->nh) BCHK(b, hipMemcpyAsync(b->d_hitems, hi.data(), hi.size() * sizeof(uint2), hipMemcpyHostToDevice, b->stream));
    BCHK(b, launch_bitem_walls(b->B, nt, b->d_hitems, b->nh, b->stream));
    if (b->np) BCHK(b, hipMemcpyAsync(b->d_pitems, pi.data(), pi.size() * sizeof(uint2), hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    b->sch = s;
    drop_graphs(b);
    return CAC_OK;
}

// self: the first step of a gradient-form batch (each node pulls its own
// equilibrium); never captured in a graph.
cac_status run_bstep(cac_batch *b, hipStream_t s, bool self = false)
{
    const int c = b->cur;
    const int nt = sched_nt(b->sch);
    BCHK(b, launch_bghost(b->B, b->nwall, c, s));
    if (b->coll) {
        // one workgroup per item whatever the grid multiplier
        if (!self) BCHK(b, launch_br1_rebuild(b->B, b->sch.phase, b->d_pitems, b->np, s));
        BCHK(b, launch_br1_stream(b->B, b->pstar0, nt, b->d_hitems, b->nh, b->hlds, c, self, s));
    } else {
        BCHK(b, launch_bhydro(b->B, nt, b->d_hitems, b->nh, b->hgrid, b->hlds, c, s));
    }
    BCHK(b, launch_bphase(b->B, b->sch.phase, b->d_pitems, b->np, b->pgrid, c, s));
    BCHK(b, launch_bvolume(b->B, nt, b->d_hitems, b->nh, b->hgrid, c ^ 1, s));
    return CAC_OK;
}

cac_status capture(cac_batch *b, int par)
{
    if (!b->cap_stream) BCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    const int save = b->cur;
    b->cur = par;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        b->cur = save;
        return bfail(b, CAC_ERR_HIP, "begin capture: %s", hipGetErrorString(e));
    }
    cac_status st = run_bstep(b, b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &graph);
    b->cur = save;
    if (st != CAC_OK) return st;
    if (e != hipSuccess) return bfail(b, CAC_ERR_HIP, "end capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->gexec[par], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return bfail(b, CAC_ERR_HIP, "instantiate: %s", hipGetErrorString(e));
    return CAC_OK;
}

Fields domain_fields(const cac_batch *b, int k)
{
    const BatchDomain &d = b->dom[k];
    Fields F{};
    F.f[0] = b->B.f[0] + 27ull * d.off;
    F.f[1] = b->B.f[1] + 27ull * d.off;
    F.phi[0] = b->B.phi[0] + d.off;
    F.phi[1] = b->B.phi[1] + d.off;
    F.u = b->B.u + 3ull * d.off;
    F.a = b->B.a + 3ull * d.off;
    F.nbr = b->B.nbr + d.off;
    F.solid = b->B.solid + d.off;
    F.partial = b->mass_partial;
    F.scal = b->B.scal + 8ull * k;
    F.flag = b->B.flag;
    F.pstar0 = b->pstar0 + d.off;
    return F;
}

// Dynamic state (populations of the current parity, both phi buffers, u, a).
size_t state_bytes(const cac_batch *b) { return (size_t)b->Ntot * (27 + 2 + 3 + 3) * sizeof(float); }

cac_status snapshot(cac_batch *b, float *buf, bool save)
{
    const size_t N = b->Ntot;
    struct Part {
        float *p;
        size_t n;
    } parts[] = {{b->coll ? b->B.f[1] : b->B.f[b->cur], 27 * N}, {b->B.phi[0], N}, {b->B.phi[1], N}, {b->B.u, 3 * N},
                 {b->B.a, 3 * N}};
    size_t o = 0;
    for (auto &pt : parts) {
        if (save)
            BCHK(b, hipMemcpyAsync(buf + o, pt.p, pt.n * sizeof(float), hipMemcpyDeviceToDevice, b->stream));
        else
            BCHK(b, hipMemcpyAsync(pt.p, buf + o, pt.n * sizeof(float), hipMemcpyDeviceToDevice, b->stream));
        o += pt.n;
    }
    return CAC_OK;
}

std::string tune_key(const cac_batch *b)
{
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, b->dev);
    std::vector<std::string> sh;
    for (auto &d : b->dom) sh.push_back(std::to_string(d.g.nx) + "x" + std::to_string(d.g.ny) + "x" + std::to_string(d.g.nz));
    std::sort(sh.begin(), sh.end());
    // shape histogram
    std::string key = std::string(prop.gcnArchName) + "|cu" + std::to_string(b->ncu) + "|";
    for (size_t i = 0; i < sh.size();) {
        size_t j = i;
        while (j < sh.size() && sh[j] == sh[i]) ++j;
        key += sh[i] + ":" + std::to_string(j - i) + ",";
        i = j;
    }
    return key;
}

bool cache_lookup(const char *path, const std::string &key, Schedule &s)
{
    if (!path) return false;
    FILE *fp = fopen(path, "r");
    if (!fp) return false;
    char line[4096];
    bool found = false;
    while (fgets(line, sizeof line, fp)) {
        const char *k = strstr(line, "\"key\": \"");
        if (!k) continue;
        k += 8;
        const char *e = strchr(k, '"');
        if (!e || std::string(k, e) != key) continue;
        Schedule t;
        if (sscanf(e, "\", \"bx\": %d, \"by\": %d, \"bz\": %d, \"phase\": %d, \"mult\": %d, \"order\": %d", &t.bx, &t.by,
                   &t.bz, &t.phase, &t.mult, &t.order) == 6) {
            s = t;
            found = true;
        }
    }
    fclose(fp);
    return found;
}

void cache_store(const char *path, const std::string &key, const Schedule &s, double ms)
{
    if (!path) return;
    std::vector<std::string> keep;
    if (FILE *fp = fopen(path, "r")) {
        char line[4096];
        while (fgets(line, sizeof line, fp)) {
            std::string l(line);
            if (l.find("\"key\": \"") == std::string::npos) continue;
            if (l.find("\"key\": \"" + key + "\"") != std::string::npos) continue;
            while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
            keep.push_back(l);
        }
        fclose(fp);
    }
    char buf[4096];
    snprintf(buf, sizeof buf,
             "  {\"key\": \"%s\", \"bx\": %d, \"by\": %d, \"bz\": %d, \"phase\": %d, \"mult\": %d, \"order\": %d, "
             "\"ms_per_step\": %.5f}",
             key.c_str(), s.bx, s.by, s.bz, s.phase, s.mult, s.order, ms);
    keep.push_back(buf);
    FILE *fp = fopen(path, "w");
    if (!fp) return;
    fprintf(fp, "{\"schedules\": [\n");
    for (size_t i = 0; i < keep.size(); ++i) fprintf(fp, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    fprintf(fp, "]}\n");
    fclose(fp);
}

}  // namespace

extern "C" {

cac_status cac_batch_init(cac_batch **bp, int ndom, const cac_domain_desc *d, cac_alloc_fn alloc, void *alloc_user,
                          void *hip_stream)
{
    if (!bp || ndom < 1 || ndom > 65535 || !d) return CAC_ERR_ARG;
    *bp = nullptr;
    unsigned long long Ntot = 0;
    for (int k = 0; k < ndom; ++k) {
        if (d[k].nx < 2 || d[k].ny < 2 || d[k].nz < 2 || !d[k].solid || !d[k].d_phi0 || !valid_params(d[k].params) ||
            d[k].params.collision != d[0].params.collision)
            return CAC_ERR_ARG;
        Ntot += (unsigned long long)d[k].nx * d[k].ny * d[k].nz;
    }
    if (27ull * Ntot >= (1ull << 31)) return CAC_ERR_ARG;
    cac_batch *b = new cac_batch();
    b->stream = (hipStream_t)hip_stream;
    b->alloc = alloc;
    b->alloc_user = alloc_user;
    b->ndom = ndom;
    b->Ntot = (uint32_t)Ntot;
    b->coll = d[0].params.collision;
    auto bail = [&](cac_status st) {
        for (void *q : b->owned) (void)hipFree(q);
        delete b;
        return st;
    };
    if (hipGetDevice(&b->dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->dev) != hipSuccess)
        return bail(CAC_ERR_HIP);
    // descriptors, geometry
    b->dom.resize(ndom);
    b->prm.resize(ndom);
    std::vector<uint32_t> nbr_all(Ntot);
    std::vector<int32_t> widx;
    std::vector<uint8_t> wq;
    std::vector<float> wn, th;
    std::vector<uint16_t> wdom;
    uint32_t off = 0;
    size_t maxN = 0, ptiles = 0;
    for (int k = 0; k < ndom; ++k) {
        BatchDomain &bd = b->dom[k];
        bd.g.nx = d[k].nx;
        bd.g.ny = d[k].ny;
        bd.g.nz = d[k].nz;
        bd.g.N = (uint32_t)d[k].nx * d[k].ny * d[k].nz;
        bd.g.nxny = (uint32_t)d[k].nx * d[k].ny;
        bd.p = make_dev_params(d[k].params);
        bd.off = off;
        b->prm[k] = d[k].params;
        std::vector<uint32_t> nbr;
        std::vector<int32_t> wi, w6, wd;
        int nskip = 0;
        build_geometry(bd.g, d[k].solid, nbr, wi, w6, wd, nskip);
        std::copy(nbr.begin(), nbr.end(), nbr_all.begin() + off);
        for (size_t j = 0; j < wi.size(); ++j) {
            widx.push_back(wi[j]);
            wq.push_back(wd[j] < 0 ? 255 : (uint8_t)wd[j]);
            const double a = w6[3 * j], c = w6[3 * j + 1], e = w6[3 * j + 2];
            const double nn = std::sqrt(a * a + c * c + e * e);
            wn.push_back(nn > 0 ? (float)(a / nn) : 0.f);
            wn.push_back(nn > 0 ? (float)(c / nn) : 0.f);
            wn.push_back(nn > 0 ? (float)(e / nn) : 0.f);
            th.push_back(d[k].theta_rad ? d[k].theta_rad[wi[j]] : (float)(M_PI / 2));
            wdom.push_back((uint16_t)k);
        }
        off += bd.g.N;
        maxN = std::max<size_t>(maxN, bd.g.N);
        // the most phase tiles any shape can give this domain
        uint32_t mt = 0;
        for (int code = 1; code <= 6; ++code) {
            int bx, by;
            phase_shape_of(code, bx, by);
            mt = std::max(mt, phase_tiling(bd.g, bx, by).ntiles);
        }
        ptiles += mt;
    }
    b->nwall = (uint32_t)widx.size();
    b->nptot = (uint32_t)ptiles;
    const size_t N = Ntot;
    BatchPtrs &B = b->B;
    for (int k = 0; k < 2; ++k) {
        B.f[k] = (float *)balloc(b, 27 * N * sizeof(float));
        B.phi[k] = (float *)balloc(b, N * sizeof(float));
    }
    B.u = (float *)balloc(b, 3 * N * sizeof(float));
    B.a = (float *)balloc(b, 3 * N * sizeof(float));
    B.nbr = (uint32_t *)balloc(b, N * sizeof(uint32_t));
    B.solid = (uint8_t *)balloc(b, N);
    const size_t nw = std::max<size_t>(b->nwall, 1);
    B.wall_idx = (int32_t *)balloc(b, nw * sizeof(int32_t));
    B.wall_q = (uint8_t *)balloc(b, nw);
    B.wall_n = (float *)balloc(b, 3 * nw * sizeof(float));
    B.theta = (float *)balloc(b, nw * sizeof(float));
    B.wall_dom = (uint16_t *)balloc(b, nw * sizeof(uint16_t));
    B.partial = (double2 *)balloc(b, (ptiles + 64) * sizeof(double2));
    B.scal = (double *)balloc(b, 8 * (size_t)ndom * sizeof(double));
    B.flag = (uint32_t *)balloc(b, 256);
    B.chunk = (uint8_t *)balloc(b, (N + 1023) / 1024);
    b->d_dom = (BatchDomain *)balloc(b, ndom * sizeof(BatchDomain));
    uint32_t *d_start = (uint32_t *)balloc(b, (ndom + 1) * sizeof(uint32_t));
    const size_t nblk = (N + 255) / 256;
    uint16_t *d_blk = (uint16_t *)balloc(b, nblk * sizeof(uint16_t));
    b->pstar0 = (float *)balloc(b, N * sizeof(float));
    b->mass_partial = (double2 *)balloc(b, (maxN / 256 + 64) * sizeof(double2));
    if (!B.f[0] || !B.f[1] || !B.phi[0] || !B.phi[1] || !B.u || !B.a || !B.nbr || !B.solid || !B.wall_idx ||
        !B.wall_q || !B.wall_n || !B.theta || !B.wall_dom || !B.partial || !B.scal || !B.flag || !B.chunk || !b->d_dom ||
        !b->pstar0 || !b->mass_partial || !d_start || !d_blk)
        return bail(CAC_ERR_ALLOC);
    B.dom = b->d_dom;
    B.dom_start = d_start;
    B.blk_dom = d_blk;
    B.ntot = (uint32_t)N;
    B.ndom = ndom;
    hipStream_t s = b->stream;
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    std::vector<uint32_t> starts(ndom + 1);
    for (int k = 0; k < ndom; ++k) starts[k] = b->dom[k].off;
    starts[ndom] = (uint32_t)N;
    std::vector<uint16_t> blk(nblk);
    for (size_t q = 0, k = 0; q < nblk; ++q) {
        while (256 * q >= starts[k + 1]) ++k;
        blk[q] = (uint16_t)k;
    }
    if (up(B.nbr, nbr_all.data(), N * sizeof(uint32_t)) != hipSuccess ||
        up(d_start, starts.data(), starts.size() * sizeof(uint32_t)) != hipSuccess ||
        up(d_blk, blk.data(), blk.size() * sizeof(uint16_t)) != hipSuccess)
        return bail(CAC_ERR_HIP);
    for (int k = 0; k < ndom; ++k)
        if (up(B.solid + b->dom[k].off, d[k].solid, b->dom[k].g.N) != hipSuccess) return bail(CAC_ERR_HIP);
    if (up(B.wall_idx, widx.data(), widx.size() * 4) != hipSuccess || up(B.wall_q, wq.data(), wq.size()) != hipSuccess ||
        up(B.wall_n, wn.data(), wn.size() * 4) != hipSuccess || up(B.theta, th.data(), th.size() * 4) != hipSuccess ||
        up(B.wall_dom, wdom.data(), wdom.size() * 2) != hipSuccess)
        return bail(CAC_ERR_HIP);
    // initial state per domain
    if (hipMemsetAsync(B.u, 0, 3 * N * sizeof(float), s) != hipSuccess ||
        hipMemsetAsync(B.a, 0, 3 * N * sizeof(float), s) != hipSuccess ||
        hipMemsetAsync(b->pstar0, 0, N * sizeof(float), s) != hipSuccess ||
        hipMemsetAsync(B.flag, 0, 256, s) != hipSuccess ||
        hipMemsetAsync(B.chunk, 0, (N + 1023) / 1024, s) != hipSuccess ||
        hipMemsetAsync(B.scal, 0, 8 * (size_t)ndom * sizeof(double), s) != hipSuccess)
        return bail(CAC_ERR_HIP);
    for (int k = 0; k < ndom; ++k) {
        const Fields F = domain_fields(b, k);
        const size_t bytes = b->dom[k].g.N * sizeof(float);
        if (hipMemcpyAsync(F.phi[0], d[k].d_phi0, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(F.phi[1], d[k].d_phi0, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            launch_init(b->dom[k].g, F, 0, nullptr, nullptr, s) != hipSuccess)
            return bail(CAC_ERR_HIP);
        Tiling t{};
        if (launch_mass(b->dom[k].g, t, F, F.phi[0], F.scal + 0, s) != hipSuccess) return bail(CAC_ERR_HIP);
    }
    if (hipStreamSynchronize(s) != hipSuccess) return bail(CAC_ERR_HIP);
    Schedule def;
    if (apply_schedule(b, def) != CAC_OK) return bail(CAC_ERR_HIP);
    *bp = b;
    return CAC_OK;
}

cac_status cac_batch_set_schedule(cac_batch *b, int bx, int by, int bz, int phase_tile, int grid_mult, int order,
                                  int use_graph)
{
    if (!b) return CAC_ERR_ARG;
    Schedule s;
    s.bx = bx;
    s.by = by;
    s.bz = bz;
    s.phase = phase_tile;
    s.mult = grid_mult;
    s.order = order;
    cac_status st = apply_schedule(b, s);
    if (st == CAC_OK) b->use_graph = use_graph != 0;
    return st;
}

cac_status cac_batch_get_schedule(cac_batch *b, int *out7)
{
    if (!b || !out7) return CAC_ERR_ARG;
    const Schedule &s = b->sch;
    const int v[7] = {s.bx, s.by, s.bz, s.phase, s.mult, s.order, b->use_graph ? 1 : 0};
    std::copy(v, v + 7, out7);
    return CAC_OK;
}

cac_status cac_batch_step(cac_batch *b, int nsteps)
{
    if (!b) return CAC_ERR_ARG;
    if (nsteps < 0) return bfail(b, CAC_ERR_ARG, "nsteps < 0");
    for (int k = 0; k < nsteps; ++k) {
        const bool self = b->coll && b->steps == 0;
        if (b->use_graph && !self) {
            if (!b->gexec[b->cur]) {
                cac_status st = capture(b, b->cur);
                if (st != CAC_OK) return st;
            }
            BCHK(b, hipGraphLaunch(b->gexec[b->cur], b->stream));
        } else {
            cac_status st = run_bstep(b, b->stream, self);
            if (st != CAC_OK) return st;
        }
        b->cur ^= 1;
        b->steps++;
    }
    return CAC_OK;
}

cac_status cac_batch_sync(cac_batch *b)
{
    if (!b) return CAC_ERR_ARG;
    BCHK(b, hipStreamSynchronize(b->stream));
    uint32_t flag = 0;
    BCHK(b, hipMemcpy(&flag, b->B.flag, sizeof flag, hipMemcpyDeviceToHost));
    if (flag) return bfail(b, CAC_ERR_NONFINITE, "non-finite value detected in phi or u");
    return CAC_OK;
}

cac_status cac_batch_volume(cac_batch *b, double *out)
{
    if (!b || !out) return CAC_ERR_ARG;
    for (int k = 0; k < b->ndom; ++k) {
        const Fields F = domain_fields(b, k);
        Tiling t{};
        BCHK(b, launch_mass(b->dom[k].g, t, F, F.phi[b->cur], F.scal + 4, b->stream));
    }
    std::vector<double> sc(8 * (size_t)b->ndom);
    BCHK(b, hipMemcpyAsync(sc.data(), b->B.scal, sc.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    cac_status st = cac_batch_sync(b);
    for (int k = 0; k < b->ndom; ++k) out[k] = sc[8 * (size_t)k + 4];
    return st;
}

cac_status cac_batch_get_fields(cac_batch *b, int k, float *d_phi, float *d_u, float *d_pstar)
{
    if (!b || k < 0 || k >= b->ndom) return CAC_ERR_ARG;
    const Fields F = domain_fields(b, k);
    const Grid &g = b->dom[k].g;
    // p*: the post-collision populations' zeroth moment, or the record's p* plane (collision = 1)
    if (d_phi || d_pstar)
        BCHK(b, launch_gather(g, F, b->coll ? 1 : b->cur, b->cur, b->steps > 0, b->coll ? 1 : 27, d_phi, d_pstar,
                              b->stream));
    if (d_u) BCHK(b, hipMemcpyAsync(d_u, F.u, 3 * (size_t)g.N * sizeof(float), hipMemcpyDeviceToDevice, b->stream));
    return CAC_OK;
}

cac_status cac_batch_info(cac_batch *b, int *ndom, long long *total_nodes, long long *fluid_nodes)
{
    if (!b) return CAC_ERR_ARG;
    if (ndom) *ndom = b->ndom;
    if (total_nodes) *total_nodes = b->Ntot;
    if (fluid_nodes) {
        // fluid count = nodes whose bitmask bit 0 is clear; computed once from the host copy
        std::vector<uint8_t> sol(b->Ntot);
        BCHK(b, hipMemcpy(sol.data(), b->B.solid, b->Ntot, hipMemcpyDeviceToHost));
        long long c = 0;
        for (uint8_t v : sol) c += v ? 0 : 1;
        *fluid_nodes = c;
    }
    return CAC_OK;
}

cac_status cac_batch_profile(cac_batch *b, int nsteps, double *ms)
{
    if (!b || !ms || nsteps < 0) return CAC_ERR_ARG;
    const int nt = sched_nt(b->sch);
    std::vector<hipEvent_t> ev(5 * (size_t)nsteps);
    for (auto &e : ev) BCHK(b, hipEventCreate(&e));
    for (int k = 0; k < nsteps; ++k) {
        hipEvent_t *e = &ev[5 * (size_t)k];
        const int c = b->cur;
        BCHK(b, hipEventRecord(e[0], b->stream));
        BCHK(b, launch_bghost(b->B, b->nwall, c, b->stream));
        BCHK(b, hipEventRecord(e[1], b->stream));
        if (b->coll) {
            const bool self = b->steps == 0;
            if (!self) BCHK(b, launch_br1_rebuild(b->B, b->sch.phase, b->d_pitems, b->np, b->stream));
            BCHK(b, launch_br1_stream(b->B, b->pstar0, nt, b->d_hitems, b->nh, b->hlds, c, self, b->stream));
        } else {
            BCHK(b, launch_bhydro(b->B, nt, b->d_hitems, b->nh, b->hgrid, b->hlds, c, b->stream));
        }
        BCHK(b, hipEventRecord(e[2], b->stream));
        BCHK(b, launch_bphase(b->B, b->sch.phase, b->d_pitems, b->np, b->pgrid, c, b->stream));
        BCHK(b, hipEventRecord(e[3], b->stream));
        BCHK(b, launch_bvolume(b->B, nt, b->d_hitems, b->nh, b->hgrid, c ^ 1, b->stream));
        BCHK(b, hipEventRecord(e[4], b->stream));
        b->cur ^= 1;
        b->steps++;
    }
    BCHK(b, hipStreamSynchronize(b->stream));
    for (int k = 0; k < nsteps; ++k)
        for (int j = 0; j < 4; ++j) {
            float t = 0.f;
            BCHK(b, hipEventElapsedTime(&t, ev[5 * (size_t)k + j], ev[5 * (size_t)k + j + 1]));
            ms[j] += t;
        }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return CAC_OK;
}

// Coordinate search over the hydro tile, the phase tile, the grid multiplier
// and the item order; each trial times `trial_steps` eager steps with HIP
// events after one warm-up step.  The state is saved before and restored
// after, so tuning leaves the simulation where it was.  The winner is applied
// (with graph replay) and, when cache_path is given, stored there keyed by the
// device and the histogram of domain shapes; a cached entry is used directly.
cac_status cac_batch_autotune(cac_batch *b, const char *cache_path, int trial_steps, double *best_ms)
{
    if (!b || trial_steps < 1) return CAC_ERR_ARG;
    const std::string key = tune_key(b);
    Schedule best = b->sch;
    if (cache_lookup(cache_path, key, best)) {
        cac_status st = apply_schedule(b, best);
        if (st == CAC_OK) b->use_graph = true;
        if (best_ms) *best_ms = -1.0;
        return st;
    }
    float *snap = (float *)balloc(b, state_bytes(b));
    if (!snap) return bfail(b, CAC_ERR_ALLOC, "autotune snapshot");
    const int cur0 = b->cur;
    const long long steps0 = b->steps;
    cac_status st = snapshot(b, snap, true);
    if (st != CAC_OK) return st;
    hipEvent_t e0, e1;
    BCHK(b, hipEventCreate(&e0));
    BCHK(b, hipEventCreate(&e1));
    auto trial = [&](const Schedule &s, double &ms) -> cac_status {
        cac_status r = apply_schedule(b, s);
        if (r != CAC_OK) return r;
        // warm-up step (the first gradient-form step pulls the equilibrium); the timed ones are ordinary
        r = run_bstep(b, b->stream, b->coll && b->steps == 0);
        if (r != CAC_OK) return r;
        b->cur ^= 1;
        BCHK(b, hipEventRecord(e0, b->stream));
        for (int k = 0; k < trial_steps; ++k) {
            r = run_bstep(b, b->stream);
            if (r != CAC_OK) return r;
            b->cur ^= 1;
        }
        BCHK(b, hipEventRecord(e1, b->stream));
        BCHK(b, hipEventSynchronize(e1));
        float t = 0.f;
        BCHK(b, hipEventElapsedTime(&t, e0, e1));
        ms = t / trial_steps;
        return CAC_OK;
    };
    double best_t = 1e30;
    {
        double t;
        st = trial(best, t);
        if (st != CAC_OK) return st;
        best_t = t;
    }
    const int tiles[][3] = {{0, 256, 0}, {0, 512, 0}, {0, 128, 0}, {16, 4, 4}, {32, 4, 2}, {32, 8, 1},
                            {64, 4, 1},  {64, 2, 2},  {64, 8, 1},  {128, 2, 1}};
    // two passes of the coordinate search: the second revisits the tile with
    // the phase tile, multiplier and order the first pass chose
    for (int pass = 0; pass < 2; ++pass) {
        for (auto &tl : tiles) {
            Schedule s = best;
            s.bx = tl[0];
            s.by = tl[1];
            s.bz = tl[2];
            double t;
            if (trial(s, t) == CAC_OK && t < best_t) {
                best_t = t;
                best = s;
            }
        }
        for (int code = 1; code <= 6; ++code) {
            Schedule s = best;
            s.phase = code;
            double t;
            if (trial(s, t) == CAC_OK && t < best_t) {
                best_t = t;
                best = s;
            }
        }
        for (int m : {0, 1, 2, 4, 8}) {
            Schedule s = best;
            s.mult = m;
            double t;
            if (trial(s, t) == CAC_OK && t < best_t) {
                best_t = t;
                best = s;
            }
        }
        for (int o : {0, 1}) {
            Schedule s = best;
            s.order = o;
            double t;
            if (trial(s, t) == CAC_OK && t < best_t) {
                best_t = t;
                best = s;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->cur = cur0;
    b->steps = steps0;
    st = snapshot(b, snap, false);
    if (st != CAC_OK) return st;
    BCHK(b, hipMemsetAsync(b->B.flag, 0, 256, b->stream));
    st = apply_schedule(b, best);
    if (st != CAC_OK) return st;
    b->use_graph = true;
    cache_store(cache_path, key, best, best_t);
    if (best_ms) *best_ms = best_t;
    return CAC_OK;
}

cac_status cac_batch_destroy(cac_batch *b)
{
    if (!b) return CAC_ERR_ARG;
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (void *q : b->owned) (void)hipFree(q);
    delete b;
    return CAC_OK;
}

cac_status cac_batch_last_error(cac_batch *b, char *buf, size_t n)
{
    if (!b || !buf || n == 0) return CAC_ERR_ARG;
    snprintf(buf, n, "%s", b->err.c_str());
    return CAC_OK;
}

}  // extern "C"
