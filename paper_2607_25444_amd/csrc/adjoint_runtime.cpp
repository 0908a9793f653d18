// adjoint_runtime.cpp -- host side of the adjoint (cac_tape_*, cac_loss,
// cac_adjoint): a recorded forward sweep keeps the state every K steps
// (checkpoints); the reverse sweep replays one segment at a time, keeping
// every step of the segment in rings (populations entering the step, phi with
// its ghosts, velocity, phi before the volume correction), then runs the
// reverse steps of the segment backwards.  Device memory is bounded by
// ceil(nsteps/K) checkpoints of 29 N words plus rings of about 33 K N words.
// The recorded sweep runs its last segment straight into the rings, so that
// segment is never replayed; with K >= nsteps (one segment, about 128 bytes
// per node and step: 134 GB for 1000 steps of 128x128x64) nothing is.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "adjoint_tables.hpp"
#include "handle.hpp"

namespace cac {

struct AdjTape {
    int nsteps = 0, K = 0;
    bool recorded = false;       // cleared by cac_set_state (the target mass may change)
    long long rec_serial = -1;   // geometry of the recorded sweep
    float *theta = nullptr;      // contact angles of the recorded sweep (nwall)
    int theta_cap = 0;
    std::vector<float *> ck;     // checkpoints: 27N populations, N phi (current), N phi (previous ghosts)
    int ring_K = 0;              // rings sized for this K
    // One or two sets of segment rings: with two, the replay of the next
    // segment (on the auxiliary stream) runs while this one is reversed.
    int nsets = 0;
    bool last_in_rings = false;    // ring set 0 holds the last segment, left by the recorded sweep
    std::vector<float *> rf[2];    // K+1 population sets: rf[j] enters step j of the segment
    std::vector<float *> rphi[2];  // K+2 phase fields: rphi[j+1] = phi with the ghosts of step j
    std::vector<float *> ru[2];    // K velocities (zero on solid nodes)
    std::vector<float *> rps[2];   // K fields phi* (before the correction)
    hipStream_t aux = nullptr;     // replay stream (default priority)
    hipEvent_t ready[2] = {nullptr, nullptr}, released[2] = {nullptr, nullptr}, joined = nullptr;
    ~AdjTape()
    {
        if (aux) (void)hipStreamSynchronize(aux);
        for (hipEvent_t e : {ready[0], ready[1], released[0], released[1], joined})
            if (e) (void)hipEventDestroy(e);
        if (aux) (void)hipStreamDestroy(aux);
    }
    // reverse state
    bool adj_ready = false;
    float *mb[2] = {nullptr, nullptr}, *pb[2] = {nullptr, nullptr};
    float *rec = nullptr, *awb = nullptr, *seed = nullptr, *psi = nullptr;
    double *thb = nullptr, *red = nullptr, *rs = nullptr;
    // donor tables (rebuilt when the geometry changes)
    long long geom_serial = -1;
    float4 *dg = nullptr;
    int32_t *don_node = nullptr, *don_start = nullptr, *don_wall = nullptr, *don_map = nullptr;
    uint32_t *near = nullptr;
    int ndon = 0;
    uint32_t nnear = 0;
};

void tape_free(cac_handle *h)
{
    delete h->tape;  // device memory belongs to the handle's allocations
    h->tape = nullptr;
}

void tape_invalidate(cac_handle *h)
{
    if (h->tape) h->tape->recorded = false;
}

namespace {

AdjTape *tape_of(cac_handle *h)
{
    if (!h->tape) h->tape = new AdjTape();
    return h->tape;
}

template <class T>
bool alloc_n(cac_handle *h, T *&p, size_t n)
{
    p = (T *)dev_alloc(h, std::max<size_t>(n, 1) * sizeof(T));
    return p != nullptr;
}

// One set of segment rings; false when the device memory is not there.
bool alloc_ring_set(cac_handle *h, AdjTape &T, int k)
{
    const size_t N = h->g.N;
    const int K = T.K;
    while ((int)T.rf[k].size() < K + 1) {
        float *p;
        if (!alloc_n(h, p, 27 * N)) return false;
        T.rf[k].push_back(p);
    }
    while ((int)T.rphi[k].size() < K + 2) {
        float *p;
        if (!alloc_n(h, p, N)) return false;
        T.rphi[k].push_back(p);
    }
    while ((int)T.ru[k].size() < K) {
        float *p;
        if (!alloc_n(h, p, 3 * N)) return false;
        // the collision never writes solid nodes: keep their velocity at zero
        if (hipMemsetAsync(p, 0, 3 * N * sizeof(float), h->stream) != hipSuccess) return false;
        T.ru[k].push_back(p);
    }
    while ((int)T.rps[k].size() < K) {
        float *p;
        if (!alloc_n(h, p, N)) return false;
        T.rps[k].push_back(p);
    }
    return true;
}

cac_status ensure_rings(cac_handle *h, AdjTape &T)
{
    const size_t N = h->g.N;
    const int K = T.K;
    if (!alloc_ring_set(h, T, 0)) return fail(h, CAC_ERR_ALLOC, "adjoint ring");
    // a second set (for the overlapped replay) only with room to spare
    bool two = (int)T.rf[1].size() >= K + 1 && (int)T.rphi[1].size() >= K + 2 && (int)T.ru[1].size() >= K &&
               (int)T.rps[1].size() >= K;
    if (!two) {
        size_t free_b = 0, total_b = 0;
        const size_t set_b = ((size_t)(K + 1) * 27 + (size_t)(K + 2) + (size_t)K * 4) * N * sizeof(float);
        two = hipMemGetInfo(&free_b, &total_b) == hipSuccess && 2 * set_b < free_b && alloc_ring_set(h, T, 1);
    }
    T.nsets = two ? 2 : 1;
    if (T.nsets == 2 && !T.aux) {
        if (hipStreamCreateWithFlags(&T.aux, hipStreamNonBlocking) != hipSuccess) {
            T.aux = nullptr;
            T.nsets = 1;
        } else {
            for (hipEvent_t *e : {&T.ready[0], &T.ready[1], &T.released[0], &T.released[1], &T.joined})
                HIPCHK(h, hipEventCreateWithFlags(e, hipEventDisableTiming));
        }
    }
    if (!T.adj_ready) {
        bool ok = alloc_n(h, T.mb[0], 10 * N) && alloc_n(h, T.mb[1], 10 * N) && alloc_n(h, T.pb[0], N) &&
                  alloc_n(h, T.pb[1], N) && alloc_n(h, T.rec, 5 * N) && alloc_n(h, T.awb, 3 * N) &&
                  alloc_n(h, T.psi, N) &&
                  (T.seed || alloc_n(h, T.seed, N)) &&
                  (T.red || alloc_n(h, T.red, 3 * (size_t)adj_red_blocks(h->g) + 64)) && (T.rs || alloc_n(h, T.rs, 8));
        if (!ok) return fail(h, CAC_ERR_ALLOC, "adjoint buffers");
        HIPCHK(h, hipMemsetAsync(T.awb, 0, 3 * N * sizeof(float), h->stream));
        T.adj_ready = true;
    }
    return CAC_OK;
}

cac_status ensure_tables(cac_handle *h, AdjTape &T)
{
    if (T.geom_serial == h->geom_serial) return CAC_OK;
    DonorTables D;
    build_donor_tables(h->g, h->widx.data(), h->wdonor.data(), (int)h->widx.size(), D);
    T.ndon = (int)D.don_node.size();
    T.nnear = (uint32_t)D.near.size();
    const size_t N = h->g.N;
    bool ok = alloc_n(h, T.dg, T.ndon) && alloc_n(h, T.don_node, T.ndon) && alloc_n(h, T.don_start, T.ndon + 1) &&
              alloc_n(h, T.don_wall, D.don_wall.size()) && alloc_n(h, T.don_map, N) && alloc_n(h, T.near, T.nnear) &&
              alloc_n(h, T.thb, h->widx.size());
    if (!ok) return fail(h, CAC_ERR_ALLOC, "adjoint donor tables");
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream) : hipSuccess;
    };
    HIPCHK(h, up(T.don_node, D.don_node.data(), D.don_node.size() * 4));
    HIPCHK(h, up(T.don_start, D.don_start.data(), D.don_start.size() * 4));
    HIPCHK(h, up(T.don_wall, D.don_wall.data(), D.don_wall.size() * 4));
    HIPCHK(h, up(T.don_map, D.don_map.data(), D.don_map.size() * 4));
    HIPCHK(h, up(T.near, D.near.data(), D.near.size() * 4));
    HIPCHK(h, hipStreamSynchronize(h->stream));  // host vectors go out of scope
    T.geom_serial = h->geom_serial;
    return CAC_OK;
}

// Forward step j of a segment on stream st, keeping its state in ring set k.
// Only the replay touches the handle's compressive flux, tile partials and
// volume scalars (the reverse step reads the target volume alone).
cac_status replay_step(cac_handle *h, AdjTape &T, int k, int j, hipStream_t st)
{
    Fields F = h->F;
    F.theta = T.theta;
    F.chunk = nullptr;  // the out-of-place correction below visits every node
    F.phi[0] = T.rphi[k][j + 1];
    F.phi[1] = T.rphi[k][j];
    HIPCHK(h, launch_ghost(h->g, h->dp, F, 0, st));
    F.f[0] = T.rf[k][j];
    F.f[1] = T.rf[k][j + 1];
    F.u = T.ru[k][j];
    HIPCHK(h, launch_hydro(h->g, h->t, h->dp, F, 0, 0, st));
    F.phi[1] = T.rps[k][j];
    HIPCHK(h, launch_phase(h->g, h->t, h->dp, F, 0, st));
    HIPCHK(h, launch_volume_copy(h->g, h->t, h->dp, F, T.rps[k][j], T.rphi[k][j + 1], T.rphi[k][j + 2], st));
    return CAC_OK;
}

// Replay of segment seg (from its checkpoint) into ring set k on stream st.
cac_status replay_segment(cac_handle *h, AdjTape &T, int seg, int k, hipStream_t st)
{
    const size_t N = h->g.N;
    const int n0 = seg * T.K;
    const int L = std::min(T.K, T.nsteps - n0);
    const float *ck = T.ck[seg];
    HIPCHK(h, hipMemcpyAsync(T.rf[k][0], ck, 27 * N * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(h, hipMemcpyAsync(T.rphi[k][1], ck + 27 * N, N * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(h, hipMemcpyAsync(T.rphi[k][0], ck + 28 * N, N * sizeof(float), hipMemcpyDeviceToDevice, st));
    for (int j = 0; j < L; ++j) {
        cac_status s = replay_step(h, T, k, j, st);
        if (s != CAC_OK) return s;
    }
    return CAC_OK;
}

// Reverse of step j of a segment held in ring set k; cotangents move from
// parity c to c ^ 1.
cac_status reverse_step(cac_handle *h, AdjTape &T, int k, int j, int c)
{
    AdjStep S{};
    S.fprev = T.rf[k][j];
    S.phihat = T.rphi[k][j + 1];
    S.phiold = T.rphi[k][j];
    S.u = T.ru[k][j];
    S.phistar = T.rps[k][j];
    S.pb_in = T.pb[c];
    S.mb_in = T.mb[c];
    S.pb_out = T.pb[c ^ 1];
    S.mb_out = T.mb[c ^ 1];
    S.psi = T.psi;
    S.rec = T.rec;
    S.awb = T.awb;
    S.nbr = h->F.nbr;
    S.solid = h->F.solid;
    S.widx = h->F.wall_idx;
    S.wq = h->F.wall_q;
    S.wn = h->F.wall_n;
    S.theta = T.theta;
    S.don_start = T.don_start;
    S.don_wall = T.don_wall;
    S.don_node = T.don_node;
    S.ndon = T.ndon;
    S.don_map = T.don_map;
    S.dg = T.dg;
    S.near = T.near;
    S.nnear = T.nnear;
    S.thb = T.thb;
    S.red = T.red;
    S.rs = T.rs;
    S.scal = h->F.scal;
    HIPCHK(h, launch_adj_vsum(h->g, h->dp, S, h->stream));
    HIPCHK(h, launch_adj_main(h->g, h->t, h->dp, S, h->stream));
    HIPCHK(h, launch_adj_assemble(h->g, h->t, S, h->stream));
    HIPCHK(h, launch_adj_wall(h->g, h->dp, S, h->stream));
    HIPCHK(h, launch_adj_fix(h->g, S, h->stream));
    return CAC_OK;
}

}  // namespace
}  // namespace cac

using namespace cac;

extern "C" {

cac_status cac_tape_forward(cac_handle *h, int nsteps, int K)
{
    if (!h) return CAC_ERR_ARG;
    if (nsteps < 1 || K < 1) return fail(h, CAC_ERR_ARG, "nsteps and K must be >= 1");
    if (!h->state) return fail(h, CAC_ERR_STATE, "cac_set_state must come first");
    if (h->sub != 0) return fail(h, CAC_ERR_STATE, "a step was started with cac_debug_substep");
    if (h->prm.collision != 0) return fail(h, CAC_ERR_STATE, "the adjoint is built for collision = 0");
    if (h->prm.ghost_localization != 1)
        return fail(h, CAC_ERR_STATE, "the adjoint is built for the localisation factor of Eq. (47)");
    AdjTape &T = *tape_of(h);
    T.recorded = false;
    T.last_in_rings = false;
    const size_t N = h->g.N;
    const int nck = (nsteps + K - 1) / K;
    while ((int)T.ck.size() < nck) {
        float *p;
        if (!alloc_n(h, p, 29 * N)) return fail(h, CAC_ERR_ALLOC, "checkpoint storage");
        T.ck.push_back(p);
    }
    const int nwall = h->F.nwall;
    if (nwall > T.theta_cap) {
        if (!alloc_n(h, T.theta, (size_t)nwall + 64)) return fail(h, CAC_ERR_ALLOC, "tape angles");
        T.theta_cap = nwall + 64;
    }
    if (nwall)
        HIPCHK(h, hipMemcpyAsync(T.theta, h->F.theta, nwall * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    // The last segment runs as the replay would, into ring set 0 (which the
    // reverse sweep needs in any case), and its end state is copied back to
    // the handle; the steps before it are ordinary steps.
    const int last0 = (nck - 1) * K;
    T.K = K;
    if (!alloc_ring_set(h, T, 0)) return fail(h, CAC_ERR_ALLOC, "adjoint ring");
    for (int n = 0; n < nsteps; ++n) {
        if (n % K == 0) {
            float *c = T.ck[n / K];
            const int cur = h->cur;
            HIPCHK(h, hipMemcpyAsync(c, h->F.f[cur], 27 * N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
            HIPCHK(h, hipMemcpyAsync(c + 27 * N, h->F.phi[cur], N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
            HIPCHK(h, hipMemcpyAsync(c + 28 * N, h->F.phi[cur ^ 1], N * sizeof(float), hipMemcpyDeviceToDevice,
                                     h->stream));
        }
        if (n == last0) {
            const int cur = h->cur;
            HIPCHK(h, hipMemcpyAsync(T.rf[0][0], h->F.f[cur], 27 * N * sizeof(float), hipMemcpyDeviceToDevice,
                                     h->stream));
            HIPCHK(h, hipMemcpyAsync(T.rphi[0][1], h->F.phi[cur], N * sizeof(float), hipMemcpyDeviceToDevice,
                                     h->stream));
            HIPCHK(h, hipMemcpyAsync(T.rphi[0][0], h->F.phi[cur ^ 1], N * sizeof(float), hipMemcpyDeviceToDevice,
                                     h->stream));
        }
        if (n >= last0) {
            cac_status st = replay_step(h, T, 0, n - last0, h->stream);
            if (st != CAC_OK) return st;
        } else {
            cac_status st = cac_step(h, 1);
            if (st != CAC_OK) return st;
        }
    }
    {
        // The handle continues from the end of the last segment, in the state
        // the in-place steps leave.  No step writes populations or velocity
        // on solid nodes, so only the fluid entries are copied.  The current
        // phi holds the corrected fluid values and, on solid nodes, what that
        // buffer held before (the ghosts of the step before last): what the
        // correction writes when given the ring entry of that step as phi-hat.
        const int L = nsteps - last0, cur = h->cur ^ (L & 1);  // the parity L in-place steps end on
        HIPCHK(h, launch_copy_fluid(h->g, h->F.solid, 27, T.rf[0][L], h->F.f[cur], h->stream));
        HIPCHK(h, launch_volume_copy(h->g, h->t, h->dp, h->F, T.rps[0][L - 1], T.rphi[0][L - 1], h->F.phi[cur],
                                     h->stream));
        HIPCHK(h, hipMemcpyAsync(h->F.phi[cur ^ 1], T.rphi[0][L], N * sizeof(float), hipMemcpyDeviceToDevice,
                                 h->stream));
        HIPCHK(h, launch_copy_fluid(h->g, h->F.solid, 3, T.ru[0][L - 1], h->F.u, h->stream));
        h->cur = cur;
        h->steps += L;
    }
    T.last_in_rings = true;
    T.nsteps = nsteps;
    T.rec_serial = h->geom_serial;
    T.recorded = true;
    return CAC_OK;
}

cac_status cac_tape_backward(cac_handle *h, const float *d_phibar, double *d_dtheta, float *d_phibar0)
{
    if (!h || !d_phibar || !d_dtheta) return CAC_ERR_ARG;
    AdjTape *Tp = h->tape;
    if (!Tp || !Tp->recorded) return fail(h, CAC_ERR_STATE, "no recorded sweep (cac_tape_forward)");
    if (Tp->rec_serial != h->geom_serial) return fail(h, CAC_ERR_STATE, "geometry changed after the recorded sweep");
    AdjTape &T = *Tp;
    cac_status st = ensure_rings(h, T);
    if (st != CAC_OK) return st;
    st = ensure_tables(h, T);
    if (st != CAC_OK) return st;
    const size_t N = h->g.N;
    const int nwall = h->F.nwall;
    HIPCHK(h, hipMemcpyAsync(T.pb[0], d_phibar, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemsetAsync(T.mb[0], 0, 10 * N * sizeof(float), h->stream));
    if (nwall) HIPCHK(h, hipMemsetAsync(T.thb, 0, nwall * sizeof(double), h->stream));
    HIPCHK(h, hipMemsetAsync(T.rs, 0, 4 * sizeof(double), h->stream));
    int c = 0;
    const int nck = (T.nsteps + T.K - 1) / T.K;
    // Segments are reversed from the last to the first.  With two ring sets
    // the replay of segment seg - 1 (auxiliary stream, set k ^ 1) overlaps the
    // reverse of segment seg (handle stream, set k); events order each replay
    // after the reverse that last used its set, and each reverse after its
    // replay.  With one set the two alternate on the handle stream.
    const bool overlap = T.nsets == 2;
    // the last segment is in ring set 0 when the recorded sweep left it there
    // and no earlier reverse sweep has reused the set since
    const bool have_last = T.last_in_rings;
    T.last_in_rings = have_last && nck == 1;
    if (overlap) {
        HIPCHK(h, hipEventRecord(T.joined, h->stream));  // the aux stream starts after everything queued so far
        HIPCHK(h, hipStreamWaitEvent(T.aux, T.joined, 0));
        if (!have_last) {
            st = replay_segment(h, T, nck - 1, 0, T.aux);
            if (st != CAC_OK) return st;
        }
        HIPCHK(h, hipEventRecord(T.ready[0], T.aux));
    }
    for (int seg = nck - 1; seg >= 0; --seg) {
        const int L = std::min(T.K, T.nsteps - seg * T.K);
        const int k = overlap ? (nck - 1 - seg) & 1 : 0;
        if (overlap) {
            if (seg > 0) {
                if (seg + 1 <= nck - 1) HIPCHK(h, hipStreamWaitEvent(T.aux, T.released[k ^ 1], 0));
                st = replay_segment(h, T, seg - 1, k ^ 1, T.aux);
                if (st != CAC_OK) return st;
                HIPCHK(h, hipEventRecord(T.ready[k ^ 1], T.aux));
            }
            HIPCHK(h, hipStreamWaitEvent(h->stream, T.ready[k], 0));
        } else if (!(have_last && seg == nck - 1)) {
            st = replay_segment(h, T, seg, 0, h->stream);
            if (st != CAC_OK) return st;
        }
        for (int j = L - 1; j >= 0; --j) {
            st = reverse_step(h, T, k, j, c);
            if (st != CAC_OK) return st;
            c ^= 1;
        }
        if (overlap) HIPCHK(h, hipEventRecord(T.released[k], h->stream));
    }
    if (overlap) {
        HIPCHK(h, hipEventRecord(T.joined, T.aux));  // nothing on the aux stream outlives this call
        HIPCHK(h, hipStreamWaitEvent(h->stream, T.joined, 0));
    }
    if (nwall)
        HIPCHK(h, hipMemcpyAsync(d_dtheta, T.thb, nwall * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    if (d_phibar0) {
        HIPCHK(h, launch_adj_mtarget(h->g, h->F.solid, T.pb[c], T.rs, h->stream));
        HIPCHK(h, hipMemcpyAsync(d_phibar0, T.pb[c], N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    }
    return CAC_OK;
}

cac_status cac_loss(cac_handle *h, const float *d_phi_target, float *d_seed, double *loss_host)
{
    if (!h || !d_phi_target) return CAC_ERR_ARG;
    if (!h->state) return fail(h, CAC_ERR_STATE, "no state");
    AdjTape &T = *tape_of(h);
    const size_t N = h->g.N;
    if (!T.seed && !alloc_n(h, T.seed, N)) return fail(h, CAC_ERR_ALLOC, "seed");
    if (!T.red && !alloc_n(h, T.red, 3 * (size_t)adj_red_blocks(h->g) + 64)) return fail(h, CAC_ERR_ALLOC, "partials");
    if (!T.rs && !alloc_n(h, T.rs, 8)) return fail(h, CAC_ERR_ALLOC, "scalars");
    HIPCHK(h, launch_loss_seed(h->g, h->F.solid, h->F.phi[h->cur], d_phi_target, d_seed ? d_seed : T.seed, T.red,
                               T.rs + 4, h->stream));
    if (loss_host) {
        HIPCHK(h, hipMemcpyAsync(loss_host, T.rs + 4, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        return cac_sync(h);
    }
    return CAC_OK;
}

cac_status cac_adjoint(cac_handle *h, int nsteps, int K, const float *d_phi_target, double *loss_host,
                       double *d_dL_dtheta)
{
    if (!h || !d_phi_target || !d_dL_dtheta) return CAC_ERR_ARG;
    cac_status st = cac_tape_forward(h, nsteps, K);
    if (st != CAC_OK) return st;
    AdjTape &T = *h->tape;
    st = cac_loss(h, d_phi_target, nullptr, nullptr);
    if (st != CAC_OK) return st;
    st = cac_tape_backward(h, T.seed, d_dL_dtheta, nullptr);
    if (st != CAC_OK) return st;
    if (loss_host) HIPCHK(h, hipMemcpyAsync(loss_host, T.rs + 4, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    return cac_sync(h);
}

}  // extern "C"
