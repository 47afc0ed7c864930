// gv_batch.cpp -- the batch ABI: many uneven instances (Graph-VQE's
// concurrent block updates, Sec. IV-D, Eq. 11) in one persistent kernel,
// optionally recorded once as a HIP graph and replayed.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "gv_internal.hpp"

constexpr int kSideStreams = 8;

struct gv_batch_s {
    int count = 0;
    int nsmall = 0;                 // instances in the persistent kernels' queues
    int nlds = 0;                   // ... of which the first nlds keep their vectors in LDS
    gv_precision prec = GV_C64;
    void *work = nullptr;
    size_t work_bytes = 0;
    hipStream_t stream = nullptr;
    gv::BatchInst *dev_insts = nullptr;
    int *dev_order = nullptr;
    unsigned *counter = nullptr;
    int grid = 0, grid_lds = 0;
    bool graph = false;
    hipStream_t capture_stream = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    // instances run as whole-GPU passes: their instance records and output
    // slots, states (the batch's psi buffer of the instance and a work region
    // of their own) and device gradient masks; side streams with fork / join
    // events (or none: then they run one after another on the batch stream)
    std::vector<gv_instance> large;
    std::vector<double *> large_e, large_g;
    std::vector<uint64_t> large_q;   // their qubit blocks (0: energy only)
    std::vector<gv_state_s> states;
    std::vector<uint8_t *> masks;
    bool side_streams = true;
    // every instance's Hamiltonian and its prepare generation at creation
    std::vector<std::pair<const gv_pauli_s *, uint64_t>> hgen;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr, fork2 = nullptr;
    hipEvent_t join[kSideStreams] = {};
};

namespace gv {

namespace {

constexpr int kBatchK = 12, kBatchLogR = 4;

struct BatchLayout {
    size_t counter, insts, order, total;
    std::vector<size_t> offp, ry, dtab, gtab, g0tab, psi, lam;
    std::vector<size_t> stride;
    std::vector<size_t> fwork, fwork_bytes, mask;   // whole-GPU instances (0 bytes otherwise)
};

int split_of(const gv_batch_tuning *tu)
{
    const int s = tu ? tu->split_n : 0;
    return s <= 0 ? 17 : s;
}

// instances with n <= lds_n keep psi and lam in LDS (complex64, n = 12:
// 2 x 32 KB beside the tile exchange buffer); 0 = default, < 0 = never
int lds_n_of(const gv_batch_tuning *tu, gv_precision prec)
{
    const int v = tu ? tu->lds_n : 0;
    if (prec != GV_C64 || v < 0) return 0;
    return v == 0 ? kBatchK : std::min(v, kBatchK);
}

gv_status check_instances(int count, const gv_instance *inst, gv_precision prec)
{
    if (count < 0) return set_error(GV_EINVAL, "count < 0");
    if (count > 0 && !inst) return set_error(GV_EINVAL, "instances is NULL");
    if (prec != GV_C64 && prec != GV_C128) return set_error(GV_EINVAL, "precision %d", prec);
    const int C = std::min(kBatchK - 1, prec == GV_C64 ? 4 : 3);
    for (int i = 0; i < count; ++i) {
        const gv_instance &I = inst[i];
        const gv_ansatz &a = I.ansatz;
        if (a.n < kBatchK || a.n > 30)
            return set_error(GV_EUNSUPPORTED, "instance %d: n=%d outside %d..30", i, a.n, kBatchK);
        if (a.layers < 0 || a.layers > 4096 || (a.final_rotation != 0 && a.final_rotation != 1))
            return set_error(GV_EINVAL, "instance %d: bad ansatz", i);
        if (a.layers + a.final_rotation < 1)
            return set_error(GV_EUNSUPPORTED, "instance %d: no rotation layer", i);
        if (a.ent != GV_ENT_NONE && a.ent != GV_ENT_CZ_LINEAR && a.ent != GV_ENT_CZ_CIRCULAR)
            return set_error(GV_EUNSUPPORTED, "instance %d: batches take CZ or no entangler", i);
        if (!I.params_dev || !I.h)
            return set_error(GV_EINVAL, "instance %d: NULL pointer", i);
        const gv_pauli_s *h = I.h;
        if (!h->prepared || h->n != a.n)
            return set_error(GV_ESTATE, "instance %d: Hamiltonian not prepared for n=%d", i, a.n);
        if (!h->loose_terms.empty())
            return set_error(GV_EUNSUPPORTED, "instance %d: off-diagonal terms too wide for a tile", i);
        if (!h->ox.empty() && (h->cover_K != kBatchK || h->cover_C != C))
            return set_error(GV_ESTATE, "instance %d: Hamiltonian prepared for another precision", i);
    }
    return GV_OK;
}

BatchLayout batch_layout(int count, const gv_instance *inst, gv_precision prec, int split)
{
    BatchLayout L;
    const size_t s = amp_bytes(prec);
    size_t off = 0;
    L.counter = off;
    off += kAlign;
    L.insts = off;
    off += align_up((size_t)count * sizeof(BatchInst) + 8);
    L.order = off;
    off += align_up((size_t)count * sizeof(int) + 8);
    for (int i = 0; i < count; ++i) {
        const gv_ansatz &a = inst[i].ansatz;
        const Chunks ch = make_chunks(a.n, kBatchK, kBatchLogR);
        const size_t stride = align_up((size_t)ch.off[4] * s);
        const int R = a.layers + a.final_rotation;
        L.stride.push_back(stride);
        L.offp.push_back(off);
        off += align_up(inst[i].h->off_passes.size() * sizeof(BatchOffPass) + 8);
        L.ry.push_back(off);
        off += align_up((size_t)2 * a.n * R * 2 * sizeof(double) + 8);
        L.dtab.push_back(off);
        off += stride * (size_t)R;
        L.gtab.push_back(off);
        off += stride;
        L.g0tab.push_back(off);
        off += stride;
        L.psi.push_back(off);
        off += align_up(((size_t)1 << a.n) * s);
        L.lam.push_back(off);
        off += align_up(((size_t)1 << a.n) * s);
        size_t fw = 0, mk = 0;
        if (a.n >= split) {
            WorkLayout wl;
            if (work_layout(a, prec, GV_ENGINE_FUSED, GV_GRAD_STORE, &wl) == GV_OK) fw = wl.total;
            mk = (size_t)2 * a.n * R;
        }
        L.fwork.push_back(off);
        L.fwork_bytes.push_back(fw);
        off += align_up(fw);
        L.mask.push_back(off);
        off += align_up(mk + 8);
    }
    L.total = off;
    return L;
}

// One evaluation of every instance, enqueued on s: the persistent kernel
// for the small instances on s; the LDS-resident instances' kernel and the
// whole-GPU instances (round-robin) on the side streams, between fork events
// and a join (so a HIP-graph capture of s records every branch).
gv_status launch_all(gv_batch b, hipStream_t s)
{
    hipError_t e = hipSuccess;
    const bool fork = b->side_streams && (!b->large.empty() || b->nlds > 0);
    if (fork) {
        e = hipEventRecord(b->fork, s);
        for (int k = 0; k < kSideStreams - 1 && e == hipSuccess; ++k)
            e = hipStreamWaitEvent(b->side[k], b->fork, 0);
        if (e != hipSuccess) return check_hip(e, "batch fork");
    }
    e = batch_tables(b->prec, b->dev_insts, b->count, s);
    if (e == hipSuccess) e = batch_zero(b->counter, s);
    // the LDS-resident kernel needs the tables and its counter: a second fork
    hipStream_t sl = s;
    if (e == hipSuccess && fork) {
        sl = b->side[kSideStreams - 1];
        e = hipEventRecord(b->fork2, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(sl, b->fork2, 0);
    }
    if (e == hipSuccess && b->nlds > 0)
        e = batch_run(b->prec, b->dev_insts, b->dev_order, b->nlds, b->counter + 1, b->grid_lds,
                      true, sl);
    if (e == hipSuccess && b->nsmall > b->nlds)
        e = batch_run(b->prec, b->dev_insts, b->dev_order + b->nlds, b->nsmall - b->nlds,
                      b->counter, b->grid, false, s);
    if (e != hipSuccess) return check_hip(e, "batch launch");
    for (size_t j = 0; j < b->large.size(); ++j) {
        gv_state_s &st = b->states[j];
        st.stream = fork ? b->side[j % kSideStreams] : s;   // after the LDS kernel on the last
        const gv_instance &I = b->large[j];
        if (b->large_q[j] == 0) {   // empty block: the energy alone
            if (gv_status r = gv_apply_ansatz(&st, I.params_dev, &I.ansatz)) return r;
            if (gv_status r = gv_energy(&st, I.h, b->large_e[j])) return r;
            const int64_t P = 2ll * I.ansatz.n * (I.ansatz.layers + I.ansatz.final_rotation);
            if (gv_status r = check_hip(fill_zero_f64(b->large_g[j], (u64)P, st.stream), "zero grad"))
                return r;
            continue;
        }
        if (gv_status r = gv_energy_grad(&st, I.h, I.params_dev, &I.ansatz, b->masks[j],
                                         GV_GRAD_STORE, b->large_e[j], b->large_g[j]))
            return r;
    }
    if (fork) {
        for (int k = 0; k < kSideStreams && e == hipSuccess; ++k) {
            e = hipEventRecord(b->join[k], b->side[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[k], 0);
        }
        if (e != hipSuccess) return check_hip(e, "batch join");
    }
    return GV_OK;
}

}  // namespace
}  // namespace gv

using namespace gv;

extern "C" {

gv_status gv_batch_query(int32_t count, const gv_instance *inst, gv_precision prec,
                         const gv_batch_tuning *tuning, size_t *work_bytes)
{
    if (!work_bytes) return set_error(GV_EINVAL, "work_bytes is NULL");
    if (gv_status r = check_instances(count, inst, prec)) return r;
    *work_bytes = batch_layout(count, inst, prec, split_of(tuning)).total;
    return GV_OK;
}

static gv_status batch_create_impl(int32_t count, const gv_instance *inst,
                                   const gv_cluster *clusters, gv_precision prec,
                                   const gv_batch_tuning *tuning, void *work, size_t work_bytes,
                                   void *stream, int32_t use_graph, double *energies,
                                   double *grads, bool side_streams, gv_batch *out)
{
    if (!out) return set_error(GV_EINVAL, "out is NULL");
    if (gv_status r = check_instances(count, inst, prec)) return r;
    if (count > 0 && (!energies || !grads)) return set_error(GV_EINVAL, "output buffers are NULL");
    std::vector<uint64_t> qmask(count), goff(count);
    {
        uint64_t off = 0;
        for (int i = 0; i < count; ++i) {
            const gv_ansatz &a = inst[i].ansatz;
            const uint64_t all = a.n >= 64 ? ~0ull : ((1ull << a.n) - 1);
            qmask[i] = clusters ? clusters[i].qubit_mask : all;
            if (qmask[i] & ~all)
                return set_error(GV_EINVAL, "cluster %d: qubit mask bit >= n", i);
            goff[i] = off;
            off += 2ull * a.n * (a.layers + a.final_rotation);
        }
    }
    if (!work || ((uintptr_t)work % kAlign)) return set_error(GV_EINVAL, "work must be 256-byte aligned");
    gv_batch_tuning tu = {2, 0, 0, 0};
    if (tuning) tu = *tuning;
    if (tu.blocks_per_cu < 1 || tu.blocks_per_cu > 8 || tu.order < 0 || tu.order > 1 ||
        tu.split_n < 0 || tu.lds_n < -1 || tu.lds_n > 30)
        return set_error(GV_EINVAL, "tuning out of range");
    const int split = split_of(&tu);
    const BatchLayout L = batch_layout(count, inst, prec, split);
    if (work_bytes < L.total)
        return set_error(GV_ESIZE, "work buffer %zu bytes < %zu needed", work_bytes, L.total);

    char *w = (char *)work;
    const int C = std::min(kBatchK - 1, prec == GV_C64 ? 4 : 3);
    std::vector<BatchInst> hi(count);
    std::vector<std::vector<BatchOffPass>> offp(count);
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) {
        const gv_instance &I = inst[i];
        const gv_ansatz &a = I.ansatz;
        const gv_pauli_s *h = I.h;
        BatchInst &b = hi[i];
        memset(&b, 0, sizeof(b));
        TilePlan plan;
        if (!make_tile_plan(a.n, kBatchK, C, &plan))
            return set_error(GV_EUNSUPPORTED, "instance %d: no tile plan", i);
        const Chunks ch = make_chunks(a.n, kBatchK, kBatchLogR);
        b.n = a.n;
        b.layers = a.layers;
        b.rot = a.layers + a.final_rotation;
        b.np = plan.npass;
        b.noff = (int)h->off_passes.size();
        b.zonly = h->ox.empty();
        b.cz = a.ent == GV_ENT_CZ_LINEAR ? 1 : (a.ent == GV_ENT_CZ_CIRCULAR ? 2 : 0);
        b.ntiles = 1ull << (a.n - kBatchK);
        b.qmask = qmask[i];
        b.theta = I.params_dev;
        b.energy = energies + 2 * (size_t)i;
        b.grad = grads + goff[i];
        b.hdiag = h->diag;
        b.cls = h->dev_cls;
        b.terms = h->dev_terms;
        b.offp = (const BatchOffPass *)(w + L.offp[i]);
        b.psi = w + L.psi[i];
        b.lam = w + L.lam[i];
        b.ry = w + L.ry[i];
        b.dtab = w + L.dtab[i];
        b.dtab_stride = L.stride[i];
        b.gtab = w + L.gtab[i];
        b.g0tab = w + L.g0tab[i];
        b.dt_cz = make_diagtab(a, ch, b.dtab, true);
        b.dt_plain = make_diagtab(a, ch, b.dtab, false);
        b.gt = make_diagtab(a, ch, b.gtab, a.layers > 0);
        b.g0 = make_diagtab(a, ch, b.g0tab, false);
        b.ta = make_tab_args(a, ch, L.stride[i]);
        for (int p = 0; p < plan.npass; ++p) {
            pass_runs(plan.pass[p].pos, kBatchK, a.n, &b.pass[p]);
            b.pass[p].active = plan.pass[p].active;
        }
        for (const OffPass &op : h->off_passes) {
            BatchOffPass bo;
            memset(&bo, 0, sizeof(bo));
            pass_runs(op.pos, kBatchK, a.n, &bo.tile);
            bo.c0 = op.c0;
            bo.c1 = op.c1;
            offp[i].push_back(bo);
        }
        cost[i] = (double)(1ull << a.n) * (double)(b.rot * b.np * 3 + b.noff);
    }
    // three classes: LDS-resident, the persistent kernel's, whole-GPU
    const int lds_n = lds_n_of(&tu, prec);
    std::vector<int> order, order_lds, large;
    for (int i = 0; i < count; ++i) {
        const int n = inst[i].ansatz.n;
        if (n >= split) large.push_back(i);
        else if (n <= lds_n) order_lds.push_back(i);
        else order.push_back(i);
    }
    if (tu.order == 0) {
        auto by_cost = [&](int x, int y) { return cost[x] > cost[y]; };
        std::stable_sort(order.begin(), order.end(), by_cost);
        std::stable_sort(order_lds.begin(), order_lds.end(), by_cost);
        std::stable_sort(large.begin(), large.end(), by_cost);
    }
    const int nlds = (int)order_lds.size();
    order.insert(order.begin(), order_lds.begin(), order_lds.end());

    gv_batch b = new (std::nothrow) gv_batch_s;
    if (!b) return set_error(GV_EINVAL, "out of host memory");
    b->count = count;
    b->prec = prec;
    b->work = work;
    b->work_bytes = work_bytes;
    b->stream = (hipStream_t)stream;
    b->dev_insts = (BatchInst *)(w + L.insts);
    b->dev_order = (int *)(w + L.order);
    b->counter = (unsigned *)(w + L.counter);
    b->nsmall = (int)order.size();
    b->side_streams = side_streams;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) b->hgen.push_back({inst[i].h, inst[i].h->prep_gen});
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    b->nlds = nlds;
    b->grid = std::max(1, std::min(b->nsmall - nlds, tu.blocks_per_cu * cus));
    b->grid_lds = std::max(1, std::min(nlds, cus));   // one 99 KB block per CU

    hipError_t e = hipSuccess;
    for (int i : large) {
        const gv_instance &I = inst[i];
        const gv_ansatz &a = I.ansatz;
        const int64_t P = 2ll * a.n * (a.layers + a.final_rotation);
        std::vector<uint8_t> m((size_t)P);
        for (int64_t p = 0; p < P; ++p) m[(size_t)p] = (uint8_t)((qmask[i] >> (p % a.n)) & 1);
        uint8_t *dm = (uint8_t *)(w + L.mask[i]);
        if (e == hipSuccess) e = hipMemcpyAsync(dm, m.data(), m.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // m is about to go
        gv_state_s st;
        st.n = a.n;
        st.prec = prec;
        st.engine = GV_ENGINE_FUSED;
        st.amps = w + L.psi[i];
        st.amps_bytes = ((size_t)1 << a.n) * amp_bytes(prec);
        st.work = w + L.fwork[i];
        st.work_bytes = L.fwork_bytes[i];
        b->large.push_back(I);
        b->large_q.push_back(qmask[i]);
        b->large_e.push_back(energies + 2 * (size_t)i);
        b->large_g.push_back(grads + goff[i]);
        b->states.push_back(st);
        b->masks.push_back(dm);
    }
    if ((!large.empty() || nlds > 0) && side_streams) {
        for (int k = 0; k < kSideStreams && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork2, hipEventDisableTiming);
    }
    if (e == hipSuccess && count > 0) {
        // stream-ordered behind whatever the caller still runs on the work
        // buffer; the host arrays live until the synchronisation below
        e = hipMemcpyAsync(b->dev_insts, hi.data(), hi.size() * sizeof(BatchInst),
                           hipMemcpyHostToDevice, s);
        if (e == hipSuccess && !order.empty())
            e = hipMemcpyAsync(b->dev_order, order.data(), order.size() * sizeof(int),
                               hipMemcpyHostToDevice, s);
        for (int i = 0; i < count && e == hipSuccess; ++i)
            if (!offp[i].empty())
                e = hipMemcpyAsync(w + L.offp[i], offp[i].data(),
                                   offp[i].size() * sizeof(BatchOffPass), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e == hipSuccess && use_graph) {
        e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const gv_status r = launch_all(b, b->capture_stream);
            e = hipStreamEndCapture(b->capture_stream, &b->g);
            if (e == hipSuccess && r != GV_OK) {
                gv_batch_destroy(b);
                return r;
            }
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->g, nullptr, nullptr, 0);
        b->graph = e == hipSuccess;
    }
    if (e != hipSuccess) {
        gv_batch_destroy(b);
        return check_hip(e, "batch setup");
    }
    *out = b;
    return GV_OK;
}

gv_status gv_batch_create(int32_t count, const gv_instance *inst, const gv_cluster *clusters,
                          gv_precision prec, const gv_batch_tuning *tuning, void *work,
                          size_t work_bytes, void *stream, int32_t use_graph, double *energies,
                          double *grads, gv_batch *out)
{
    return batch_create_impl(count, inst, clusters, prec, tuning, work, work_bytes, stream,
                             use_graph, energies, grads, true, out);
}

gv_status gv_batch_run(gv_batch b)
{
    if (!b) return set_error(GV_EINVAL, "batch is NULL");
    for (size_t i = 0; i < b->hgen.size(); ++i)
        if (b->hgen[i].first->prep_gen != b->hgen[i].second || !b->hgen[i].first->prepared)
            return set_error(GV_ESTATE, "instance %zu: its Hamiltonian was prepared again after "
                                        "the batch was created (generation %llu, now %llu, "
                                        "prepared %d)", i, (unsigned long long)b->hgen[i].second,
                             (unsigned long long)b->hgen[i].first->prep_gen,
                             (int)b->hgen[i].first->prepared);
    if (b->graph) return check_hip(hipGraphLaunch(b->exec, b->stream), "graph launch");
    return launch_all(b, b->stream);
}

gv_status gv_batch_destroy(gv_batch b)
{
    if (!b) return GV_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->g) (void)hipGraphDestroy(b->g);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    for (int k = 0; k < kSideStreams; ++k) {
        if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->fork2) (void)hipEventDestroy(b->fork2);
    delete b;
    return GV_OK;
}

gv_status gv_batch_energy_grad(int32_t count, const gv_instance *inst, const gv_cluster *clusters,
                               gv_precision prec, void *work, size_t work_bytes, void *stream,
                               double *energies, double *grads)
{
    gv_batch b = nullptr;
    if (gv_status r = batch_create_impl(count, inst, clusters, prec, nullptr, work, work_bytes,
                                        stream, 0, energies, grads, false, &b))
        return r;
    // everything is enqueued on `stream` (no side streams, no graph) and
    // the launches hold their arguments, so the host handle can go now
    const gv_status r = gv_batch_run(b);
    gv_batch_destroy(b);
    return r;
}

}  // extern "C"
