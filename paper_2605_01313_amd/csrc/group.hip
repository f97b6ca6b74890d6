// Groups of plans: segmented launches over many members, captured in HIP
// graphs.  setpts: per precision, one point-binning launch over every
// member's points, one scan launch (a workgroup per member), one scatter
// launch.  exec: per class of identically shaped members, one theta-pass,
// one phi-pass and one gather launch over all of the class's members, the
// classes as parallel branches of the exec graph.  nufft2_group_run puts
// both in one graph.  The kernels find their member in device tables that
// the host rewrites only when a pointer or a point count changes; the graphs
// hold the launches and are captured once (those holding the setpts
// launches again when the members' point-block counts change).
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "nufft2.h"
#include "nufft2_internal.hpp"
#include "plan_state.hpp"

#define NUFFT2_API extern "C" __attribute__((visibility("default")))

using namespace nufft2;

namespace {

constexpr int kPointBlock = 256;  // threads per block of the setpts point kernels

struct ExecClass {
    int prec = 0;
    std::vector<int> members;
    ThetaJob *d_theta = nullptr;
    PhiJob *d_phi = nullptr;
    GatherJob *d_gather = nullptr;
    std::vector<ThetaJob> h_theta;
    std::vector<PhiJob> h_phi;
    std::vector<GatherJob> h_gather;
};

struct PointSet {
    int prec = 0;
    std::vector<int> members;
    SetptsJob *d_jobs = nullptr;
    int32_t *d_job_of_block = nullptr;
    int64_t block_cap = 0;
    int64_t n_blocks = 0;
    std::vector<SetptsJob> h_jobs;
    std::vector<int32_t> h_job_of_block;
};

// Two plans share an exec class iff every launch parameter but the device
// pointers and the point count agrees.
bool same_class(const nufft2_plan_s *a, const nufft2_plan_s *b)
{
    return a->prec == b->prec && a->Kt == b->Kt && a->Kp == b->Kp && a->F == b->F && a->w == b->w &&
           a->beta == b->beta && a->tile_t == b->tile_t && a->tile_p == b->tile_p &&
           a->real_output == b->real_output && a->hermitian == b->hermitian &&
           a->fields_per_pass == b->fields_per_pass &&
           a->tile_pitch == b->tile_pitch &&
           a->fp.theta_batch == b->fp.theta_batch && a->fp.phi_batch == b->fp.phi_batch &&
           a->fp.theta_ept == b->fp.theta_ept && a->fp.phi_ept == b->fp.phi_ept && a->fp.m_major == b->fp.m_major;
}


// What the tables depend on besides the fixed plan parameters: the call's
// pointers and point counts, and the members' point workspaces (which
// setpts may reallocate).
using Signature = std::vector<uint64_t>;
inline uint64_t sig_of(const void *q) { return (uint64_t)(uintptr_t)q; }

}  // namespace

// Exec classes are independent (disjoint members), so the exec graph runs
// them as parallel branches: class c on branch c mod kExecBranches, branch 0
// on the group's stream, the others on side streams forked from it and
// joined back inside the capture.  A class's kernels then fill the tails and
// launch gaps of another's.
constexpr int kExecBranches = 4;

struct nufft2_group_s {
    std::vector<nufft2_plan_s *> m;
    hipStream_t user_stream = nullptr;  // the members' stream
    hipStream_t stream = nullptr;       // the group's own (capturable) stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<hipStream_t> side;      // exec branches 1.. (default priority)
    std::vector<hipEvent_t> ev_join;    // one per side stream
    hipEvent_t ev_fork = nullptr;
    std::vector<ExecClass> classes;
    std::vector<PointSet> sets;
    hipGraphExec_t g_setpts = nullptr, g_exec = nullptr, g_run = nullptr;
    // shape of the setpts launches: bumped whenever they change; a graph
    // holding them is captured again when its version differs
    uint64_t setpts_version = 1, g_setpts_version = 0, g_run_version = 0;
    Signature setpts_sig, exec_sig;  // of the tables on the device
    int setpts_kernels = 0, exec_kernels = 0;
    size_t table_bytes = 0;
    hipError_t last_err = hipSuccess;
};

namespace {

// The FFT launch shape of a class: its members' parameters, with the
// elements per thread chosen for the launch of the whole class.
FFTParams class_fft_params(const nufft2_group_s *g, const ExecClass &c)
{
    const nufft2_plan_s *p = g->m[c.members[0]];
    FFTParams fp = p->fp;
    fft_launch_shape(p, (int64_t)c.members.size(), fp);
    return fp;
}

}  // namespace

namespace {

template <typename J> bool table_alloc(nufft2_group_s *g, J **ptr, size_t n)
{
    if (hipMalloc((void **)ptr, sizeof(J) * (n ? n : 1)) != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return false;
    }
    g->table_bytes += sizeof(J) * (n ? n : 1);
    return true;
}

void group_free(nufft2_group_s *g)
{
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->g_setpts) (void)hipGraphExecDestroy(g->g_setpts);
    if (g->g_exec) (void)hipGraphExecDestroy(g->g_exec);
    if (g->g_run) (void)hipGraphExecDestroy(g->g_run);
    for (auto &c : g->classes) {
        if (c.d_theta) (void)hipFree(c.d_theta);
        if (c.d_phi) (void)hipFree(c.d_phi);
        if (c.d_gather) (void)hipFree(c.d_gather);
    }
    for (auto &s : g->sets) {
        if (s.d_jobs) (void)hipFree(s.d_jobs);
        if (s.d_job_of_block) (void)hipFree(s.d_job_of_block);
    }
    if (g->ev_in) (void)hipEventDestroy(g->ev_in);
    if (g->ev_out) (void)hipEventDestroy(g->ev_out);
    if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
    for (hipEvent_t ev : g->ev_join)
        if (ev) (void)hipEventDestroy(ev);
    for (hipStream_t st : g->side)
        if (st) (void)hipStreamDestroy(st);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

nufft2_status group_fail(nufft2_group_s *g, hipError_t e)
{
    g->last_err = e;
    (void)hipGetLastError();
    return NUFFT2_ERR_HIP;
}

// Order the group's stream after the work queued so far on the members'
// stream.
hipError_t enter(nufft2_group_s *g)
{
    hipError_t e = hipEventRecord(g->ev_in, g->user_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(g->stream, g->ev_in, 0);
    return e;
}

// Order later work on the members' stream after the group's.
hipError_t leave(nufft2_group_s *g)
{
    hipError_t e = hipEventRecord(g->ev_out, g->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(g->user_stream, g->ev_out, 0);
    return e;
}

// Capture the launches that `body` issues on the group's stream into *exec.
template <typename F> hipError_t capture(nufft2_group_s *g, hipGraphExec_t *exec, F body)
{
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t eb = body();
    e = hipStreamEndCapture(g->stream, &graph);
    if (eb != hipSuccess) e = eb;
    if (e == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    return e;
}

}  // namespace

NUFFT2_API nufft2_status nufft2_group_create(const nufft2_handle *plans, int32_t n, nufft2_group *out)
{
    if (!plans || n < 1 || !out) return NUFFT2_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return NUFFT2_ERR_ARG;
        if (plans[i]->stream != plans[0]->stream || plans[i]->device != plans[0]->device) return NUFFT2_ERR_ARG;
        for (int k = 0; k < i; ++k)
            if (plans[k] == plans[i]) return NUFFT2_ERR_ARG;
    }
    nufft2_group_s *g = new (std::nothrow) nufft2_group_s();
    if (!g) return NUFFT2_ERR_ALLOC;
    g->m.assign(plans, plans + n);
    g->user_stream = plans[0]->stream;
    for (int i = 0; i < n; ++i) {
        bool placed = false;
        for (auto &c : g->classes)
            if (same_class(g->m[c.members[0]], g->m[i])) {
                c.members.push_back(i);
                placed = true;
                break;
            }
        if (!placed) {
            ExecClass c;
            c.prec = g->m[i]->prec;
            c.members.push_back(i);
            g->classes.push_back(c);
        }
        placed = false;
        for (auto &s : g->sets)
            if (s.prec == g->m[i]->prec) {
                s.members.push_back(i);
                placed = true;
                break;
            }
        if (!placed) {
            PointSet s;
            s.prec = g->m[i]->prec;
            s.members.push_back(i);
            g->sets.push_back(s);
        }
    }
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess || dev != plans[0]->device) {
        (void)hipGetLastError();
        delete g;
        return e != hipSuccess ? NUFFT2_ERR_HIP : NUFFT2_ERR_ARG;
    }
    if ((e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming)) != hipSuccess) {
        (void)hipGetLastError();
        group_free(g);
        return NUFFT2_ERR_HIP;
    }
    const int n_side = std::min((int)g->classes.size(), kExecBranches) - 1;
    if (n_side > 0 && (e = hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming)) != hipSuccess) {
        (void)hipGetLastError();
        group_free(g);
        return NUFFT2_ERR_HIP;
    }
    for (int b = 0; b < n_side; ++b) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) == hipSuccess) g->side.push_back(st);
        if (e == hipSuccess && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) == hipSuccess)
            g->ev_join.push_back(ev);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            group_free(g);
            return NUFFT2_ERR_HIP;
        }
    }
    bool ok = true;
    for (auto &c : g->classes) {
        const size_t k = c.members.size();
        ok = ok && table_alloc(g, &c.d_theta, k) && table_alloc(g, &c.d_phi, k) && table_alloc(g, &c.d_gather, k);
    }
    for (auto &s : g->sets) ok = ok && table_alloc(g, &s.d_jobs, s.members.size());
    if (!ok) {
        group_free(g);
        return NUFFT2_ERR_ALLOC;
    }
    g->exec_kernels = 3 * (int)g->classes.size();
    g->setpts_kernels = 3 * (int)g->sets.size();
    *out = g;
    return NUFFT2_OK;
}

namespace {

// setpts, host side: argument checks, point workspaces, the device tables
// (rewritten when a pointer or a count changed).  A change of the setpts
// launches' shape bumps setpts_version.
nufft2_status prepare_setpts(nufft2_group_s *g, const int64_t *n_pts, const double *const *phi_dev,
                             const double *const *theta_dev)
{
    if (!n_pts || !phi_dev || !theta_dev) return NUFFT2_ERR_ARG;
    const int n = (int)g->m.size();
    for (int i = 0; i < n; ++i) {
        if (n_pts[i] < 0 || n_pts[i] > (int64_t)0x7fffffff) return NUFFT2_ERR_ARG;
        if (n_pts[i] > 0 && (!phi_dev[i] || !theta_dev[i])) return NUFFT2_ERR_ARG;
    }
    for (int i = 0; i < n; ++i) {
        nufft2_status st = plan_reserve_points(g->m[i], n_pts[i]);
        if (st != NUFFT2_OK) return st;
    }
    // tables for this call
    Signature sig;
    for (int i = 0; i < n; ++i) {
        const nufft2_plan_s *p = g->m[i];
        sig.insert(sig.end(), {sig_of(phi_dev[i]), sig_of(theta_dev[i]), (uint64_t)n_pts[i], sig_of(p->keyrank),
                               sig_of(p->rec), sig_of(p->perm)});
    }
    const bool rewrite = sig != g->setpts_sig;
    bool recap = false;
    for (auto &s : g->sets) {
        std::vector<SetptsJob> jobs;
        std::vector<int32_t> owner;
        int64_t blocks = 0;
        for (size_t k = 0; k < s.members.size(); ++k) {
            nufft2_plan_s *p = g->m[s.members[k]];
            const int64_t np = n_pts[s.members[k]];
            SetptsJob J{};
            J.phi = phi_dev[s.members[k]];
            J.theta = theta_dev[s.members[k]];
            J.sp = plan_setpts_params(p, np);
            J.bincount = p->bincount;
            J.binstart = p->binstart;
            J.binlist = p->binlist;
            J.nbins = p->nbins;
            J.keyrank = p->keyrank;
            J.rowmark = p->rowmark;
            J.rowtouched = p->rowtouched;
            J.rec = p->rec;
            J.perm = p->perm;
            J.flags = p->flags;
            J.block_begin = (int32_t)blocks;
            const int64_t nb = (np + kPointBlock - 1) / kPointBlock;
            for (int64_t b = 0; b < nb; ++b) owner.push_back((int32_t)k);
            blocks += nb;
            jobs.push_back(J);
        }
        if (blocks > (int64_t)0x7fffffff) return NUFFT2_ERR_ARG;
        if (blocks != s.n_blocks) {
            // bumped now, not after the uploads: a failed upload below must
            // still leave the graphs marked stale for the next call
            recap = true;
            ++g->setpts_version;
        }
        s.h_jobs.swap(jobs);
        s.h_job_of_block.swap(owner);
        s.n_blocks = blocks;
    }
    hipError_t e;
    if (rewrite || recap) {
        // earlier launches of the group may still read the tables
        if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return group_fail(g, e);
        for (auto &s : g->sets) {
            if (s.n_blocks > s.block_cap) {
                if (s.d_job_of_block) (void)hipFree(s.d_job_of_block);
                s.d_job_of_block = nullptr;
                s.block_cap = 0;
                recap = true;
                ++g->setpts_version;
                if (!table_alloc(g, &s.d_job_of_block, (size_t)s.n_blocks)) return NUFFT2_ERR_ALLOC;
                s.block_cap = s.n_blocks;
            }
            if ((e = hipMemcpy(s.d_jobs, s.h_jobs.data(), sizeof(SetptsJob) * s.h_jobs.size(),
                               hipMemcpyHostToDevice)) != hipSuccess)
                return group_fail(g, e);
            if (s.n_blocks > 0 &&
                (e = hipMemcpy(s.d_job_of_block, s.h_job_of_block.data(), sizeof(int32_t) * s.h_job_of_block.size(),
                               hipMemcpyHostToDevice)) != hipSuccess)
                return group_fail(g, e);
        }
        g->setpts_sig = sig;
    }
    return NUFFT2_OK;
}

// The setpts launches, on the group's stream.
hipError_t issue_setpts(nufft2_group_s *g)
{
    for (auto &s : g->sets) {
        hipError_t es = launch_setpts_group(s.prec, s.d_jobs, (int)s.members.size(), s.d_job_of_block,
                                            (int)s.n_blocks, g->stream);
        if (es != hipSuccess) return es;
    }
    return hipSuccess;
}

// After setpts: the members' point counts; group setpts does not rotate.
void commit_setpts(nufft2_group_s *g, const int64_t *n_pts)
{
    for (size_t i = 0; i < g->m.size(); ++i) {
        g->m[i]->n_pts = n_pts[i];
        g->m[i]->rot_u = g->m[i]->rot_v = -1;
    }
}

// exec, host side: argument checks and the device tables (rewritten when a
// pointer or a point count changed; the graph launches stay the same).
nufft2_status prepare_exec(nufft2_group_s *g, const void *const *coeffs_dev, void *const *out_dev)
{
    if (!coeffs_dev || !out_dev) return NUFFT2_ERR_ARG;
    const int n = (int)g->m.size();
    for (int i = 0; i < n; ++i) {
        if (g->m[i]->n_pts < 0) return NUFFT2_ERR_NO_POINTS;
        if (!coeffs_dev[i] || !out_dev[i]) return NUFFT2_ERR_ARG;
    }
    Signature sig;
    for (int i = 0; i < n; ++i) {
        const nufft2_plan_s *p = g->m[i];
        sig.insert(sig.end(), {sig_of(coeffs_dev[i]), sig_of(out_dev[i]), (uint64_t)p->n_pts, sig_of(p->rec),
                               sig_of(p->perm)});
    }
    const bool rewrite = sig != g->exec_sig;
    for (auto &c : g->classes) {
        if (!rewrite) break;
        std::vector<ThetaJob> th;
        std::vector<PhiJob> ph;
        std::vector<GatherJob> ga;
        const FFTParams cfp = class_fft_params(g, c);
        for (int i : c.members) {
            nufft2_plan_s *p = g->m[i];
            ThetaJob tj{};
            tj.coeffs = coeffs_dev[i];
            tj.fac_t = p->twist_t;
            tj.corr_p = p->corr_p;
            tj.tws = p->tw_t;
            tj.touched = p->rowtouched;
            tj.S = p->S;
            tj.fp = cfp;
            th.push_back(tj);
            PhiJob pj{};
            pj.S = p->S;
            pj.tws = p->tw_p;
            pj.c2r = p->c2r;
            pj.touched = p->rowtouched;
            pj.grid = p->grid;
            pj.fp = cfp;
            ph.push_back(pj);
            GatherJob gj{};
            gj.grid = p->grid;
            gj.rec = p->rec;
            gj.perm = p->perm;
            gj.binlist = p->binlist;
            gj.out = out_dev[i];
            gj.gp = plan_gather_params(p);
            ga.push_back(gj);
        }
        c.h_theta.swap(th);
        c.h_phi.swap(ph);
        c.h_gather.swap(ga);
    }
    hipError_t e;
    if (rewrite) {
        if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return group_fail(g, e);
        for (auto &c : g->classes) {
            const size_t k = c.members.size();
            if ((e = hipMemcpy(c.d_theta, c.h_theta.data(), sizeof(ThetaJob) * k, hipMemcpyHostToDevice)) !=
                    hipSuccess ||
                (e = hipMemcpy(c.d_phi, c.h_phi.data(), sizeof(PhiJob) * k, hipMemcpyHostToDevice)) != hipSuccess ||
                (e = hipMemcpy(c.d_gather, c.h_gather.data(), sizeof(GatherJob) * k, hipMemcpyHostToDevice)) !=
                    hipSuccess)
                return group_fail(g, e);
        }
        g->exec_sig = sig;
    }
    return NUFFT2_OK;
}

// The exec launches: every class's theta pass, phi pass and gather, the
// classes as parallel branches forked from the group's stream and joined
// back into it.
hipError_t issue_exec(nufft2_group_s *g)
{
    // fork: the side streams join the capture by waiting on an event of
    // the captured stream
    hipError_t es = hipSuccess;
    if (!g->side.empty()) es = hipEventRecord(g->ev_fork, g->stream);
    for (size_t b = 0; es == hipSuccess && b < g->side.size(); ++b) es = hipStreamWaitEvent(g->side[b], g->ev_fork, 0);
    for (size_t ci = 0; es == hipSuccess && ci < g->classes.size(); ++ci) {
        const ExecClass &c = g->classes[ci];
        const int br = (int)(ci % (g->side.size() + 1));
        hipStream_t st = br == 0 ? g->stream : g->side[br - 1];
        const nufft2_plan_s *p = g->m[c.members[0]];
        const int k = (int)c.members.size();
        const FFTParams cfp = class_fft_params(g, c);
        es = launch_theta_group(c.prec, cfp, c.d_theta, k, st);
        if (es == hipSuccess) es = launch_phi_group(c.prec, cfp, c.d_phi, k, st);
        if (es == hipSuccess) es = launch_gather_group(c.prec, plan_gather_params(p), c.d_gather, k, st);
    }
    // join every side stream back (also after an error, so that a capture
    // can end)
    for (size_t b = 0; b < g->side.size(); ++b) {
        hipError_t ej = hipEventRecord(g->ev_join[b], g->side[b]);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(g->stream, g->ev_join[b], 0);
        if (es == hipSuccess) es = ej;
    }
    return es;
}

// Launch a graph between the members' stream's earlier and later work.
nufft2_status launch_graph(nufft2_group_s *g, hipGraphExec_t exec)
{
    hipError_t e;
    if ((e = enter(g)) != hipSuccess || (e = hipGraphLaunch(exec, g->stream)) != hipSuccess ||
        (e = leave(g)) != hipSuccess)
        return group_fail(g, e);
    return NUFFT2_OK;
}

}  // namespace

NUFFT2_API nufft2_status nufft2_group_setpts(nufft2_group g, const int64_t *n_pts, const double *const *phi_dev,
                                             const double *const *theta_dev)
{
    if (!g) return NUFFT2_ERR_ARG;
    nufft2_status st = prepare_setpts(g, n_pts, phi_dev, theta_dev);
    if (st != NUFFT2_OK) return st;
    if (!g->g_setpts || g->g_setpts_version != g->setpts_version) {
        if (g->g_setpts) (void)hipGraphExecDestroy(g->g_setpts);
        g->g_setpts = nullptr;
        hipError_t e = capture(g, &g->g_setpts, [&]() { return issue_setpts(g); });
        if (e != hipSuccess) {
            g->g_setpts = nullptr;
            return group_fail(g, e);
        }
        g->g_setpts_version = g->setpts_version;
    }
    if ((st = launch_graph(g, g->g_setpts)) != NUFFT2_OK) return st;
    commit_setpts(g, n_pts);
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_group_exec(nufft2_group g, const void *const *coeffs_dev, void *const *out_dev)
{
    if (!g) return NUFFT2_ERR_ARG;
    nufft2_status st = prepare_exec(g, coeffs_dev, out_dev);
    if (st != NUFFT2_OK) return st;
    if (!g->g_exec) {
        hipError_t e = capture(g, &g->g_exec, [&]() { return issue_exec(g); });
        if (e != hipSuccess) {
            g->g_exec = nullptr;
            return group_fail(g, e);
        }
    }
    return launch_graph(g, g->g_exec);
}

NUFFT2_API nufft2_status nufft2_group_run(nufft2_group g, const int64_t *n_pts, const double *const *phi_dev,
                                          const double *const *theta_dev, const void *const *coeffs_dev,
                                          void *const *out_dev)
{
    if (!g || !n_pts || !phi_dev || !theta_dev || !coeffs_dev || !out_dev) return NUFFT2_ERR_ARG;
    const int n = (int)g->m.size();
    for (int i = 0; i < n; ++i)
        if (!coeffs_dev[i] || !out_dev[i]) return NUFFT2_ERR_ARG;
    nufft2_status st = prepare_setpts(g, n_pts, phi_dev, theta_dev);
    if (st != NUFFT2_OK) return st;
    // the exec tables take the new point counts (and workspaces)
    std::vector<int64_t> old(n);
    for (int i = 0; i < n; ++i) {
        old[i] = g->m[i]->n_pts;
        g->m[i]->n_pts = n_pts[i];
    }
    st = prepare_exec(g, coeffs_dev, out_dev);
    if (st != NUFFT2_OK) {
        for (int i = 0; i < n; ++i) g->m[i]->n_pts = old[i];
        return st;
    }
    if (!g->g_run || g->g_run_version != g->setpts_version) {
        if (g->g_run) (void)hipGraphExecDestroy(g->g_run);
        g->g_run = nullptr;
        hipError_t e = capture(g, &g->g_run, [&]() {
            hipError_t es = issue_setpts(g);
            return es == hipSuccess ? issue_exec(g) : es;
        });
        if (e != hipSuccess) {
            g->g_run = nullptr;
            for (int i = 0; i < n; ++i) g->m[i]->n_pts = old[i];
            return group_fail(g, e);
        }
        g->g_run_version = g->setpts_version;
    }
    st = launch_graph(g, g->g_run);
    if (st != NUFFT2_OK) {
        for (int i = 0; i < n; ++i) g->m[i]->n_pts = old[i];
        return st;
    }
    commit_setpts(g, n_pts);
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_group_destroy(nufft2_group g)
{
    if (!g) return NUFFT2_OK;
    group_free(g);
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_group_get_info(nufft2_group g, nufft2_group_info *info)
{
    if (!g || !info) return NUFFT2_ERR_ARG;
    memset(info, 0, sizeof(*info));
    info->n_members = (int32_t)g->m.size();
    info->n_classes = (int32_t)g->classes.size();
    info->setpts_kernels = g->setpts_kernels;
    info->exec_kernels = g->exec_kernels;
    info->table_bytes = g->table_bytes;
    return NUFFT2_OK;
}
