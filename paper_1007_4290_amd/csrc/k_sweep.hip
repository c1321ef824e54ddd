// Dispatch of the sweep (Alg. 2.4) to its compiled instantiations, the
// workgroup placement and the launch geometry shared with the host code.
#include "sweep_impl.hpp"

#define HSWEEP_SWEEP_DECLARE_G(BB, RR, LL, GG)    \
    HSWEEP_SWEEP_SIG(f, float, BB, RR, LL, GG);   \
    HSWEEP_SWEEP_SIG(d, double, BB, RR, LL, GG);
#define HSWEEP_SWEEP_DECLARE(BB, RR, LL) HSWEEP_SWEEP_DECLARE_G(BB, RR, LL, 1)
#define HSWEEP_SWEEP_DECLARE4(BB, RR, LL) HSWEEP_SWEEP_DECLARE_G(BB, RR, LL, 4)
HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_DECLARE)
HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_DECLARE)
HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_DECLARE)
HSWEEP_SWEEP_LIST_G4(HSWEEP_SWEEP_DECLARE4)

namespace {

// A compiled kernel for leaf b, rank r (ignored without levels), levels L
// and group size G.
#define HSWEEP_SWEEP_IS(BB, RR, LL) (b == (BB) && L == (LL) && ((LL) == 0 || r == (RR)))

bool call_sweep(int b, int r, int L, int G, const SweepArgs<float>& a, int blocks, size_t lds, hipStream_t s) {
    bool done = false;
#define HSWEEP_SWEEP_CALL(BB, RR, LL) \
    if (!done && G == 1 && HSWEEP_SWEEP_IS(BB, RR, LL)) { HSWEEP_SWEEP_NAME(f, BB, RR, LL, 1)(a, blocks, lds, s); done = true; }
#define HSWEEP_SWEEP_CALL4(BB, RR, LL) \
    if (!done && G == 4 && HSWEEP_SWEEP_IS(BB, RR, LL)) { HSWEEP_SWEEP_NAME(f, BB, RR, LL, 4)(a, blocks, lds, s); done = true; }
    HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_G4(HSWEEP_SWEEP_CALL4)
#undef HSWEEP_SWEEP_CALL
#undef HSWEEP_SWEEP_CALL4
    return done;
}

bool call_sweep(int b, int r, int L, int G, const SweepArgs<double>& a, int blocks, size_t lds, hipStream_t s) {
    bool done = false;
#define HSWEEP_SWEEP_CALL(BB, RR, LL) \
    if (!done && G == 1 && HSWEEP_SWEEP_IS(BB, RR, LL)) { HSWEEP_SWEEP_NAME(d, BB, RR, LL, 1)(a, blocks, lds, s); done = true; }
#define HSWEEP_SWEEP_CALL4(BB, RR, LL) \
    if (!done && G == 4 && HSWEEP_SWEEP_IS(BB, RR, LL)) { HSWEEP_SWEEP_NAME(d, BB, RR, LL, 4)(a, blocks, lds, s); done = true; }
    HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_G4(HSWEEP_SWEEP_CALL4)
#undef HSWEEP_SWEEP_CALL
#undef HSWEEP_SWEEP_CALL4
    return done;
}

bool has_kernel(int b, int r, int L, int G) {
#define HSWEEP_SWEEP_MATCH(BB, RR, LL) \
    if (G == 1 && HSWEEP_SWEEP_IS(BB, RR, LL)) return true;
#define HSWEEP_SWEEP_MATCH4(BB, RR, LL) \
    if (G == 4 && HSWEEP_SWEEP_IS(BB, RR, LL)) return true;
    HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_MATCH)
    HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_MATCH)
    HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_MATCH)
    HSWEEP_SWEEP_LIST_G4(HSWEEP_SWEEP_MATCH4)
#undef HSWEEP_SWEEP_MATCH
#undef HSWEEP_SWEEP_MATCH4
    return false;
}

int threads_for(int b, int r, int L) {
    int t = (b << L) < 64 ? 64 : (b << L);
    const int need = ((1 << L) - 1) * 2 * r;    // core rows, one per thread
    if (need > t) t = need;
    return (t + 63) / 64 * 64;
}

}  // namespace

size_t sweep_lds_bytes(const Plan& p, size_t elem, int G) {
    size_t e = (size_t)p.np + (size_t)((1 << (p.L + 1)) - 1) * p.r + (size_t)((1 << p.L) - 1) * 2 * p.r;
    return e * (size_t)G * elem;
}

bool sweep_supported(const Plan& p) {
    if (threads_for(p.b, p.r, p.L) > 1024) return false;
    return has_kernel(p.b, p.r, p.L, 1);
}

bool sweep_group_supported(const Plan& p) { return has_kernel(p.b, p.r, p.L, 4); }

// One instance: nrhs right-hand sides in groups of G, the groups spread over
// as few XCDs as hold them at one workgroup per compute unit (32 per XCD),
// so that the workgroups that read the same layers share an L2.
template <typename T>
int launch_sweep(const Plan& p, SweepArgs<T> a, int G, hipStream_t s) {
    const int groups = (a.one.nrhs + G - 1) / G;
    int nxcd = (groups + 31) / 32;
    if (nxcd > 8) nxcd = 8;
    a.insts = nullptr;
    a.tasks = nullptr;
    a.ngroups = groups;
    a.nxcd = nxcd;
    const int blocks = 8 * ((groups + nxcd - 1) / nxcd);
    const size_t lds = sweep_lds_bytes(p, sizeof(cpx<T>), G);
    return call_sweep(p.b, p.r, p.L, G, a, blocks, lds, s) ? 0 : -1;
}

// Several instances in one launch, call column (jf, ju) of the fields: the
// kernel compiled for the largest level count among them (same leaf size
// and rank).  `tasks` is a device table of `blocks` entries built by
// sweep_task_table.
template <typename T>
int launch_sweep_multi_col(const Plan* plans, int ninst, const SweepInst<T>* insts, const int* tasks, int blocks,
                           int G, int jf, int ju, hipStream_t s) {
    int Lmax = 0;
    size_t lds = 0;
    int r = plans[0].r;
    for (int q = 0; q < ninst; ++q) {
        if (plans[q].b != plans[0].b) return -1;
        if (plans[q].L > Lmax) Lmax = plans[q].L;
        if (plans[q].L > 0) r = plans[q].r;
        const size_t l = sweep_lds_bytes(plans[q], sizeof(cpx<T>), G);
        if (l > lds) lds = l;
    }
    SweepArgs<T> a{};
    a.insts = insts;
    a.tasks = tasks;
    a.jf = jf;
    a.ju = ju;
    return call_sweep(plans[0].b, r, Lmax, G, a, blocks, lds, s) ? 0 : -1;
}

template int launch_sweep<float>(const Plan&, SweepArgs<float>, int, hipStream_t);
template int launch_sweep<double>(const Plan&, SweepArgs<double>, int, hipStream_t);
template int launch_sweep_multi_col<float>(const Plan*, int, const SweepInst<float>*, const int*, int, int, int, int,
                                           hipStream_t);
template int launch_sweep_multi_col<double>(const Plan*, int, const SweepInst<double>*, const int*, int, int, int, int,
                                            hipStream_t);
