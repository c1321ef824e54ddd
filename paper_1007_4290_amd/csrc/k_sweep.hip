// Dispatch of the sweep (Alg. 2.4) to its compiled instantiations and the
// launch geometry shared with the host code.
#include "sweep_impl.hpp"

#define HSWEEP_SWEEP_DECLARE(BB, RR, LL)     \
    HSWEEP_SWEEP_SIG(f, float, BB, RR, LL);  \
    HSWEEP_SWEEP_SIG(d, double, BB, RR, LL);
HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_DECLARE)
HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_DECLARE)
HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_DECLARE)

#define HSWEEP_SWEEP_IS(BB, RR, LL) (p.b == (BB) && p.L == (LL) && ((LL) == 0 || p.r == (RR)))

namespace {
void call_sweep(const Plan& p, const SweepArgs<float>& a, size_t lds, int th, hipStream_t s, bool& done) {
#define HSWEEP_SWEEP_CALL(BB, RR, LL) \
    if (!done && HSWEEP_SWEEP_IS(BB, RR, LL)) { HSWEEP_SWEEP_NAME(f, BB, RR, LL)(p, a, lds, th, s); done = true; }
    HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_CALL)
#undef HSWEEP_SWEEP_CALL
}
void call_sweep(const Plan& p, const SweepArgs<double>& a, size_t lds, int th, hipStream_t s, bool& done) {
#define HSWEEP_SWEEP_CALL(BB, RR, LL) \
    if (!done && HSWEEP_SWEEP_IS(BB, RR, LL)) { HSWEEP_SWEEP_NAME(d, BB, RR, LL)(p, a, lds, th, s); done = true; }
    HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_CALL)
    HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_CALL)
#undef HSWEEP_SWEEP_CALL
}
}  // namespace

size_t sweep_lds_bytes(const Plan& p, size_t elem) {
    size_t e = (size_t)p.np + (size_t)((1 << (p.L + 1)) - 1) * p.r + (size_t)((1 << p.L) - 1) * 2 * p.r;
    return e * elem;
}

int sweep_threads(const Plan& p) {
    int t = p.np < 64 ? 64 : p.np;
    int need = ((1 << p.L) - 1) * 2 * p.r;    // core rows, one per thread
    if (need > t) t = need;
    return (t + 63) / 64 * 64;
}

bool sweep_supported(const Plan& p) {
    if (sweep_threads(p) > 1024) return false;
    #define HSWEEP_SWEEP_MATCH(BB, RR, LL) \
    if (p.b == BB && p.L == LL && (LL == 0 || p.r == RR)) return true;
    HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_MATCH)
    HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_MATCH)
    HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_MATCH)
#undef HSWEEP_SWEEP_MATCH
    return false;
}

template <typename T>
int launch_sweep(const Plan& p, const SweepArgs<T>& a, hipStream_t s) {
    size_t lds = sweep_lds_bytes(p, sizeof(cpx<T>));
    int th = sweep_threads(p);
    bool done = false;
    call_sweep(p, a, lds, th, s, done);
    return done ? 0 : -1;
}

template int launch_sweep<float>(const Plan&, const SweepArgs<float>&, hipStream_t);
template int launch_sweep<double>(const Plan&, const SweepArgs<double>&, hipStream_t);
