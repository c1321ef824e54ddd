// Factorization kernels for complex64, and the host-side plan checks.
#include "factor_impl.hpp"

// Largest dynamic LDS (bytes) any factorization kernel needs for this plan.
size_t factor_lds_bytes(const Plan& p, size_t elem) {
    size_t mx = (size_t)(2 * p.L * p.b * p.r + p.L * p.r * p.r + 1);
    if (mx < (size_t)p.b * p.b) mx = (size_t)p.b * p.b;
    if (mx < (size_t)5 * p.r * p.r) mx = (size_t)5 * p.r * p.r;
    mx *= elem;
    for (int lam = 1; lam <= p.L; ++lam) {
        int s = p.np >> lam;
        RecompLayout l = recomp_layout(s, 1 + p.r * lam, p.r, lam * p.r * p.r, elem, elem,
                                       gram_path(elem, p.tol, 1 + p.r * lam));
        size_t a = l.gEnd * sizeof(c128);
        size_t w = wood_layout(s, p.r, p.b, p.L, lam).oEnd * elem;
        if (a > mx) mx = a;
        if (w > mx) mx = w;
    }
    return mx;
}

bool factor_supported(const Plan& p) {
    bool leaf_ok = p.b == 4 || p.b == 8 || p.b == 16 || p.b == 32 || p.b == 64;
    if (!leaf_ok) return false;
    if (p.L == 0) return true;
    return p.r == 2 || p.r == 4 || p.r == 8 || p.r == 16;
}

template void factor_kernels_init<float>();
template int launch_factor_layer<float>(const InstDesc<float>*, const Plan*, int, int, hipStream_t, hipEvent_t);
