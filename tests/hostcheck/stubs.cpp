// Stand-ins of the kernel launchers: each checks that every device range the
// kernel would read or write lies inside a live allocation, and aborts with
// the range otherwise.  The dot products return 1.
#include <stdio.h>
#include <stdlib.h>
#include <complex>
#include "internal.hpp"
void fake_describe(const void* p);
static void need(const void* p, size_t b, const char* what) {
    if (b && !fake_in_alloc(p, b)) { fprintf(stderr, "OUT OF RANGE: %s %p %zu\n", what, p, b); fake_describe(p); abort(); }
}
void launch_pml_1d(int n, double, double, double, double, c128* isn, c128* sh, hipStream_t) {
    need(isn, n * 16, "isn"); need(sh, (n + 1) * 16, "sh");
}
static void need_tables(const AxisTables& t, int n) {
    need(t.isn1, n * 16, "isn1"); need(t.sh1, (n + 1) * 16, "sh1");
    need(t.isn2, n * 16, "isn2"); need(t.sh2, (n + 1) * 16, "sh2");
}
template <typename T>
void launch_layer_coeffs(int n, int np, int dir, double, const double* c, const AxisTables& t, cpx<T>* dg,
                         cpx<T>* eo, cpx<T>* cp, hipStream_t) {
    if (dir < 0 || dir > 3) { fprintf(stderr, "direction %d\n", dir); abort(); }
    need(c, (size_t)n * n * 8, "c"); need_tables(t, n); need(dg, (size_t)n * np * sizeof(cpx<T>), "dg");
    need(eo, (size_t)n * np * sizeof(cpx<T>), "eo"); need(cp, (size_t)(n - 1) * np * sizeof(cpx<T>), "cp");
}
template void launch_layer_coeffs<float>(int, int, int, double, const double*, const AxisTables&, c64*, c64*, c64*,
                                         hipStream_t);
template void launch_layer_coeffs<double>(int, int, int, double, const double*, const AxisTables&, c128*, c128*, c128*,
                                          hipStream_t);
void launch_stencil(int n, int nrhs, double, const double* c, const AxisTables& t, const c128* x, const c128* f,
                    c128* y, const int* active, hipStream_t) {
    size_t N = (size_t)n * n;
    need(c, N * 8, "st c"); need_tables(t, n);
    need(x, nrhs * N * 16, "st x"); if (f) need(f, nrhs * N * 16, "st f"); need(y, nrhs * N * 16, "st y");
    if (active) need(active, nrhs * 4, "st active");
}
void launch_grad(int n, int nrhs, double, const double* c, const AxisTables& t, const c128* u, const c128* mu,
                 double* grad, hipStream_t) {
    size_t N = (size_t)n * n;
    need(c, N * 8, "gr c"); need_tables(t, n); need(u, nrhs * N * 16, "gr u"); need(mu, nrhs * N * 16, "gr mu");
    need(grad, N * 8, "grad");
}
void launch_dirichlet(int n, int nrhs, double, const double* c, const AxisTables& t, int edge, const c128* b, c128* f,
                      hipStream_t) {
    if (edge < 0 || edge > 3) abort();
    need(c, (size_t)n * n * 8, "di c"); need_tables(t, n); need(b, nrhs * n * 16, "di b");
    need(f, (size_t)nrhs * n * n * 16, "di f");
}
// Layer step m of each instance reads layer m-1 of its factor store and its
// couplings, writes layer m, and uses the shared Q, G, rank and status buffers.
template <typename T>
int launch_factor_layer(const InstDesc<T>* descs, const Plan* plans, int ninst, int m, hipStream_t, hipEvent_t) {
    need(descs, ninst * sizeof(InstDesc<T>), "descs");
    for (int q = 0; q < ninst; ++q) {
        const InstDesc<T>& d = descs[q];
        const Plan& p = plans[q];
        if (d.p.n != p.n || d.p.np != p.np || d.p.L != p.L || d.p.eLayer != p.eLayer) {
            fprintf(stderr, "descriptor %d does not match its plan\n", q); abort();
        }
        if (p.b != plans[0].b || (p.L > 0 && plans[0].L > 0 && p.r != plans[0].r)) return -1;
        if (m >= p.n) continue;
        const size_t e = sizeof(cpx<T>);
        need(d.fac + (size_t)m * p.eLayer, p.eLayer * e, "fac layer m");
        if (m > 0) {
            need(d.fac + (size_t)(m - 1) * p.eLayer, p.eLayer * e, "fac layer m-1");
            need(d.cp + (size_t)(m - 1) * p.np, p.np * e, "factor cp");
        }
        need(d.dg + (size_t)m * p.np, p.np * e, "factor dg");
        need(d.eo + (size_t)m * p.np, p.np * e, "factor eo");
        if (p.L > 0) {
            need(d.Q, (size_t)p.L * p.r * p.np * e, "Q");
            need(d.G, ((size_t)2 << p.L) * p.r * p.r * e, "G");
        }
        need(d.rank + (size_t)m * (1 << p.L), (size_t)(1 << p.L) * 4, "rank");
        need(d.status, 4, "status");
    }
    return 0;
}
template int launch_factor_layer<float>(const InstDesc<float>*, const Plan*, int, int, hipStream_t, hipEvent_t);
template int launch_factor_layer<double>(const InstDesc<double>*, const Plan*, int, int, hipStream_t, hipEvent_t);
template <typename T> void factor_kernels_init() {}
template void factor_kernels_init<float>();
template void factor_kernels_init<double>();
size_t factor_lds_bytes(const Plan&, size_t) { return 1024; }
bool factor_supported(const Plan&) { return true; }
size_t sweep_lds_bytes(const Plan& p, size_t elem, int G) {
    size_t e = (size_t)p.np + (size_t)((1 << (p.L + 1)) - 1) * p.r + (size_t)((1 << p.L) - 1) * 2 * p.r;
    return e * (size_t)G * elem;
}
bool sweep_supported(const Plan&) { return true; }
bool sweep_group_supported(const Plan&) { return true; }
template <typename T>
static void check_inst(const SweepInst<T>& in, int jf, int ju, const char* tag) {
    size_t N = (size_t)in.n * in.n;
    need(in.fac, (size_t)in.n * in.eLayer * sizeof(cpx<T>), "fac");
    if (in.n > 1) need(in.cp, (size_t)(in.n - 1) * in.np * sizeof(cpx<T>), "cp");
    need(in.f + (size_t)jf * in.fstride, in.nrhs * N * 16, tag);
    need(in.u + (size_t)ju * in.ustride, in.nrhs * N * 16, tag);
    need(in.w, (size_t)in.nrhs * in.n * in.np * sizeof(cpx<T>), tag);
    if (in.active) need(in.active, in.nrhs * 4, "active");
}
template <typename T> int launch_sweep(const Plan&, SweepArgs<T> a, int, hipStream_t) {
    check_inst(a.one, a.jf, a.ju, "single f/u"); return 0;
}
template int launch_sweep<float>(const Plan&, SweepArgs<float>, int, hipStream_t);
template int launch_sweep<double>(const Plan&, SweepArgs<double>, int, hipStream_t);
static int g_multi = 0;
template <typename T>
int launch_sweep_multi_col(const Plan* plans, int ninst, const SweepInst<T>* insts, const int* tasks, int blocks,
                           int, int jf, int ju, hipStream_t) {
    need(insts, ninst * sizeof(SweepInst<T>), "insts");
    need(tasks, blocks * 4, "tasks");
    for (int b = 0; b < blocks; ++b) {
        int t = tasks[b];
        if (t < 0) continue;
        int q = t >> 16, r0 = t & 0xffff;
        if (q >= ninst) { fprintf(stderr, "task instance %d >= %d\n", q, ninst); abort(); }
        if (r0 >= insts[q].nrhs) { fprintf(stderr, "task rhs\n"); abort(); }
        if (insts[q].n != plans[q].n || insts[q].np != plans[q].np) { fprintf(stderr, "plan mismatch q=%d\n", q); abort(); }
        check_inst(insts[q], jf, ju, "multi f/u");
    }
    ++g_multi;
    return 0;
}
template int launch_sweep_multi_col<float>(const Plan*, int, const SweepInst<float>*, const int*, int, int, int, int, hipStream_t);
template int launch_sweep_multi_col<double>(const Plan*, int, const SweepInst<double>*, const int*, int, int, int, int, hipStream_t);
int krylov_dot_blocks(size_t N) { size_t b = (N + 8191) / 8192; if (b < 1) b = 1; if (b > 256) b = 256; return (int)b; }
void launch_conj(const c128* x, c128* y, size_t n, hipStream_t) { need(x, n * 16, "conj x"); need(y, n * 16, "conj y"); }
void launch_multi_dot(const c128* V, int nv, size_t ld, const c128* w, const size_t* off, int S, c128* partial,
                      c128* out, int nblk, hipStream_t) {
    need(off, (S + 1) * 8, "off");
    for (int j = 0; j < nv; ++j) need(V + j * ld, off[S] * 16, "dot V");
    need(w, off[S] * 16, "dot w"); need(partial, (size_t)nblk * S * nv * 16, "partial"); need(out, nv * S * 16, "dot out");
    for (int i = 0; i < nv * S; ++i) out[i] = mk<double>(1.0, 0.0);
}
void launch_multi_axpy(const c128* V, int nv, size_t ld, const c128* h, c128* w, const size_t* off, int S, size_t,
                       hipStream_t) {
    for (int j = 0; j < nv; ++j) need(V + j * ld, off[S] * 16, "axpy V");
    need(h, nv * S * 16, "axpy h"); need(w, off[S] * 16, "axpy w");
}
void launch_scale(const c128* w, const double* sc, c128* out, const size_t* off, int S, size_t, hipStream_t) {
    need(w, off[S] * 16, "scale w"); need(sc, S * 8, "scale sc"); need(out, off[S] * 16, "scale out");
}
void launch_combine(const c128* Z, int nz, size_t ld, const c128* y, c128* x, const size_t* off, int S, size_t,
                    hipStream_t) {
    for (int j = 0; j < nz; ++j) need(Z + j * ld, off[S] * 16, "combine Z");
    need(y, nz * S * 16, "combine y"); need(x, off[S] * 16, "combine x");
}
int multi_launches() { return g_multi; }
void launch_small_qr(int p, int k, const c128* A, int lda, c128* W, c128* Vh, c128* Q, c128* R, c128* Qc,
                     hipStream_t) {
    const int kk = p < k ? p : k;
    if (Qc) need(Qc, (size_t)p * kk * 16, "qr conj(Q)");
    if (k > 0) need(A, ((size_t)(k - 1) * lda + p) * 16, "qr A");
    need(W, (size_t)p * k * 16, "qr W"); need(Vh, (size_t)p * kk * 16, "qr Vh");
    need(Q, (size_t)p * kk * 16, "qr Q"); need(R, (size_t)kk * k * 16, "qr R");
}
void launch_small_svd(int a, int b, c128* A, int lda, c128* V, double* sig, int* perm, int* rank, double, int,
                      hipStream_t) {
    if (b > 0) need(A, ((size_t)(b - 1) * lda + a) * 16, "svd A");
    need(V, (size_t)b * b * 16, "svd V"); need(sig, (size_t)b * 8, "svd sig"); need(perm, (size_t)b * 4, "svd perm");
    need(rank, 4, "svd rank");
}
void launch_small_inv(int m, const c128* A, int lda, c128* W, c128* X, int* status, hipStream_t) {
    if (m > 0) need(A, ((size_t)(m - 1) * lda + m) * 16, "inv A");
    need(W, (size_t)m * (m + 1) * 16, "inv W"); need(X, (size_t)m * m * 16, "inv X"); need(status, 4, "inv status");
}
static void recompress_ranges(int m, int q, int k1, int k2, int rmax, const c128* au, const c128* av,
                              const c128* U, int ldu, const c128* V, int ldv, c128* work, c128* ou, c128* ov) {
    const int k = k1 + k2, kk1 = m < k ? m : k, kk2 = q < k ? q : k;
    const int r0 = kk1 < kk2 ? kk1 : kk2, r = r0 < rmax ? r0 : rmax;
    need(au, (size_t)m * k1 * 16, "recompress au"); need(av, (size_t)q * k1 * 16, "recompress av");
    if (k2 > 0) { need(U, ((size_t)(k2 - 1) * ldu + m) * 16, "recompress U"); need(V, ((size_t)(k2 - 1) * ldv + q) * 16, "recompress V"); }
    need(work, recompress_layout(m, q, k, rmax).total * 16, "recompress work");
    need(ou, (size_t)m * r * 16, "recompress ou"); need(ov, (size_t)q * r * 16, "recompress ov");
}
void launch_block_jobs(const BlockJob* jobs, int count, int rmax, double, hipStream_t) {
    for (int j = 0; j < count; ++j) {
        const BlockJob& J = jobs[j];
        if (J.kind != JOB_RECOMPRESS) {
            const size_t n = (size_t)J.m * J.q * 16;
            need(J.ou, n, "block job out");
            if (J.kind == JOB_SUM) { need(J.au, n, "sum a"); need(J.av, n, "sum b"); }
            if (J.kind == JOB_SCALE || J.kind == JOB_COPY) need(J.au, n, "scaled/copied block");
            if (J.kind == JOB_SCALE) { need(J.U, (size_t)J.m * 16, "row scale"); if (J.V) need(J.V, (size_t)J.q * 16, "column scale"); }
            if (J.kind == JOB_LOWRANK && J.k2 > 0) {
                need(J.U, ((size_t)(J.k2 - 1) * J.ldu + J.m) * 16, "low-rank U");
                need(J.V, ((size_t)(J.k2 - 1) * J.ldv + J.q) * 16, "low-rank V");
            }
            continue;
        }
        recompress_ranges(J.m, J.q, J.k1, J.k2, rmax, J.au, J.av, J.U, J.ldu, J.V, J.ldv, J.work, J.ou, J.ov);
    }
}
void launch_hmatvec(const MatvecOp* ops, int count, int trans, int, const c128* X, int ldx, c128* Y, int ldy,
                    int ncol, c128, c128* tscratch, hipStream_t) {
    need(tscratch, hmatvec_scratch(ops, count, ncol) * 16, "hmatvec T");
    for (int t = 0; t < count; ++t) {
        const MatvecOp& o = ops[t];
        const int out = trans ? o.q : o.m, in = trans ? o.m : o.q;
        if (o.kind == 2) {
            if (ncol > 0) need(Y + o.yo, ((size_t)(ncol - 1) * ldy + o.m) * 16, "hmatvec cleared rows");
            continue;
        }
        if (o.kind == 0) need(o.a, (size_t)o.m * o.q * 16, "hmatvec D");
        else { need(o.a, (size_t)o.m * o.r * 16, "hmatvec U"); need(o.b, (size_t)o.q * o.r * 16, "hmatvec V"); }
        if (ncol > 0) {
            need(X + o.xo, ((size_t)(ncol - 1) * ldx + in) * 16, "hmatvec X");
            need(Y + o.yo, ((size_t)(ncol - 1) * ldy + out) * 16, "hmatvec Y");
        }
    }
}
void launch_rsvd_tails(const RsvdTail* jobs, int count, int rmax, double, hipStream_t) {
    for (int t = 0; t < count; ++t) {
        const RsvdTail& J = jobs[t];
        const int r = J.ell < rmax ? J.ell : rmax;
        need(J.Q, (size_t)J.m * J.ell * 16, "tail Q"); need(J.M, (size_t)J.q * J.ell * 16, "tail M");
        need(J.V, (size_t)J.ell * J.ell * 16, "tail V"); need(J.sig, (size_t)J.ell * 8, "tail sig");
        need(J.perm, (size_t)J.ell * 4, "tail perm"); need(J.rank, 4, "tail rank");
        need(J.Vg, (size_t)J.ell * r * 16, "tail Vg"); need(J.Uo, (size_t)J.m * r * 16, "tail Uo");
        need(J.Vo, (size_t)J.q * r * 16, "tail Vo");
        need(J.work, rsvd_tail_work(J.q, J.ell) * 16, "tail work");
    }
}
