// CPU stand-ins of the small dense launchers (k_dense.hip) for the
// sequential kernel emulation, which runs each kernel once per thread index
// and cannot run the wavefront kernels' cross-lane exchanges and barriers
// (those are checked on their own by tests/wavecheck).  Same contracts,
// plain loops: Householder QR, cyclic one-sided Jacobi SVD, Gauss-Jordan.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <vector>
#include "internal.hpp"

void launch_small_qr(int p, int k, const c128* A, int lda, c128* W, c128* Vh, c128* Q, c128* R, c128* Qc,
                     hipStream_t) {
    const int kk = p < k ? p : k;
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < p; ++i) W[(size_t)j * p + i] = A[(size_t)j * lda + i];
    for (size_t e = 0; e < (size_t)p * kk; ++e) Vh[e] = czero<double>();
    for (int c = 0; c < kk; ++c) {
        c128* v = Vh + (size_t)c * p;
        double nx2 = 0.0;
        for (int i = c; i < p; ++i) nx2 += abs2(W[(size_t)c * p + i]);
        const double nx = sqrt(nx2);
        if (nx == 0.0) continue;
        const c128 x0 = W[(size_t)c * p + c];
        const double a0 = hypot(x0.re, x0.im);
        const c128 ph = a0 > 0.0 ? mk(x0.re / a0, x0.im / a0) : mk(1.0, 0.0);
        for (int i = c; i < p; ++i) v[i] = W[(size_t)c * p + i];
        v[c] = x0 + nx * ph;
        double vv = 0.0;
        for (int i = c; i < p; ++i) vv += abs2(v[i]);
        for (int j = c; j < k; ++j) {
            c128 d = czero<double>();
            for (int i = c; i < p; ++i) cfma_conj(d, v[i], W[(size_t)j * p + i]);
            const c128 f = (2.0 / vv) * d;
            for (int i = c; i < p; ++i) W[(size_t)j * p + i] -= f * v[i];
        }
    }
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < kk; ++i) R[(size_t)j * kk + i] = i <= j ? W[(size_t)j * p + i] : czero<double>();
    for (int j = 0; j < kk; ++j)
        for (int i = 0; i < p; ++i) Q[(size_t)j * p + i] = mk(i == j ? 1.0 : 0.0, 0.0);
    for (int c = kk - 1; c >= 0; --c) {
        const c128* v = Vh + (size_t)c * p;
        double vv = 0.0;
        for (int i = c; i < p; ++i) vv += abs2(v[i]);
        if (vv == 0.0) continue;
        for (int j = c; j < kk; ++j) {
            c128 d = czero<double>();
            for (int i = c; i < p; ++i) cfma_conj(d, v[i], Q[(size_t)j * p + i]);
            const c128 f = (2.0 / vv) * d;
            for (int i = c; i < p; ++i) Q[(size_t)j * p + i] -= f * v[i];
        }
    }
    if (Qc)
        for (size_t e = 0; e < (size_t)p * kk; ++e) Qc[e] = conj(Q[e]);
}

void launch_small_svd(int a, int b, c128* A, int lda, c128* V, double* sig, int* perm, int* rank, double tol,
                      int rmax, hipStream_t) {
    for (int j = 0; j < b; ++j)
        for (int i = 0; i < b; ++i) V[(size_t)j * b + i] = mk(i == j ? 1.0 : 0.0, 0.0);
    double fro = 0.0;
    for (int j = 0; j < b; ++j)
        for (int i = 0; i < a; ++i) fro += abs2(A[(size_t)j * lda + i]);
    const double noise = 1e-30 * fro;
    for (int sweep = 0; sweep < 80; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < b - 1; ++p)
            for (int q = p + 1; q < b; ++q) {
                c128* x = A + (size_t)p * lda;
                c128* y = A + (size_t)q * lda;
                double al = 0.0, be = 0.0;
                c128 ga = czero<double>();
                for (int i = 0; i < a; ++i) {
                    al += abs2(x[i]);
                    be += abs2(y[i]);
                    cfma_conj(ga, x[i], y[i]);
                }
                const double g = hypot(ga.re, ga.im);
                if (!(g > 1e-15 * sqrt(al) * sqrt(be))) continue;
                if (be < 1e-30 * al || al < 1e-30 * be || (al <= noise && be <= noise)) continue;
                rotated = true;
                const c128 e = mk(ga.re / g, -ga.im / g);
                const double zeta = (be - al) / (2.0 * g);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < a; ++i) {
                    const c128 xi = x[i], wi = e * y[i];
                    x[i] = cs * xi - sn * wi;
                    y[i] = sn * xi + cs * wi;
                }
                c128* vx = V + (size_t)p * b;
                c128* vy = V + (size_t)q * b;
                for (int i = 0; i < b; ++i) {
                    const c128 xi = vx[i], wi = e * vy[i];
                    vx[i] = cs * xi - sn * wi;
                    vy[i] = sn * xi + cs * wi;
                }
            }
        if (!rotated) break;
    }
    for (int j = 0; j < b; ++j) {
        double s = 0.0;
        for (int i = 0; i < a; ++i) s += abs2(A[(size_t)j * lda + i]);
        sig[j] = sqrt(s);
    }
    for (int j = 0; j < b; ++j) {
        const double sj = isnan(sig[j]) ? -1.0 : sig[j];
        int pos = 0;
        for (int i = 0; i < b; ++i) {
            const double si = isnan(sig[i]) ? -1.0 : sig[i];
            pos += (si > sj || (si == sj && i < j)) ? 1 : 0;
        }
        perm[pos] = j;
    }
    int r = 0;
    if (b > 0 && sig[perm[0]] > 0.0) {
        const double cut = tol > 0.0 ? tol * sig[perm[0]] : 0.0;
        for (int j = 0; j < b; ++j) r += sig[perm[j]] > cut ? 1 : 0;
        if (r > rmax) r = rmax;
    }
    *rank = r;
}

void launch_small_inv(int m, const c128* A, int lda, c128* W, c128* X, int* status, hipStream_t) {
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            W[(size_t)j * m + i] = A[(size_t)j * lda + i];
            X[(size_t)j * m + i] = mk(i == j ? 1.0 : 0.0, 0.0);
        }
    for (int c = 0; c < m; ++c) {
        int p = c;
        double best = abs2(W[(size_t)c * m + c]);
        for (int r = c + 1; r < m; ++r)
            if (abs2(W[(size_t)c * m + r]) > best) { best = abs2(W[(size_t)c * m + r]); p = r; }
        if (!(best > 0.0)) { *status = 1; return; }
        for (int j = 0; j < m && p != c; ++j) {
            c128 t = W[(size_t)j * m + c]; W[(size_t)j * m + c] = W[(size_t)j * m + p]; W[(size_t)j * m + p] = t;
            t = X[(size_t)j * m + c]; X[(size_t)j * m + c] = X[(size_t)j * m + p]; X[(size_t)j * m + p] = t;
        }
        const c128 piv = cinv(W[(size_t)c * m + c]);
        for (int j = 0; j < m; ++j) {
            W[(size_t)j * m + c] = piv * W[(size_t)j * m + c];
            X[(size_t)j * m + c] = piv * X[(size_t)j * m + c];
        }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const c128 f = W[(size_t)c * m + r];
            for (int j = 0; j < m; ++j) {
                W[(size_t)j * m + r] -= f * W[(size_t)j * m + c];
                X[(size_t)j * m + r] -= f * X[(size_t)j * m + c];
            }
        }
    }
}

static void recompress_one(int m, int q, int k1, int k2, int rmax, double tol, c128 alpha, const c128* au,
                           const c128* av, const c128* U, int ldu, const c128* V, int ldv, c128* work, c128* ou,
                           c128* ov, hipStream_t s) {
    const int k = k1 + k2, kk1 = m < k ? m : k, kk2 = q < k ? q : k;
    const int r0 = kk1 < kk2 ? kk1 : kk2, r = r0 < rmax ? r0 : rmax;
    const RecompressLayout L = recompress_layout(m, q, k, rmax);
    c128 *W1 = work + L.W1, *W2 = work + L.W2, *C = work + L.C, *Vs = work + L.Vs, *Cg = work + L.Cg,
         *Vg = work + L.Vg, *Q1 = work + L.Q1, *Q2 = work + L.Q2, *R1 = work + L.R1, *R2 = work + L.R2;
    // the stacked factors go to the output-side pieces Q (m x kk1 is not
    // always m x k), so build them in W and let the QR copy them onto itself
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < m; ++i)
            W1[(size_t)j * m + i] = j < k1 ? au[(size_t)j * m + i] : alpha * U[(size_t)(j - k1) * ldu + i];
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < q; ++i) W2[(size_t)j * q + i] = j < k1 ? av[(size_t)j * q + i] : V[(size_t)(j - k1) * ldv + i];
    launch_small_qr(m, k, W1, m, W1, work + L.Vh1, Q1, R1, nullptr, s);
    launch_small_qr(q, k, W2, q, W2, work + L.Vh2, Q2, R2, nullptr, s);
    for (int j = 0; j < kk2; ++j)
        for (int i = 0; i < kk1; ++i) {
            c128 acc = czero<double>();
            for (int l = 0; l < k; ++l) cfma(acc, R1[(size_t)l * kk1 + i], R2[(size_t)l * kk2 + j]);
            C[(size_t)j * kk1 + i] = acc;
        }
    double* sig = (double*)(work + L.sig);
    int* perm = (int*)(work + L.perm);
    int* rank = (int*)(work + L.rank);
    launch_small_svd(kk1, kk2, C, kk1, Vs, sig, perm, rank, tol, rmax, s);
    for (int j = 0; j < r; ++j) {
        for (int i = 0; i < kk1; ++i) Cg[(size_t)j * kk1 + i] = j < *rank ? C[(size_t)perm[j] * kk1 + i] : czero<double>();
        for (int i = 0; i < kk2; ++i) Vg[(size_t)j * kk2 + i] = j < *rank ? conj(Vs[(size_t)perm[j] * kk2 + i]) : czero<double>();
    }
    for (int j = 0; j < r; ++j) {
        for (int i = 0; i < m; ++i) {
            c128 acc = czero<double>();
            for (int l = 0; l < kk1; ++l) cfma(acc, Q1[(size_t)l * m + i], Cg[(size_t)j * kk1 + l]);
            ou[(size_t)j * m + i] = acc;
        }
        for (int i = 0; i < q; ++i) {
            c128 acc = czero<double>();
            for (int l = 0; l < kk2; ++l) cfma(acc, Q2[(size_t)l * q + i], Vg[(size_t)j * kk2 + l]);
            ov[(size_t)j * q + i] = acc;
        }
    }
}

static void dense_one(const BlockJob& J) {
    for (int j = 0; j < J.q; ++j)
        for (int i = 0; i < J.m; ++i) {
            const size_t e = (size_t)j * J.m + i;
            if (J.kind == JOB_SUM) {
                J.ou[e] = J.au[e] + J.alpha * J.av[e];
            } else if (J.kind == JOB_LOWRANK) {
                c128 acc = czero<double>();
                for (int l = 0; l < J.k2; ++l) cfma(acc, J.U[(size_t)l * J.ldu + i], J.V[(size_t)l * J.ldv + j]);
                J.ou[e] += J.alpha * acc;
            } else if (J.kind == JOB_SCALE) {
                c128 v = J.U[i] * J.au[e];
                if (J.V) v = v * J.V[j];
                J.ou[e] = v;
            } else {
                J.ou[e] = J.au[e];
            }
        }
}

// The byte ranges a job reads and writes (its work buffer counts as written).
struct Span {
    const char* p;
    size_t n;
};
static Span span(const void* p, size_t entries) { return Span{(const char*)p, entries * sizeof(c128)}; }
static Span cols(const c128* p, int ld, int rows, int ncol) {
    return ncol > 0 && p ? span(p, (size_t)(ncol - 1) * ld + rows) : Span{nullptr, 0};
}
static void job_spans(const BlockJob& J, int rmax, std::vector<Span>& rd, std::vector<Span>& wr) {
    const size_t mq = (size_t)J.m * J.q;
    if (J.kind == JOB_RECOMPRESS) {
        const int k = J.k1 + J.k2, kk1 = J.m < k ? J.m : k, kk2 = J.q < k ? J.q : k;
        const int r0 = kk1 < kk2 ? kk1 : kk2, r = r0 < rmax ? r0 : rmax;
        rd = {cols(J.au, J.m, J.m, J.k1), cols(J.av, J.q, J.q, J.k1), cols(J.U, J.ldu, J.m, J.k2),
              cols(J.V, J.ldv, J.q, J.k2)};
        wr = {span(J.work, recompress_layout(J.m, J.q, k, rmax).total), span(J.ou, (size_t)J.m * r),
              span(J.ov, (size_t)J.q * r)};
    } else if (J.kind == JOB_SUM) {
        rd = {span(J.au, mq), span(J.av, mq)};
        wr = {span(J.ou, mq)};
    } else if (J.kind == JOB_LOWRANK) {
        rd = {cols(J.U, J.ldu, J.m, J.k2), cols(J.V, J.ldv, J.q, J.k2), span(J.ou, mq)};
        wr = {span(J.ou, mq)};
    } else if (J.kind == JOB_SCALE) {
        rd = {span(J.au, mq), span(J.U, J.m), J.V ? span(J.V, J.q) : Span{nullptr, 0}};
        wr = {span(J.ou, mq)};
    } else {
        rd = {span(J.au, mq)};
        wr = {span(J.ou, mq)};
    }
}
static bool meet(const Span& a, const Span& b) {
    return a.p && b.p && a.n && b.n && a.p < b.p + b.n && b.p < a.p + a.n;
}

void launch_block_jobs(const BlockJob* jobs, int count, int rmax, double tol, hipStream_t s) {
    // the jobs of a batch run side by side on the device: none may write what
    // another reads or writes
    for (int a = 0; a < count; ++a) {
        std::vector<Span> ra, wa, rb, wb;
        job_spans(jobs[a], rmax, ra, wa);
        for (int b = 0; b < count; ++b) {
            if (a == b) continue;
            job_spans(jobs[b], rmax, rb, wb);
            for (const Span& w : wa) {
                for (const Span& x : rb)
                    if (meet(w, x)) { fprintf(stderr, "BATCH DEPENDENCE: job %d writes what job %d reads\n", a, b); abort(); }
                for (const Span& x : wb)
                    if (meet(w, x)) { fprintf(stderr, "BATCH DEPENDENCE: jobs %d and %d write the same bytes\n", a, b); abort(); }
            }
        }
    }
    for (int j = 0; j < count; ++j) {
        const BlockJob& J = jobs[j];
        if (J.kind != JOB_RECOMPRESS) {
            dense_one(J);
            continue;
        }
        recompress_one(J.m, J.q, J.k1, J.k2, rmax, tol, J.alpha, J.au, J.av, J.U, J.ldu, J.V, J.ldv, J.work, J.ou,
                       J.ov, s);
    }
}

void launch_hmatvec(const MatvecOp* ops, int count, int trans, int assign, const c128* X, int ldx, c128* Y, int ldy,
                    int ncol, c128 alpha, c128*, hipStream_t) {
    for (int t = 0; t < count; ++t) {
        const MatvecOp& o = ops[t];
        const int out = trans ? o.q : o.m, in = trans ? o.m : o.q;
        const int cleared = o.kind == 2 ? o.m : out;
        if (o.kind == 2 || assign)
            for (int j = 0; j < ncol; ++j)
                for (int i = 0; i < cleared; ++i) Y[(size_t)j * ldy + o.yo + i] = czero<double>();
        if (o.kind == 2) continue;
        for (int j = 0; j < ncol; ++j) {
            const c128* x = X + (size_t)j * ldx + o.xo;
            c128* y = Y + (size_t)j * ldy + o.yo;
            if (o.kind == 0) {
                for (int i = 0; i < out; ++i) {
                    c128 acc = czero<double>();
                    for (int l = 0; l < in; ++l)
                        cfma(acc, trans ? o.a[(size_t)i * o.m + l] : o.a[(size_t)l * o.m + i], x[l]);
                    y[i] += alpha * acc;
                }
            } else {
                const c128* P = trans ? o.a : o.b;
                const c128* Q = trans ? o.b : o.a;
                for (int i = 0; i < out; ++i) {
                    c128 acc = czero<double>();
                    for (int k = 0; k < o.r; ++k) {
                        c128 tk = czero<double>();
                        for (int l = 0; l < in; ++l) cfma(tk, P[(size_t)k * in + l], x[l]);
                        cfma(acc, Q[(size_t)k * out + i], tk);
                    }
                    y[i] += alpha * acc;
                }
            }
        }
    }
}

void launch_rsvd_tails(const RsvdTail* jobs, int count, int rmax, double tol, hipStream_t s) {
    for (int t = 0; t < count; ++t) {
        const RsvdTail& J = jobs[t];
        launch_small_svd(J.q, J.ell, J.M, J.q, J.V, J.sig, J.perm, J.rank, tol, rmax, s);
        const int r = J.ell < rmax ? J.ell : rmax, kept = *J.rank;
        for (int j = 0; j < r; ++j) {
            for (int i = 0; i < J.ell; ++i)
                J.Vg[(size_t)j * J.ell + i] = j < kept ? conj(J.V[(size_t)J.perm[j] * J.ell + i]) : czero<double>();
            for (int i = 0; i < J.q; ++i)
                J.Vo[(size_t)j * J.q + i] = j < kept ? J.M[(size_t)J.perm[j] * J.q + i] : czero<double>();
            for (int i = 0; i < J.m; ++i) {
                c128 acc = czero<double>();
                for (int l = 0; l < J.ell; ++l) cfma(acc, J.Q[(size_t)l * J.m + i], J.Vg[(size_t)j * J.ell + l]);
                J.Uo[(size_t)j * J.m + i] = acc;
            }
        }
    }
}
