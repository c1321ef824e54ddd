// Driver of the threaded check of the small dense launchers (k_dense.hip):
// reads one problem, runs the launcher, writes the results.
//
// Input: int32 op (0 QR, 1 SVD, 2 inverse), rows, cols, lda, rmax; float64
// tol; then the lda x cols complex128 matrix (column-major).
// Output: QR: Q (rows x kk), R (kk x cols); SVD: A after the call (lda x
// cols), V (cols x cols), sigma (cols float64), perm (cols int32), rank
// (int32); inverse: X (rows x rows), status (int32).
#include <stdint.h>
#include <stdio.h>
#include <vector>
#include <hip/hip_runtime.h>
#include "internal.hpp"

thread_local emu_index blockIdx, threadIdx;
thread_local dim3 blockDim, gridDim;
pthread_barrier_t wave_barrier;
unsigned long long wave_slot[1024];
std::vector<char> wave_dyn_shared;

static bool rd(FILE* fp, void* p, size_t b) { return fread(p, 1, b, fp) == b; }
template <typename T> static T* dev(size_t count) {
    void* p = nullptr;
    hipMalloc(&p, (count ? count : 1) * sizeof(T));
    return (T*)p;
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    fake_poison = true;
    FILE* fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int32_t hd[5];
    double tol;
    if (!rd(fp, hd, sizeof hd) || !rd(fp, &tol, 8)) return 2;
    const int op = hd[0], p = hd[1], k = hd[2], lda = hd[3], rmax = hd[4];
    if (op == 3) {
        // a batch of recompressions: p = number of jobs, k = rmax, lda unused;
        // per job int32 m, q, k1, k2, float64 alpha (re, im), then au (m x k1),
        // av (q x k1), U (m x k2), V (q x k2); output each job's ou, ov
        const int count = p;
        std::vector<BlockJob> jobs(count);
        std::vector<int> rw(count);
        for (int t = 0; t < count; ++t) {
            int32_t kind;
            int32_t d[4];
            double al[2];
            if (!rd(fp, &kind, 4) || !rd(fp, d, 16) || !rd(fp, al, 16)) return 2;
            const int m = d[0], q = d[1], k1 = d[2], k2 = d[3];
            if (kind != JOB_RECOMPRESS) {
                // dense kinds: a (m x q), b (m x q; SUM), U (m x k2), V (q x k2) (LOWRANK),
                // row and column scales (m, q; SCALE), the output's initial m x q
                const size_t nq = (size_t)m * q;
                const size_t na = nq, nb = kind == JOB_SUM ? nq : 0;
                const size_t nu = kind == JOB_LOWRANK ? (size_t)m * k2 : kind == JOB_SCALE ? m : 0;
                const size_t nv = kind == JOB_LOWRANK ? (size_t)q * k2 : kind == JOB_SCALE ? q : 0;
                std::vector<c128> h(na + nb + nu + nv + nq);
                if (!rd(fp, h.data(), h.size() * 16)) return 2;
                c128 *A = dev<c128>(na), *Bm = dev<c128>(nb), *Uu = dev<c128>(nu), *Vv = dev<c128>(nv), *O = dev<c128>(nq);
                hipMemcpy(A, h.data(), na * 16, hipMemcpyHostToDevice);
                hipMemcpy(Bm, h.data() + na, nb * 16, hipMemcpyHostToDevice);
                hipMemcpy(Uu, h.data() + na + nb, nu * 16, hipMemcpyHostToDevice);
                hipMemcpy(Vv, h.data() + na + nb + nu, nv * 16, hipMemcpyHostToDevice);
                hipMemcpy(O, h.data() + na + nb + nu + nv, nq * 16, hipMemcpyHostToDevice);
                BlockJob& J = jobs[t];
            J.kind = JOB_RECOMPRESS;
                J.kind = kind;
                J.au = A; J.av = Bm; J.U = nu ? Uu : nullptr; J.V = nv ? Vv : nullptr;
                J.work = nullptr; J.ou = O; J.ov = nullptr;
                J.alpha = mk(al[0], al[1]);
                J.m = m; J.q = q; J.k1 = 0; J.k2 = k2; J.ldu = m; J.ldv = q;
                rw[t] = -1;
                continue;
            }
            const size_t n1 = (size_t)m * k1, n2 = (size_t)q * k1, n3 = (size_t)m * k2, n4 = (size_t)q * k2;
            std::vector<c128> h(n1 + n2 + n3 + n4);
            if (!rd(fp, h.data(), h.size() * 16)) return 2;
            c128 *au = dev<c128>(n1), *av = dev<c128>(n2), *U = dev<c128>(n3), *V = dev<c128>(n4);
            hipMemcpy(au, h.data(), n1 * 16, hipMemcpyHostToDevice);
            hipMemcpy(av, h.data() + n1, n2 * 16, hipMemcpyHostToDevice);
            hipMemcpy(U, h.data() + n1 + n2, n3 * 16, hipMemcpyHostToDevice);
            hipMemcpy(V, h.data() + n1 + n2 + n3, n4 * 16, hipMemcpyHostToDevice);
            const int kt = k1 + k2, kk1 = m < kt ? m : kt, kk2 = q < kt ? q : kt;
            const int r0 = kk1 < kk2 ? kk1 : kk2, r = r0 < rmax ? r0 : rmax;
            BlockJob& J = jobs[t];
            J.kind = JOB_RECOMPRESS;
            J.au = au; J.av = av; J.U = U; J.V = V;
            J.work = dev<c128>(recompress_layout(m, q, kt, rmax).total);
            J.ou = dev<c128>((size_t)m * r);
            J.ov = dev<c128>((size_t)q * r);
            J.alpha = mk(al[0], al[1]);
            J.m = m; J.q = q; J.k1 = k1; J.k2 = k2; J.ldu = m; J.ldv = q;
            rw[t] = r;
        }
        fclose(fp);
        launch_block_jobs(jobs.data(), count, rmax, tol, nullptr);
        FILE* out = fopen(argv[2], "wb");
        for (int t = 0; t < count; ++t) {
            if (rw[t] < 0) {
                fwrite(jobs[t].ou, 16, (size_t)jobs[t].m * jobs[t].q, out);
                continue;
            }
            fwrite(jobs[t].ou, 16, (size_t)jobs[t].m * rw[t], out);
            fwrite(jobs[t].ov, 16, (size_t)jobs[t].q * rw[t], out);
        }
        fclose(out);
        return 0;
    }
    if (op == 4) {
        // leaf-block products: p = ops, k = trans, lda = ncol; then int32
        // rows of X and Y, float64 alpha (re, im), X, Y; per op int32 kind,
        // m, q, r, yo, xo and its data (D: m x q; F: m x r, then q x r)
        const int count = p, trans = k & 1, assign = k >> 1, ncol = lda;
        int32_t rw[2];
        double al[2];
        if (!rd(fp, rw, 8) || !rd(fp, al, 16)) return 2;
        const size_t nx = (size_t)rw[0] * ncol, ny = (size_t)rw[1] * ncol;
        std::vector<c128> hx(nx), hy(ny);
        if (!rd(fp, hx.data(), nx * 16) || !rd(fp, hy.data(), ny * 16)) return 2;
        c128 *X = dev<c128>(nx), *Y = dev<c128>(ny);
        hipMemcpy(X, hx.data(), nx * 16, hipMemcpyHostToDevice);
        hipMemcpy(Y, hy.data(), ny * 16, hipMemcpyHostToDevice);
        std::vector<MatvecOp> ops(count);
        for (int t = 0; t < count; ++t) {
            int32_t d[6];
            if (!rd(fp, d, 24)) return 2;
            MatvecOp& o = ops[t];
            o.kind = d[0]; o.m = d[1]; o.q = d[2]; o.r = d[3]; o.yo = d[4]; o.xo = d[5];
            const size_t na = o.kind == 0 ? (size_t)o.m * o.q : o.kind == 1 ? (size_t)o.m * o.r : 0;
            const size_t nb = o.kind == 1 ? (size_t)o.q * o.r : 0;
            std::vector<c128> h(na + nb);
            if (!rd(fp, h.data(), h.size() * 16)) return 2;
            c128* A = dev<c128>(na);
            hipMemcpy(A, h.data(), na * 16, hipMemcpyHostToDevice);
            o.a = A;
            o.b = nullptr;
            if (nb) {
                c128* Bv = dev<c128>(nb);
                hipMemcpy(Bv, h.data() + na, nb * 16, hipMemcpyHostToDevice);
                o.b = Bv;
            }
        }
        fclose(fp);
        const size_t need = hmatvec_scratch(ops.data(), count, ncol);
        c128* T = need ? dev<c128>(need) : nullptr;
        launch_hmatvec(ops.data(), count, trans, assign, X, rw[0], Y, rw[1], ncol, mk(al[0], al[1]), T, nullptr);
        FILE* out = fopen(argv[2], "wb");
        fwrite(Y, 16, ny, out);
        fclose(out);
        return 0;
    }
    if (op == 5) {
        // randomized-SVD tails: p = jobs, rmax; per job int32 m, q, ell, then
        // Q (m x ell), M (q x ell); output each job's Uo (m x r), Vo (q x r)
        const int count = p;
        std::vector<RsvdTail> jobs(count);
        for (int t = 0; t < count; ++t) {
            int32_t d[3];
            if (!rd(fp, d, 12)) return 2;
            RsvdTail& J = jobs[t];
            J.m = d[0]; J.q = d[1]; J.ell = d[2];
            const int r = J.ell < rmax ? J.ell : rmax;
            std::vector<c128> h((size_t)J.m * J.ell + (size_t)J.q * J.ell);
            if (!rd(fp, h.data(), h.size() * 16)) return 2;
            c128* Qd = dev<c128>((size_t)J.m * J.ell);
            J.M = dev<c128>((size_t)J.q * J.ell);
            hipMemcpy(Qd, h.data(), (size_t)J.m * J.ell * 16, hipMemcpyHostToDevice);
            hipMemcpy(J.M, h.data() + (size_t)J.m * J.ell, (size_t)J.q * J.ell * 16, hipMemcpyHostToDevice);
            J.Q = Qd;
            J.V = dev<c128>((size_t)J.ell * J.ell);
            J.work = dev<c128>(rsvd_tail_work(J.q, J.ell));
            J.sig = dev<double>(J.ell);
            J.perm = dev<int>(J.ell);
            J.rank = dev<int>(1);
            J.Vg = dev<c128>((size_t)J.ell * r);
            J.Uo = dev<c128>((size_t)J.m * r);
            J.Vo = dev<c128>((size_t)J.q * r);
        }
        fclose(fp);
        launch_rsvd_tails(jobs.data(), count, rmax, tol, nullptr);
        FILE* out = fopen(argv[2], "wb");
        for (const RsvdTail& J : jobs) {
            const int r = J.ell < rmax ? J.ell : rmax;
            fwrite(J.Uo, 16, (size_t)J.m * r, out);
            fwrite(J.Vo, 16, (size_t)J.q * r, out);
        }
        fclose(out);
        return 0;
    }
    std::vector<c128> a((size_t)lda * k);
    if (!rd(fp, a.data(), a.size() * 16)) return 2;
    fclose(fp);
    c128* A = dev<c128>(a.size());
    hipMemcpy(A, a.data(), a.size() * 16, hipMemcpyHostToDevice);
    FILE* out = fopen(argv[2], "wb");
    if (op == 0) {
        const int kk = p < k ? p : k;
        c128 *W = dev<c128>((size_t)p * k), *Vh = dev<c128>((size_t)p * kk), *Q = dev<c128>((size_t)p * kk),
             *R = dev<c128>((size_t)kk * k), *Qc = dev<c128>((size_t)p * kk);
        launch_small_qr(p, k, A, lda, W, Vh, Q, R, Qc, nullptr);
        fwrite(Q, 16, (size_t)p * kk, out);
        fwrite(R, 16, (size_t)kk * k, out);
        fwrite(Qc, 16, (size_t)p * kk, out);
    } else if (op == 1) {
        c128* V = dev<c128>((size_t)k * k);
        double* sig = dev<double>(k);
        int* perm = dev<int>(k);
        int* rank = dev<int>(1);
        launch_small_svd(p, k, A, lda, V, sig, perm, rank, tol, rmax, nullptr);
        fwrite(A, 16, a.size(), out);
        fwrite(V, 16, (size_t)k * k, out);
        fwrite(sig, 8, k, out);
        fwrite(perm, 4, k, out);
        fwrite(rank, 4, 1, out);
    } else {
        c128 *W = dev<c128>((size_t)p * (p + 1)), *X = dev<c128>((size_t)p * p);
        int* st = dev<int>(1);
        *st = 0;
        launch_small_inv(p, A, lda, W, X, st, nullptr);
        fwrite(X, 16, (size_t)p * p, out);
        fwrite(st, 4, 1, out);
    }
    fclose(out);
    return 0;
}
