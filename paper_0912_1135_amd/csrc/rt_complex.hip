// Complex-valued A (the paper's remark that the method and its analysis
// extend to complex entries, Sec. 1 end).  A complex m x n matrix A = Ar +
// i Ai is carried as the real 2m x 2n matrix
//     Ah = [ Ar  -Ai ]
//          [ Ai   Ar ],
// whose action on [Re b; Im b] is [Re A b; Im A b] and whose transpose acts
// as A^* (the conjugate transpose).  The embedding is an isometry, so the
// orthogonal projections onto the row and null spaces of Ah are those of A,
// the least-squares solution of Ah^T xh ~ bh is [Re x; Im x], Ah has full row
// rank 2m exactly when A has rank m, and cond(Ah) = cond(A).  A complex plan
// therefore runs a real plan of sizes (2m, 2n, 2l) on Ah, which it forms (and
// owns) from A at each precondition; right-hand sides and outputs are
// converted on the device.  Complex data are interleaved (re, im) binary64
// pairs (std::complex<double>, torch.complex128).
#include "rt_plan_state.h"

struct rtproj_cplan_s {
    int64_t m = 0, n = 0, l = 0;
    rtproj_plan real = nullptr;
    double *d_Ah = nullptr;          // 2m x 2n row-major
    double *d_B = nullptr;           // 2n x kcap column-major (right-hand sides, embedded)
    double *d_Z = nullptr, *d_Y = nullptr;  // 2n x kcap
    double *d_X = nullptr;           // 2m x kcap
    int64_t kcap = 0;
};

namespace {

using namespace rtp;

// Ah from A: element (i, j) of A (re, im) lands at (i, j) and (m+i, n+j) as
// re, (i, n+j) as -im, (m+i, j) as im.
__global__ void embed_matrix_kernel(const double *__restrict__ A, int64_t lda, int m, int n, double *__restrict__ Ah)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * n) return;
    const int i = (int)(e / n), j = (int)(e % n);
    const double2 a = *reinterpret_cast<const double2 *>(A + 2 * ((int64_t)i * lda + j));
    const int64_t w = 2 * (int64_t)n;
    Ah[(int64_t)i * w + j] = a.x;
    Ah[(int64_t)i * w + n + j] = -a.y;
    Ah[(int64_t)(m + i) * w + j] = a.y;
    Ah[(int64_t)(m + i) * w + n + j] = a.x;
}

// column c of a complex rows x k block (ld in complex elements) to
// [re; im] in a real 2 rows x k block (ld 2 rows), or back (dir = 1)
__global__ void embed_cols_kernel(const double *__restrict__ src, int64_t lds, double *__restrict__ dst, int64_t ldd,
                                  int rows, int k, int dir)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * k) return;
    const int c = (int)(e / rows), t = (int)(e % rows);
    if (dir == 0) {
        const double2 v = *reinterpret_cast<const double2 *>(src + 2 * ((int64_t)c * lds + t));
        dst[(int64_t)c * ldd + t] = v.x;
        dst[(int64_t)c * ldd + rows + t] = v.y;
    } else {
        double2 v;
        v.x = src[(int64_t)c * lds + t];
        v.y = src[(int64_t)c * lds + rows + t];
        *reinterpret_cast<double2 *>(dst + 2 * ((int64_t)c * ldd + t)) = v;
    }
}

hipError_t embed_cols(const double *src, int64_t lds, double *dst, int64_t ldd, int rows, int k, int dir,
                      hipStream_t s)
{
    const int64_t total = (int64_t)rows * k;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(embed_cols_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, lds, dst, ldd,
                       rows, k, dir);
    return hipGetLastError();
}

rtproj_status cplan_grow(rtproj_cplan c, int64_t k)
{
    if (k <= c->kcap) return RTPROJ_OK;
    for (double **b : {&c->d_B, &c->d_Z, &c->d_Y, &c->d_X})
        if (*b) { (void)hipFree(*b); *b = nullptr; }
    c->kcap = 0;
    RT_HIP(dalloc(&c->d_B, (size_t)2 * c->n * k));
    RT_HIP(dalloc(&c->d_Z, (size_t)2 * c->n * k));
    RT_HIP(dalloc(&c->d_Y, (size_t)2 * c->n * k));
    RT_HIP(dalloc(&c->d_X, (size_t)2 * c->m * k));
    c->kcap = k;
    return RTPROJ_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

extern "C" {

rtproj_status rtproj_cplan_create(int64_t m, int64_t n, int64_t l, uint64_t seed, rtproj_cplan *out)
{
    if (!out) return fail(RTPROJ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (m < 1 || n < m || l < m || l > n) return fail(RTPROJ_ERR_INVALID_ARG, "sizes must satisfy 1 <= m <= l <= n");
    if (n > (int64_t(1) << 29) || m > 16384) return fail(RTPROJ_ERR_UNSUPPORTED, "n above 2^29 or m above 16384");
    rtproj_cplan c = new (std::nothrow) rtproj_cplan_s();
    if (!c) return fail(RTPROJ_ERR_ALLOC, "host allocation failed");
    c->m = m; c->n = n; c->l = l;
    rtproj_status st = rtproj_plan_create(2 * m, 2 * n, 2 * l, seed, &c->real);
    if (st == RTPROJ_OK && hipMalloc((void **)&c->d_Ah, (size_t)4 * m * n * sizeof(double)) != hipSuccess) {
        c->d_Ah = nullptr;
        st = fail(RTPROJ_ERR_ALLOC, "device allocation of the embedded matrix failed");
    }
    if (st != RTPROJ_OK) {
        rtproj_cplan_destroy(c);
        return st;
    }
    *out = c;
    return RTPROJ_OK;
}

rtproj_status rtproj_cplan_destroy(rtproj_cplan c)
{
    if (!c) return RTPROJ_OK;
    if (c->real) rtproj_plan_destroy(c->real);  // waits for the stream
    for (double *b : {c->d_Ah, c->d_B, c->d_Z, c->d_Y, c->d_X})
        if (b) (void)hipFree(b);
    delete c;
    return RTPROJ_OK;
}

rtproj_plan rtproj_cplan_real(rtproj_cplan c) { return c ? c->real : nullptr; }

rtproj_status rtproj_cprecondition(rtproj_cplan c, const double *A, int64_t lda)
{
    if (!c) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (!A) return fail(RTPROJ_ERR_INVALID_ARG, "A is NULL");
    if (lda < c->n) return fail(RTPROJ_ERR_INVALID_ARG, "lda < n");
    if (!aligned16(A)) return fail(RTPROJ_ERR_INVALID_ARG, "A is not 16-byte aligned (complex binary64 elements)");
    const int64_t total = c->m * c->n;
    hipLaunchKernelGGL(embed_matrix_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->real->stream, A,
                       lda, (int)c->m, (int)c->n, c->d_Ah);
    RT_HIP(hipGetLastError());
    return rtproj_precondition(c->real, c->d_Ah, 2 * c->n);
}

rtproj_status rtproj_cproject_all(rtproj_cplan c, const double *B, int64_t ldb, int64_t k, double *Z, int64_t ldz,
                                  double *Y, int64_t ldy, double *X, int64_t ldx)
{
    if (!c) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (k < 0) return fail(RTPROJ_ERR_INVALID_ARG, "k < 0");
    if (k == 0) return RTPROJ_OK;
    if (!B) return fail(RTPROJ_ERR_INVALID_ARG, "B is NULL");
    if (ldb < c->n || (Z && ldz < c->n) || (Y && ldy < c->n) || (X && ldx < c->m))
        return fail(RTPROJ_ERR_INVALID_ARG, "leading dimension below n (B, Z, Y) or m (X)");
    for (const void *q : {(const void *)B, (const void *)Z, (const void *)Y, (const void *)X})
        if (q && !aligned16(q)) return fail(RTPROJ_ERR_INVALID_ARG, "a complex array is not 16-byte aligned");
    if (!c->real->ready) return fail(RTPROJ_ERR_STATE, "project called before a successful rtproj_cprecondition");
    rtproj_status st = cplan_grow(c, k);
    if (st != RTPROJ_OK) return st;
    hipStream_t s = c->real->stream;
    const int64_t n2 = 2 * c->n, m2 = 2 * c->m;
    RT_HIP(embed_cols(B, ldb, c->d_B, n2, (int)c->n, (int)k, 0, s));
    st = rtproj_project_all(c->real, c->d_B, n2, k, Z ? c->d_Z : nullptr, n2, Y ? c->d_Y : nullptr, n2,
                            X ? c->d_X : nullptr, m2);
    if (st != RTPROJ_OK) return st;
    if (Z) RT_HIP(embed_cols(c->d_Z, n2, Z, ldz, (int)c->n, (int)k, 1, s));
    if (Y) RT_HIP(embed_cols(c->d_Y, n2, Y, ldy, (int)c->n, (int)k, 1, s));
    if (X) RT_HIP(embed_cols(c->d_X, m2, X, ldx, (int)c->m, (int)k, 1, s));
    return RTPROJ_OK;
}

}  // extern "C"
