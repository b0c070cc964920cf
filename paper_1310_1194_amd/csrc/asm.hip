// Global assembly of element matrices and load vectors into a CSR matrix
// (Sec. 2: the global matrix is the sum of the element matrices placed
// through the element-to-global numbering; elements of one colour share no
// global entry, so a colour is assembled without atomics).
//
// Set-up, once per mesh, on the host (threads over rows / elements):
//   * node -> element incidence from the caller's dof map,
//   * the CSR pattern: row i holds every dof that shares an element with i,
//     columns ascending,
//   * the position map: for entry (a, b) of element e, the offset of column
//     dofs[e][b] inside row dofs[e][a] (uint16: a row of a degree-p prism mesh
//     holds at most (2p+1)^3 <= 3375 columns),
//   * a greedy colouring: each element takes the smallest colour not used by
//     an element sharing one of its dofs; elements are listed colour by colour.
// Per assembly, on the device: the values and rhs are cleared by a fill
// kernel (unless accumulating), then one launch per colour adds every entry
// of its elements: values[row_ptr[dofs[e][a]] + pos[e][a][b]] += A_e[a][b]
// and rhs[dofs[e][a]] += b_e[a], one wave per element.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "capi_internal.h"
#include "device_common.h"
#include "tables.h"

struct feint_asm_plan {
    int dev = 0;
    int64_t ne = 0, ndof = 0, nnz = 0;
    int n = 0, ncolors = 0;
    std::vector<int64_t> color_start;     // host: ncolors + 1 offsets into elems
    std::vector<int32_t> color_of;        // host: colour of every element
    // device buffers (one allocation)
    void *base = nullptr;
    int64_t *row_ptr = nullptr;   // [ndof + 1]
    int32_t *col_idx = nullptr;   // [nnz]
    int32_t *dofs = nullptr;      // [ne][n]
    int32_t *elems = nullptr;     // [ne], colour by colour
    uint16_t *pos = nullptr;      // [ne][n][n]
};

namespace feint {
namespace {

template <typename F>
void parallel_for(int64_t n, F fn) {
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt == 0 ? 4 : (nt > 64 ? 64 : nt);
    if (n < 4096) nt = 1;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            fn(lo, hi, t);
        });
    for (auto &x : th) x.join();
}

template <typename T>
__global__ void fill_zero(T *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (T)0;
}

// One wave per element of the colour (elements elems[first .. first + count)).
template <typename T>
__global__ __launch_bounds__(256) void scatter_color(const T *__restrict__ A, const T *__restrict__ b,
                                                     const int32_t *__restrict__ elems, int64_t first,
                                                     int64_t count, const int32_t *__restrict__ dofs,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const uint16_t *__restrict__ pos, int n, T *values,
                                                     T *rhs) {
    __shared__ int64_t rowbase[4][c_nshp(7)];
    const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    if (item >= count) return;
    const int64_t e = elems[first + item];
    const int32_t *de = dofs + e * n;
    for (int a = lane; a < n; a += 64) {
        const int32_t g = de[a];
        rowbase[wave][a] = row_ptr[g];
        rhs[g] += b[e * n + a];
    }
    wave_sync();
    const int64_t nn = (int64_t)n * n;
    const T *Ae = A + e * nn;
    const uint16_t *pe = pos + e * nn;
    for (int64_t idx = lane; idx < nn; idx += 64) {
        const int a = (int)(idx / n);
        T *v = values + rowbase[wave][a] + pe[idx];
        *v += Ae[idx];
    }
}

}  // namespace
}  // namespace feint

using namespace feint;

extern "C" {

feint_status feint_asm_plan_create(const int32_t *dofs, int64_t ne, int n, int64_t ndof, feint_asm_plan **out) {
    if (!out) return FEINT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!dofs || ne <= 0 || ndof <= 0 || ndof >= (1LL << 31)) return FEINT_ERR_INVALID_ARG;
    bool known = false;
    for (int p = 1; p <= kMaxP; ++p) known |= c_nshp(p) == n;
    if (!known) return FEINT_ERR_INVALID_ARG;
    for (int64_t i = 0; i < ne * n; ++i)
        if (dofs[i] < 0 || dofs[i] >= ndof) return FEINT_ERR_INVALID_ARG;

    // node -> element incidence
    std::vector<int64_t> inc_ptr(ndof + 1, 0);
    for (int64_t i = 0; i < ne * n; ++i) inc_ptr[dofs[i] + 1]++;
    for (int64_t i = 0; i < ndof; ++i) inc_ptr[i + 1] += inc_ptr[i];
    std::vector<int32_t> inc(inc_ptr[ndof]);
    {
        std::vector<int64_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int a = 0; a < n; ++a) inc[fill[dofs[e * n + a]]++] = (int32_t)e;
    }
    for (int64_t e = 0; e < ne; ++e) {      // a dof listed twice in one element is a bad map
        std::vector<int32_t> d(dofs + e * n, dofs + (e + 1) * n);
        std::sort(d.begin(), d.end());
        if (std::adjacent_find(d.begin(), d.end()) != d.end()) return FEINT_ERR_INVALID_ARG;
    }

    // CSR pattern: row lengths, then the sorted columns
    std::vector<int64_t> row_ptr(ndof + 1, 0);
    parallel_for(ndof, [&](int64_t lo, int64_t hi, unsigned) {
        std::vector<int32_t> seen;
        for (int64_t i = lo; i < hi; ++i) {
            seen.clear();
            for (int64_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
                const int32_t *de = dofs + (int64_t)inc[k] * n;
                seen.insert(seen.end(), de, de + n);
            }
            std::sort(seen.begin(), seen.end());
            row_ptr[i + 1] = std::unique(seen.begin(), seen.end()) - seen.begin();
        }
    });
    for (int64_t i = 0; i < ndof; ++i) {
        if (row_ptr[i + 1] > 65535) return FEINT_ERR_TOO_LARGE;
        row_ptr[i + 1] += row_ptr[i];
    }
    const int64_t nnz = row_ptr[ndof];
    std::vector<int32_t> col_idx(nnz);
    parallel_for(ndof, [&](int64_t lo, int64_t hi, unsigned) {
        std::vector<int32_t> seen;
        for (int64_t i = lo; i < hi; ++i) {
            seen.clear();
            for (int64_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
                const int32_t *de = dofs + (int64_t)inc[k] * n;
                seen.insert(seen.end(), de, de + n);
            }
            std::sort(seen.begin(), seen.end());
            const auto end = std::unique(seen.begin(), seen.end());
            std::copy(seen.begin(), end, col_idx.begin() + row_ptr[i]);
        }
    });

    // position map
    const int64_t nn = (int64_t)n * n;
    std::vector<uint16_t> pos(ne * nn);
    parallel_for(ne, [&](int64_t lo, int64_t hi, unsigned) {
        for (int64_t e = lo; e < hi; ++e)
            for (int a = 0; a < n; ++a) {
                const int32_t *c0 = col_idx.data() + row_ptr[dofs[e * n + a]];
                const int32_t *c1 = col_idx.data() + row_ptr[dofs[e * n + a] + 1];
                for (int b = 0; b < n; ++b)
                    pos[e * nn + (int64_t)a * n + b] = (uint16_t)(std::lower_bound(c0, c1, dofs[e * n + b]) - c0);
            }
    });

    // greedy colouring in element order
    std::vector<int32_t> color(ne, -1);
    std::vector<int64_t> used;          // used[c] == e: colour c taken by a neighbour of e
    int ncolors = 0;
    for (int64_t e = 0; e < ne; ++e) {
        for (int a = 0; a < n; ++a) {
            const int32_t g = dofs[e * n + a];
            for (int64_t k = inc_ptr[g]; k < inc_ptr[g + 1]; ++k) {
                const int32_t c = color[inc[k]];
                if (c >= 0) used[c] = e;
            }
        }
        int c = 0;
        while (c < ncolors && used[c] == e) ++c;
        if (c == ncolors) { ++ncolors; used.push_back(-1); }
        color[e] = c;
    }
    std::vector<int64_t> cstart(ncolors + 1, 0);
    for (int64_t e = 0; e < ne; ++e) cstart[color[e] + 1]++;
    for (int c = 0; c < ncolors; ++c) cstart[c + 1] += cstart[c];
    std::vector<int32_t> elems(ne);
    {
        std::vector<int64_t> fill(cstart.begin(), cstart.end() - 1);
        for (int64_t e = 0; e < ne; ++e) elems[fill[color[e]]++] = (int32_t)e;
    }

    // upload
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t s_rp = al((ndof + 1) * 8), s_ci = al(nnz * 4), s_d = al(ne * n * 4), s_el = al(ne * 4),
                 s_pos = al(ne * nn * 2);
    feint_asm_plan *pl = new feint_asm_plan;
    if (hipGetDevice(&pl->dev) != hipSuccess) { delete pl; return FEINT_ERR_HIP; }
    hipError_t err = hipMalloc(&pl->base, s_rp + s_ci + s_d + s_el + s_pos);
    if (err != hipSuccess) { set_error("asm plan allocation", err); delete pl; return FEINT_ERR_HIP; }
    char *p = (char *)pl->base;
    pl->row_ptr = (int64_t *)p; p += s_rp;
    pl->col_idx = (int32_t *)p; p += s_ci;
    pl->dofs = (int32_t *)p; p += s_d;
    pl->elems = (int32_t *)p; p += s_el;
    pl->pos = (uint16_t *)p;
    const bool ok = hipMemcpy(pl->row_ptr, row_ptr.data(), (ndof + 1) * 8, hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(pl->col_idx, col_idx.data(), nnz * 4, hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(pl->dofs, dofs, ne * n * 4, hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(pl->elems, elems.data(), ne * 4, hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(pl->pos, pos.data(), ne * nn * 2, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        set_error("asm plan upload", hipGetLastError());
        (void)hipFree(pl->base);
        delete pl;
        return FEINT_ERR_HIP;
    }
    pl->ne = ne; pl->ndof = ndof; pl->nnz = nnz; pl->n = n; pl->ncolors = ncolors;
    pl->color_start = std::move(cstart);
    pl->color_of = std::move(color);
    *out = pl;
    return FEINT_OK;
}

feint_status feint_asm_plan_info(const feint_asm_plan *pl, int64_t *nnz, int *ncolors) {
    if (!pl) return FEINT_ERR_INVALID_ARG;
    if (nnz) *nnz = pl->nnz;
    if (ncolors) *ncolors = pl->ncolors;
    return FEINT_OK;
}

feint_status feint_asm_plan_pattern(const feint_asm_plan *pl, int64_t *row_ptr, int32_t *col_idx, void *stream) {
    if (!pl || !row_ptr || !col_idx) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(row_ptr, pl->row_ptr, (pl->ndof + 1) * 8, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(col_idx, pl->col_idx, pl->nnz * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) { set_error("asm pattern copy", e); return FEINT_ERR_HIP; }
    return FEINT_OK;
}

feint_status feint_asm_plan_colors(const feint_asm_plan *pl, int32_t *color_of) {
    if (!pl || !color_of) return FEINT_ERR_INVALID_ARG;
    std::memcpy(color_of, pl->color_of.data(), pl->ne * sizeof(int32_t));
    return FEINT_OK;
}

feint_status feint_assemble(feint_asm_plan *pl, feint_form form, const void *A, const void *b, void *values,
                            void *rhs, int accumulate, void *stream) {
    if (!pl) return FEINT_ERR_INVALID_ARG;
    if (form != FEINT_FP64 && form != FEINT_FP32 && form != FEINT_BF16X3 && form != FEINT_FP16X3)
        return FEINT_ERR_UNSUPPORTED_FORM;
    if (!A || !b || !values || !rhs) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();
    const bool f64 = form == FEINT_FP64;
    if (!accumulate) {
        const int64_t nv = pl->nnz, nr = pl->ndof;
        if (f64) {
            hipLaunchKernelGGL(fill_zero<double>, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, (double *)values, nv);
            hipLaunchKernelGGL(fill_zero<double>, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, (double *)rhs, nr);
        } else {
            hipLaunchKernelGGL(fill_zero<float>, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, (float *)values, nv);
            hipLaunchKernelGGL(fill_zero<float>, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, (float *)rhs, nr);
        }
    }
    for (int c = 0; c < pl->ncolors; ++c) {
        const int64_t first = pl->color_start[c], count = pl->color_start[c + 1] - first;
        const unsigned blocks = (unsigned)((count + 3) / 4);
        if (f64)
            hipLaunchKernelGGL(scatter_color<double>, dim3(blocks), dim3(256), 0, st, (const double *)A,
                               (const double *)b, pl->elems, first, count, pl->dofs, pl->row_ptr, pl->pos, pl->n,
                               (double *)values, (double *)rhs);
        else
            hipLaunchKernelGGL(scatter_color<float>, dim3(blocks), dim3(256), 0, st, (const float *)A,
                               (const float *)b, pl->elems, first, count, pl->dofs, pl->row_ptr, pl->pos, pl->n,
                               (float *)values, (float *)rhs);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("assembly launch", e); return FEINT_ERR_HIP; }
    return FEINT_OK;
}

void feint_asm_plan_destroy(feint_asm_plan *pl) {
    if (!pl) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(pl->dev);
    (void)hipDeviceSynchronize();
    (void)hipFree(pl->base);
    (void)hipSetDevice(cur);
    delete pl;
}

}  // extern "C"
