// Mixed-degree batches: integer degree bucketing and one persistent,
// degree-bucketed launch (optionally captured in a HIP graph).
//
// The paper (Sec. 2.2) recommends grouping elements by type and degree so the
// reference data of a group is fetched once.  Here the grouping is done on
// the device:
//   k_count    per block of 1024 elements: count per degree, sum of n^2, n;
//   k_scan     one workgroup: exclusive scans of those block sums, bucket
//              starts (heaviest degree first), totals of the packed outputs;
//   k_scatter  per block: stable rank of every element inside its degree,
//              the permutation into bucket order and the packed offsets;
//   k_prep     one lane: work-queue extents for the chosen tile shapes;
//   k_persist  persistent waves pulling work items (element, tile block)
//              from an atomic counter, heaviest degree first, each running
//              the same per-degree device code as the direct kernels.
// No memset nodes are used (counters are cleared by kernels), so the whole
// sequence is safe to capture and replay.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "capi_internal.h"
#include "fwd_kernels.h"
#include "fwd_valu.h"
#include "fwd_fact.h"
#include "tables.h"

namespace feint {

constexpr int MIX_MAXP = 6;
constexpr int BUCKET_ELEMS = 1024;   // elements per bucketing block (256 threads x 4)
constexpr int SCAN_THREADS = 1024;

struct MixedHdr {
    int32_t count[8];    // elements of degree p
    int32_t bstart[8];   // first slot of degree p's bucket in the permutation
    int64_t gstart[8];   // first work grab of degree p
    int64_t ngrab[8];
    int64_t total_grabs;
    uint32_t queue;      // next grab
    uint32_t pad;
};

struct MixSizes {
    int32_t items[8];    // work items per group of element slots (tile blocks) of degree p
    int32_t epi[8];      // element slots per group (1, or the elements of a vector-ALU wave)
    int32_t grab[8];     // work items taken per queue grab
};

struct MixedParams {
    FwdParams base;      // element inputs, outputs, packed offsets, status
    const double *qw[8];
    const double *B64[8];
    const float *B32[8];
    const double *tau64[8];   // per-degree factor tables of the triangle-point contraction
    const float *tau32[8];
    const double *lam[8];
    const float *lam32[8];
    const int32_t *perm;
    MixedHdr *hdr;
    MixSizes sz;
};

__device__ inline int nshp_dev(int p) { return (p + 1) * (p + 1) * (p + 2) / 2; }

// 8 per-thread values: [0] sum n^2, [1..6] count of degree p, [7] sum n.
__device__ inline void thread_counts(const int8_t *p, int64_t ne, int64_t base, int64_t c[8], uint32_t *status) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t e = base + u;
        if (e < ne) {
            const int d = p[e];
            if (d >= 1 && d <= MIX_MAXP) {
                const int n = nshp_dev(d);
                c[d] += 1;
                c[0] += (int64_t)n * n;
                c[7] += n;
            } else if (status) {
                atomicOr(status, 2u);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_count(const int8_t *p, int64_t ne, int64_t *blk_sums, uint32_t *status) {
    __shared__ int64_t red[8][256];
    int64_t c[8];
    thread_counts(p, ne, (int64_t)blockIdx.x * BUCKET_ELEMS + threadIdx.x * 4, c, status);
#pragma unroll
    for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = c[k];
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 8) blk_sums[(int64_t)blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// Exclusive scan (in place) over nblk blocks of the 8 sums; bucket layout.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan(int64_t nblk, int64_t *blk_sums, MixedHdr *hdr, int64_t *offA,
                                                       int64_t *offb, int64_t ne) {
    __shared__ int64_t s[8][SCAN_THREADS];
    const int t = threadIdx.x;
    const int64_t per = (nblk + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t j0 = t * per, j1 = (j0 + per < nblk) ? j0 + per : nblk;
    int64_t loc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) loc[k] = 0;
    for (int64_t j = j0; j < j1; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k) loc[k] += blk_sums[j * 8 + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k][t] = loc[k];
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        int64_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = t >= off ? s[k][t - off] : 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k][t] += v[k];
        __syncthreads();
    }
    int64_t run[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) run[k] = s[k][t] - loc[k];
    for (int64_t j = j0; j < j1; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t v = blk_sums[j * 8 + k];
            blk_sums[j * 8 + k] = run[k];
            run[k] += v;
        }
    if (t == SCAN_THREADS - 1) {
        int32_t acc = 0;
        for (int d = MIX_MAXP; d >= 1; --d) {
            hdr->count[d] = (int32_t)s[d][t];
            hdr->bstart[d] = acc;
            acc += (int32_t)s[d][t];
        }
        hdr->count[0] = 0;
        hdr->bstart[0] = acc;
        offA[ne] = s[0][t];
        offb[ne] = s[7][t];
    }
}

__global__ __launch_bounds__(256) void k_scatter(const int8_t *p, int64_t ne, const int64_t *blk_pref,
                                                 const MixedHdr *hdr, int32_t *perm, int64_t *offA, int64_t *offb) {
    __shared__ int64_t s[8][256];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * BUCKET_ELEMS + t * 4;
    int64_t c[8];
    thread_counts(p, ne, base, c, nullptr);
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k][t] = c[k];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int64_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = t >= off ? s[k][t - off] : 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k][t] += v[k];
        __syncthreads();
    }
    int64_t run[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) run[k] = blk_pref[(int64_t)blockIdx.x * 8 + k] + s[k][t] - c[k];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t e = base + u;
        if (e < ne) {
            const int d = p[e];
            offA[e] = run[0];
            offb[e] = run[7];
            if (d >= 1 && d <= MIX_MAXP) {
                const int n = nshp_dev(d);
                perm[hdr->bstart[d] + run[d]] = (int32_t)e;
                run[d] += 1;
                run[0] += (int64_t)n * n;
                run[7] += n;
            }
        }
    }
}

__global__ void k_prep(MixedHdr *hdr, MixSizes sz) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t g = 0;
        for (int d = MIX_MAXP; d >= 1; --d) {
            const int64_t items = (hdr->count[d] + sz.epi[d] - 1) / sz.epi[d] * sz.items[d];
            hdr->ngrab[d] = (items + sz.grab[d] - 1) / sz.grab[d];
            hdr->gstart[d] = g;
            g += hdr->ngrab[d];
        }
        hdr->total_grabs = g;
        hdr->queue = 0u;
    }
}

// Each wave owns one LDS slice large enough for any degree's kernel, so waves
// of a workgroup working on different degrees never share LDS.
template <class KER>
__device__ __attribute__((noinline)) void run_item(const MixedParams &mp, int d, int64_t item, void *slice) {
    FwdParams prm = mp.base;
    prm.qw = mp.qw[d];
    prm.B64 = mp.B64[d];
    prm.B32 = mp.B32[d];
    prm.tau64 = mp.tau64[d];
    prm.tau32 = mp.tau32[d];
    prm.lam = mp.lam[d];
    prm.lam32 = mp.lam32[d];
    prm.perm = mp.perm + mp.hdr->bstart[d];
    prm.ne = mp.hdr->count[d];          // slots of this bucket
    KER::run_slice(prm, item / KER::NBLK, (int)(item % KER::NBLK), *(typename KER::Slice *)slice);
}

template <class... K> struct MaxSlice;
template <class K> struct MaxSlice<K> { static constexpr size_t value = (sizeof(typename K::Slice) + 15) / 16 * 16; };
template <class K, class... R> struct MaxSlice<K, R...> {
    static constexpr size_t value = MaxSlice<K>::value > MaxSlice<R...>::value ? MaxSlice<K>::value
                                                                               : MaxSlice<R...>::value;
};

// One wave per SIMD: the per-degree device functions are called, not inlined,
// and the largest tiles need the whole register file.
template <class K1, class K2, class K3, class K4_, class K5, class K6>
__global__ __launch_bounds__(256, 1) void k_persist(MixedParams mp) {
    constexpr size_t SL = MaxSlice<K1, K2, K3, K4_, K5, K6>::value;
    __shared__ __attribute__((aligned(16))) char sm[4 * SL];
    const int wave = wave_uniform(threadIdx.x >> 6);
    void *slice = sm + wave * SL;
    const int lane = threadIdx.x & 63;
    MixedHdr *h = mp.hdr;
    const int64_t total = h->total_grabs;
    for (;;) {
        uint32_t g = 0;
        if (lane == 0) g = atomicAdd(&h->queue, 1u);
        g = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl(g, 0, 64));
        if ((int64_t)g >= total) break;
        int d = MIX_MAXP;
        while (d > 1 && (int64_t)g >= h->gstart[d] + h->ngrab[d]) --d;
        const int64_t nitems = (h->count[d] + mp.sz.epi[d] - 1) / mp.sz.epi[d] * mp.sz.items[d];
        const int64_t first = ((int64_t)g - h->gstart[d]) * mp.sz.grab[d];
        const int64_t last = first + mp.sz.grab[d] < nitems ? first + mp.sz.grab[d] : nitems;
        for (int64_t it = first; it < last; ++it) {
            switch (d) {
            case 1: run_item<K1>(mp, 1, it, slice); break;
            case 2: run_item<K2>(mp, 2, it, slice); break;
            case 3: run_item<K3>(mp, 3, it, slice); break;
            case 4: run_item<K4_>(mp, 4, it, slice); break;
            case 5: run_item<K5>(mp, 5, it, slice); break;
            default: run_item<K6>(mp, 6, it, slice); break;
            }
        }
    }
}

// One compiled set of per-degree tile shapes.
struct MixVariant {
    const void *kernel;
    MixSizes sz;
    const char *desc;
};

template <class K1, class K2, class K3, class K4_, class K5, class K6>
MixVariant make_variant(const char *desc) {
    MixVariant v;
    v.kernel = (const void *)&k_persist<K1, K2, K3, K4_, K5, K6>;
    std::memset(&v.sz, 0, sizeof v.sz);
    const int items[7] = {0, K1::NBLK, K2::NBLK, K3::NBLK, K4_::NBLK, K5::NBLK, K6::NBLK};
    const int epi[7] = {0, K1::EPI, K2::EPI, K3::EPI, K4_::EPI, K5::EPI, K6::EPI};
    const int grab[7] = {0, 32, 8, 2, 1, 1, 1};   // elements' worth of work per grab
    for (int d = 1; d <= MIX_MAXP; ++d) {
        v.sz.items[d] = items[d];
        v.sz.epi[d] = epi[d];
        v.sz.grab[d] = grab[d] / epi[d] > 1 ? grab[d] / epi[d] : 1;
    }
    v.desc = desc;
    return v;
}

const MixVariant *mix_variants(int form, int *count) {
    // p = 1, 2 on the vector ALUs (v8: 8 lanes per element, v18: 18), MFMA tiles above:
    // the contraction per triangle point (KxTNf) or point by point (TMxTN); the last set
    // of each form keeps point-by-point MFMA tiles at every degree for comparison
    static const MixVariant f32[] = {
        make_variant<KV<1, float, 8>, KV<2, float, 18>, KF<3, float, 4, 4>, KF<4, float, 5, 3>,
                     KF<5, float, 6, 3>, KF<6, float, 7, 4>>("v8,v18,4x4f,5x3f,6x3f,7x4f"),
        make_variant<KV<1, float, 8>, KV<2, float, 18>, KF<3, float, 4, 4>, KF<4, float, 5, 5>,
                     KF<5, float, 6, 3>, KF<6, float, 7, 3>>("v8,v18,4x4f,5x5f,6x3f,7x3f"),
        make_variant<KV<1, float, 8>, KV<2, float, 18>, K4<3, float, 3, 3>, K4<4, float, 5, 5>,
                     K4<5, float, 8, 8>, K4<6, float, 13, 5>>("v8,v18,3x3,5x5,8x8,13x5"),
        make_variant<KV<1, float, 8>, KV<2, float, 18>, K4<3, float, 3, 3>, K4<4, float, 5, 5>,
                     K4<5, float, 8, 8>, K4<6, float, 13, 4>>("v8,v18,3x3,5x5,8x8,13x4"),
        make_variant<KV<1, float, 8>, KV<2, float, 18>, K4<3, float, 3, 3>, K4<4, float, 5, 5>,
                     K4<5, float, 8, 8>, K4<6, float, 13, 3>>("v8,v18,3x3,5x5,8x8,13x3"),
        make_variant<KV<1, float, 8>, KV<2, float, 18>, K4<3, float, 3, 3>, K4<4, float, 5, 3>,
                     K4<5, float, 8, 2>, K4<6, float, 13, 1>>("v8,v18,3x3,5x3,8x2,13x1"),
        make_variant<KV<1, float, 8>, KV<2, float, 18>, K4<3, float, 3, 3>, K4<4, float, 5, 5>,
                     K4<5, float, 8, 4>, K4<6, float, 13, 2>>("v8,v18,3x3,5x5,8x4,13x2"),
        make_variant<K4<1, float, 1, 1>, K4<2, float, 2, 2>, K4<3, float, 3, 3>, K4<4, float, 5, 3>,
                     K4<5, float, 8, 2>, K4<6, float, 13, 1>>("1x1,2x2,3x3,5x3,8x2,13x1"),
    };
    static const MixVariant f64[] = {
        make_variant<KV<1, double, 8>, KV<2, double, 18>, KF<3, double, 4, 2>, KF<4, double, 5, 5>,
                     KF<5, double, 6, 2>, KF<6, double, 7, 1>>("v8,v18,4x2f,5x5f,6x2f,7x1f"),
        make_variant<KV<1, double, 8>, KV<2, double, 18>, KF<3, double, 4, 2>, KF<4, double, 5, 5>,
                     KF<5, double, 3, 2>, KF<6, double, 7, 1>>("v8,v18,4x2f,5x5f,3x2f,7x1f"),
        make_variant<KV<1, double, 8>, KV<2, double, 18>, KF<3, double, 4, 2>, KF<4, double, 5, 3>,
                     KF<5, double, 6, 1>, KF<6, double, 4, 2>>("v8,v18,4x2f,5x3f,6x1f,4x2f"),
        make_variant<KV<1, double, 8>, KV<2, double, 18>, K4<3, double, 3, 3>, K4<4, double, 5, 3>,
                     K4<5, double, 8, 4>, K4<6, double, 13, 2>>("v8,v18,3x3,5x3,8x4,13x2"),
        make_variant<KV<1, double, 8>, KV<2, double, 18>, K4<3, double, 3, 3>, K4<4, double, 5, 1>,
                     K4<5, double, 8, 1>, K4<6, double, 13, 1>>("v8,v18,3x3,5x1,8x1,13x1"),
        make_variant<KV<1, double, 8>, KV<2, double, 18>, K4<3, double, 3, 1>, K4<4, double, 5, 2>,
                     K4<5, double, 8, 2>, K4<6, double, 13, 1>>("v8,v18,3x1,5x2,8x2,13x1"),
        make_variant<K4<1, double, 1, 1>, K4<2, double, 2, 2>, K4<3, double, 3, 3>, K4<4, double, 5, 1>,
                     K4<5, double, 8, 1>, K4<6, double, 13, 1>>("1x1,2x2,3x3,5x1,8x1,13x1"),
    };
    if (form == FEINT_FP32) { *count = (int)(sizeof f32 / sizeof f32[0]); return f32; }
    if (form == FEINT_FP64) { *count = (int)(sizeof f64 / sizeof f64[0]); return f64; }
    *count = 0;
    return nullptr;
}

}  // namespace feint

using namespace feint;

struct feint_mixed_plan {
    int dev = 0;
    int form = 0;
    int64_t ne_max = 0, nblk_max = 0;
    int64_t ne_bucketed = -1;    // batch size the plan's bucketing scratch holds (-1: none yet)
    int64_t ne_captured = -1;    // batch size the captured graph buckets when it is launched
    char *scratch = nullptr;
    MixedHdr *hdr = nullptr;
    int64_t *blk_sums = nullptr;
    int32_t *perm = nullptr;
    int tile = 0;
    int grid[16] = {0};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const DevTables *tab[8] = {nullptr};
};

namespace {

feint_status hip_fail(const char *what, hipError_t e) {
    set_error(what, e);
    return FEINT_ERR_HIP;
}

void drop_graph(feint_mixed_plan *pl) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
}

// Device memory one bucketing + persistent launch works in: the queue header,
// the per-block degree sums and the permutation into bucket order, plus the
// degree tables and the launch grid of each compiled tile set.
struct MixedWork {
    MixedHdr *hdr;
    int64_t *blk_sums;
    int32_t *perm;
    const DevTables *const *tab;   // [8], degrees 1..6
    int form;
    const int *grid;               // per compiled tile set
};

// Bytes of scratch a batch of ne elements needs: header, block sums, permutation.
constexpr size_t SCR_HDR = 256;
constexpr size_t scratch_blk_bytes(int64_t ne) {
    return ((size_t)((ne + BUCKET_ELEMS - 1) / BUCKET_ELEMS) * 8 * 8 + 255) / 256 * 256;
}
constexpr size_t scratch_bytes(int64_t ne) {
    return SCR_HDR + scratch_blk_bytes(ne) + ((size_t)ne * 4 + 255) / 256 * 256;
}

MixedWork work_in(char *base, int64_t ne_max, const DevTables *const *tab, int form, const int *grid) {
    MixedWork w;
    w.hdr = (MixedHdr *)base;
    w.blk_sums = (int64_t *)(base + SCR_HDR);
    w.perm = (int32_t *)(base + SCR_HDR + scratch_blk_bytes(ne_max));
    w.tab = tab;
    w.form = form;
    w.grid = grid;
    return w;
}

feint_status enqueue_bucket(const MixedWork &w, const int8_t *p, int64_t ne, int64_t *offA, int64_t *offb,
                            uint32_t *status, hipStream_t s) {
    const int64_t nblk = (ne + BUCKET_ELEMS - 1) / BUCKET_ELEMS;
    (void)hipGetLastError();
    if (nblk > 0) hipLaunchKernelGGL(k_count, dim3((unsigned)nblk), dim3(256), 0, s, p, ne, w.blk_sums, status);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(SCAN_THREADS), 0, s, nblk, w.blk_sums, w.hdr, offA, offb, ne);
    if (nblk > 0)
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)nblk), dim3(256), 0, s, p, ne, (const int64_t *)w.blk_sums,
                           (const MixedHdr *)w.hdr, w.perm, offA, offb);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FEINT_OK : hip_fail("bucketing launch", e);
}

feint_status enqueue_persist(const MixedWork &w, const feint_elements *el, void *A, void *b, const int64_t *offA,
                             const int64_t *offb, uint32_t *status, hipStream_t s, int tile) {
    int cnt = 0;
    const MixVariant *vars = mix_variants(w.form, &cnt);
    const MixVariant &v = vars[tile];
    MixedParams mp;
    std::memset(&mp, 0, sizeof mp);
    mp.base.coords = el->coords; mp.base.D = el->D; mp.base.beta = el->beta; mp.base.c = el->c; mp.base.f = el->f;
    mp.base.ne = el->ne;
    mp.base.A = A; mp.base.b = b; mp.base.status = status;
    mp.base.offA = offA; mp.base.offb = offb;
    for (int d = 1; d <= MIX_MAXP; ++d) {
        mp.qw[d] = w.tab[d]->qw;
        mp.B64[d] = w.tab[d]->B64;
        mp.B32[d] = w.tab[d]->B32;
        mp.tau64[d] = w.tab[d]->tau64;
        mp.tau32[d] = w.tab[d]->tau32;
        mp.lam[d] = w.tab[d]->lam;
        mp.lam32[d] = w.tab[d]->lam32;
    }
    mp.perm = w.perm;
    mp.hdr = w.hdr;
    mp.sz = v.sz;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(64), 0, s, w.hdr, v.sz);
    void *args[] = {&mp};
    hipError_t e = hipLaunchKernel(v.kernel, dim3(w.grid[tile]), dim3(256), args, 0, s);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? FEINT_OK : hip_fail("persistent launch", e);
}

// Launch grid of every compiled tile set of `form` on device `dev`: as many
// workgroups as fit the device at once (persistent waves).
hipError_t persistent_grids(int form, int dev, int *grid) {
    int cnt = 0, cus = 0;
    const MixVariant *vars = mix_variants(form, &cnt);
    if (cnt > 16) return hipErrorInvalidValue;          // grid arrays hold 16 tile sets
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int t = 0; t < cnt && e == hipSuccess; ++t) {
        int nb = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, vars[t].kernel, 256, 0);
        grid[t] = (nb > 0 ? nb : 1) * cus;
    }
    return e;
}

MixedWork plan_work(const feint_mixed_plan *pl) {
    return work_in(pl->scratch, pl->ne_max, pl->tab, pl->form, pl->grid);
}

// ---- The allocation-free entry point --------------------------------------
// Its bucketing scratch (queue header, block sums, permutation) is this
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int64_t NOALLOC_MAX_NE = FEINT_NOALLOC_MAX_NE;
static __device__ __align__(256) unsigned char scratch[scratch_bytes(NOALLOC_MAX_NE)];

struct NoAllocDev {
    char *ptr = nullptr;          // device address of `scratch` on this device
    int grid[2][16] = {{0}};      // persistent grid per form (FP64, FP32) and tile set
};
std::mutex g_na_mu;
std::map<int, NoAllocDev> g_na;   // key: device

// Set-up of the current device on its first call: the scratch's device
// address and the persistent grids.  Neither allocates device memory.
feint_status noalloc_device(int dev, const NoAllocDev **out) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    auto it = g_na.find(dev);
    if (it == g_na.end()) {
        NoAllocDev nd;
        hipError_t e = hipGetSymbolAddress((void **)&nd.ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !nd.ptr) return hip_fail("hipGetSymbolAddress(scratch)", e);
        e = persistent_grids(FEINT_FP64, dev, nd.grid[0]);
        if (e == hipSuccess) e = persistent_grids(FEINT_FP32, dev, nd.grid[1]);
        if (e != hipSuccess) return hip_fail("persistent grid", e);
        it = g_na.emplace(dev, nd).first;
    }
    *out = &it->second;
    return FEINT_OK;
}

}  // namespace

extern "C" {

feint_status feint_mixed_plan_create(int64_t ne_max, feint_form form, feint_mixed_plan **plan) {
    if (!plan || ne_max < 1) return FEINT_ERR_INVALID_ARG;
    *plan = nullptr;
    if (form != FEINT_FP32 && form != FEINT_FP64) return FEINT_ERR_UNSUPPORTED_FORM;
    if (ne_max > 0x7fffffffLL) return FEINT_ERR_TOO_LARGE;
    feint_mixed_plan *pl = new feint_mixed_plan();
    pl->form = form;
    pl->ne_max = ne_max;
    pl->nblk_max = (ne_max + BUCKET_ELEMS - 1) / BUCKET_ELEMS;
    if (pl->nblk_max > (int64_t)SCAN_THREADS * 4096) { delete pl; return FEINT_ERR_TOO_LARGE; }
    hipError_t e = hipGetDevice(&pl->dev);
    if (e != hipSuccess) { delete pl; return hip_fail("hipGetDevice", e); }
    for (int d = 1; d <= MIX_MAXP; ++d) {
        feint_status s = prepare_tables(d);
        if (s != FEINT_OK) { delete pl; return s; }
        pl->tab[d] = find_tables(d);
    }
    e = hipMalloc((void **)&pl->scratch, scratch_bytes(ne_max));
    if (e != hipSuccess) { delete pl; return hip_fail("hipMalloc(plan)", e); }
    e = persistent_grids(form, pl->dev, pl->grid);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(pl->scratch);
        delete pl;
        return hip_fail("plan setup", e);
    }
    *plan = pl;
    return FEINT_OK;
}

feint_status feint_mixed_bucket(feint_mixed_plan *pl, const int8_t *p, int64_t ne, int64_t *offA, int64_t *offb,
                                uint32_t *dev_status, void *stream) {
    if (!pl || !offA || !offb || ne < 0) return FEINT_ERR_INVALID_ARG;
    if (ne > pl->ne_max) return FEINT_ERR_TOO_LARGE;
    if (ne > 0 && !p) return FEINT_ERR_INVALID_ARG;
    feint_status s = enqueue_bucket(plan_work(pl), p, ne, offA, offb, dev_status, (hipStream_t)stream);
    if (s == FEINT_OK) pl->ne_bucketed = ne;
    return s;
}

feint_status feint_integrate_mixed(feint_mixed_plan *pl, const feint_elements *el, void *A, void *b,
                                   const int64_t *offA, const int64_t *offb, uint32_t *dev_status, void *stream) {
    if (!pl) return FEINT_ERR_INVALID_ARG;
    feint_status s = check_elements(el);
    if (s != FEINT_OK) return s;
    if (el->ne != pl->ne_bucketed) return FEINT_ERR_INVALID_ARG;   // bucket this batch first
    if (el->ne == 0) return FEINT_OK;
    if (!A || !b || !offA || !offb) return FEINT_ERR_INVALID_ARG;
    return enqueue_persist(plan_work(pl), el, A, b, offA, offb, dev_status, (hipStream_t)stream, pl->tile);
}

feint_status feint_mixed_graph_capture(feint_mixed_plan *pl, const feint_elements *el, const int8_t *p, void *A,
                                       void *b, int64_t *offA, int64_t *offb, uint32_t *dev_status, void *stream) {
    (void)stream;
    if (!pl) return FEINT_ERR_INVALID_ARG;
    feint_status s = check_elements(el);
    if (s != FEINT_OK) return s;
    if (el->ne > pl->ne_max) return FEINT_ERR_TOO_LARGE;
    if (el->ne > 0 && (!p || !A || !b)) return FEINT_ERR_INVALID_ARG;
    if (!offA || !offb) return FEINT_ERR_INVALID_ARG;
    drop_graph(pl);
    pl->ne_captured = -1;
    hipError_t e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail("hipStreamBeginCapture", e);
    const MixedWork w = plan_work(pl);
    s = enqueue_bucket(w, p, el->ne, offA, offb, dev_status, pl->cap_stream);
    if (s == FEINT_OK && el->ne > 0) s = enqueue_persist(w, el, A, b, offA, offb, dev_status, pl->cap_stream, pl->tile);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(pl->cap_stream, &g);
    if (s != FEINT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return hip_fail("hipStreamEndCapture", e);
    pl->graph = g;
    e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(pl);
        return hip_fail("hipGraphInstantiate", e);
    }
    // Capturing runs nothing: the bucketing scratch still holds whatever the last eager
    // bucketing (if any) left there, so ne_bucketed is unchanged until the graph runs.
    pl->ne_captured = el->ne;
    return FEINT_OK;
}

feint_status feint_mixed_graph_launch(feint_mixed_plan *pl, void *stream) {
    if (!pl) return FEINT_ERR_INVALID_ARG;
    if (!pl->exec) return FEINT_ERR_NOT_PREPARED;
    hipError_t e = hipGraphLaunch(pl->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail("hipGraphLaunch", e);
    pl->ne_bucketed = pl->ne_captured;      // the graph's bucketing rewrites the scratch
    return FEINT_OK;
}

feint_status feint_mixed_autotune(feint_mixed_plan *pl, const feint_elements *el, void *A, void *b,
                                  const int64_t *offA, const int64_t *offb, int reps, double *best_ms, void *stream) {
    if (!pl || reps < 1) return FEINT_ERR_INVALID_ARG;
    feint_status s = check_elements(el);
    if (s != FEINT_OK) return s;
    if (el->ne != pl->ne_bucketed || el->ne == 0) return FEINT_ERR_INVALID_ARG;
    if (!A || !b || !offA || !offb) return FEINT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    int cnt = 0;
    mix_variants(pl->form, &cnt);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return FEINT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return FEINT_ERR_HIP; }
    int best = pl->tile;
    float best_t = 1e30f;
    for (int t = 0; t < cnt && s == FEINT_OK; ++t) {
        const MixedWork w = plan_work(pl);
        s = enqueue_persist(w, el, A, b, offA, offb, nullptr, st, t);
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && s == FEINT_OK; ++r) s = enqueue_persist(w, el, A, b, offA, offb, nullptr, st, t);
        (void)hipEventRecord(e1, st);
        if (s != FEINT_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) { s = FEINT_ERR_HIP; break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_t) { best_t = ms; best = t; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != FEINT_OK) return s;
    if (best != pl->tile) drop_graph(pl);   // a captured graph holds the old kernels
    pl->tile = best;
    if (best_ms) *best_ms = best_t;
    return FEINT_OK;
}

int feint_mixed_tile_count(const feint_mixed_plan *pl) {
    int cnt = 0;
    if (!pl) return 0;
    mix_variants(pl->form, &cnt);
    return cnt;
}

int feint_mixed_tile_get(const feint_mixed_plan *pl) { return pl ? pl->tile : -1; }

feint_status feint_mixed_tile_describe(const feint_mixed_plan *pl, int tile, char *buf, size_t len) {
    if (!pl || !buf || len == 0 || tile < 0 || tile >= feint_mixed_tile_count(pl)) return FEINT_ERR_INVALID_ARG;
    int cnt = 0;
    const MixVariant *v = mix_variants(pl->form, &cnt);
    std::snprintf(buf, len, "%s", v[tile].desc);
    return FEINT_OK;
}

feint_status feint_mixed_tile_set(feint_mixed_plan *pl, int tile) {
    if (!pl || tile < 0 || tile >= feint_mixed_tile_count(pl)) return FEINT_ERR_INVALID_ARG;
    if (tile != pl->tile) drop_graph(pl);
    pl->tile = tile;
    return FEINT_OK;
}

void feint_mixed_plan_destroy(feint_mixed_plan *pl) {
    if (!pl) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(pl->dev);
    drop_graph(pl);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    (void)hipFree(pl->scratch);
    (void)hipSetDevice(cur);
    delete pl;
}

feint_status feint_integrate_mixed_noalloc(const feint_elements *el, const int8_t *p, feint_form form, void *A,
                                           void *b, int64_t *offA, int64_t *offb, uint32_t *dev_status,
                                           void *stream) {
    if (form != FEINT_FP32 && form != FEINT_FP64) return FEINT_ERR_UNSUPPORTED_FORM;
    feint_status s = check_elements(el);
    if (s != FEINT_OK) return s;
    if (el->ne > NOALLOC_MAX_NE) {
        set_error_msg("feint_integrate_mixed_noalloc: " + std::to_string(el->ne) + " elements exceed the " +
                      std::to_string(NOALLOC_MAX_NE) + " its fixed scratch holds");
        return FEINT_ERR_TOO_LARGE;
    }
    if (!offA || !offb) return FEINT_ERR_INVALID_ARG;
    if (el->ne > 0 && (!p || !A || !b)) return FEINT_ERR_INVALID_ARG;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    // the degree tables must exist already: preparing them would allocate
    const DevTables *tab[8] = {nullptr};
    for (int d = 1; d <= MIX_MAXP; ++d)
        if (!(tab[d] = find_tables(d))) return FEINT_ERR_NOT_PREPARED;
    const NoAllocDev *nd = nullptr;
    s = noalloc_device(dev, &nd);
    if (s != FEINT_OK) return s;
    const MixedWork w = work_in(nd->ptr, NOALLOC_MAX_NE, tab, form, nd->grid[form == FEINT_FP64 ? 0 : 1]);
    const hipStream_t st = (hipStream_t)stream;
    s = enqueue_bucket(w, p, el->ne, offA, offb, dev_status, st);
    if (s != FEINT_OK || el->ne == 0) return s;
    return enqueue_persist(w, el, A, b, offA, offb, dev_status, st, 0);
}

}  // extern "C"
