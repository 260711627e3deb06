// Context management, allocation, error reporting and the scan primitive.
#include <cstdio>
#include <cstring>

#include "common.h"

void destroy_solve_cache(SolveCache* c);
// Device address of dec_solve_noalloc's static scratch on `device` (the current
// device), taken once per device; a failure is kept and reported by that call.
void noalloc_setup(int device);

void* dec_ctx::dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) return nullptr;
    if (alloc) {
        p = alloc(bytes, user);
        if (!p) dec_fail(DEC_ENOMEM, "allocation callback returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            dec_fail(DEC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
    }
    return p;
}

void dec_ctx::dfree(void* p) {
    if (!p) return;
    if (free_fn)
        free_fn(p, user);
    else
        (void)hipFree(p);
}

void* dec_ctx::readback(const void* dptr, size_t bytes) {
    if (bytes > pinned_bytes) {
        if (pinned) (void)hipHostFree(pinned);
        pinned = nullptr;
        size_t want = bytes < 4096 ? 4096 : bytes;
        HIP_CHECK(hipHostMalloc(&pinned, want, hipHostMallocDefault));
        pinned_bytes = want;
    }
    HIP_CHECK(hipMemcpyAsync(pinned, dptr, bytes, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    return pinned;
}

dec_mesh::~dec_mesh() {
    if (solve) destroy_solve_cache(solve);
    solve = nullptr;
    delete dual;
    dual = nullptr;
    if (owner) owner->live_children -= 1;
}

// ---------------------------------------------------------------- scan
namespace {
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;

// Up to three scans of the same length in one set of launches (blockIdx.y
// picks the array).
struct ScanBatch {
    const int32_t* in[3];
    int64_t* out[3];
};

__global__ void k_scan_tile_sums(ScanBatch sb, int64_t n, int64_t* __restrict__ bsum) {
    __shared__ int64_t lds[BLOCK / 64];
    const int32_t* __restrict__ in = sb.in[blockIdx.y];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) s += in[i];
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) bsum[blockIdx.y * static_cast<int64_t>(gridDim.x) + blockIdx.x] = s;
}

// One block per scan: exclusive scan of its nb tile sums, in place.
__global__ void k_scan_tile_offsets(int64_t* __restrict__ bsum_all, int64_t nb) {
    __shared__ int64_t buf[1024];
    __shared__ int64_t carry;
    int64_t* __restrict__ bsum = bsum_all + blockIdx.y * nb;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t start = 0; start < nb; start += 1024) {
        int64_t i = start + threadIdx.x;
        int64_t v = i < nb ? bsum[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int64_t t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        int64_t incl = buf[threadIdx.x];
        if (i < nb) bsum[i] = carry + incl - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += incl;
        __syncthreads();
    }
}

__global__ void k_scan_tile_apply(ScanBatch sb, int64_t n, const int64_t* __restrict__ boff_all) {
    __shared__ int64_t buf[BLOCK];
    const int32_t* __restrict__ in = sb.in[blockIdx.y];
    int64_t* __restrict__ out = sb.out[blockIdx.y];
    const int64_t* __restrict__ boff = boff_all + blockIdx.y * static_cast<int64_t>(gridDim.x);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int64_t loc[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        s += (i < n) ? in[i] : 0;
        loc[k] = s;
    }
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < BLOCK; off <<= 1) {
        int64_t t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
    }
    const int64_t excl = boff[blockIdx.x] + buf[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) out[i + 1] = excl + loc[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

// the scans' totals side by side, for one read-back
__global__ void k_scan_totals(ScanBatch sb, int m, int64_t n, int64_t* __restrict__ tot) {
    if (threadIdx.x < static_cast<unsigned>(m)) tot[threadIdx.x] = sb.out[threadIdx.x][n];
}

__global__ void k_i64_to_i32(const int64_t* __restrict__ in, int32_t* __restrict__ out, int64_t n) {
    GRID_STRIDE_LOOP(i, n) out[i] = static_cast<int32_t>(in[i]);
}
}  // namespace

// m (1 to 3) scans of arrays of the same length in one set of launches;
// totals (when given) receives the m totals (one synchronisation).
void scan_exclusive_multi(dec_ctx* ctx, int m, const int32_t* const* in, int64_t* const* out, int64_t n,
                          int64_t* totals) {
    DEC_REQUIRE(m >= 1 && m <= 3, DEC_EINVAL, "internal: 1 to 3 scans at a time");
    if (n == 0) {
        for (int k = 0; k < m; ++k) HIP_CHECK(hipMemsetAsync(out[k], 0, sizeof(int64_t), ctx->stream));
        if (totals)
            for (int k = 0; k < m; ++k) totals[k] = 0;
        return;
    }
    ScanBatch sb{};
    for (int k = 0; k < m; ++k) {
        sb.in[k] = in[k];
        sb.out[k] = out[k];
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    DBuf<int64_t> bsum;
    bsum.alloc(ctx, m * nb + 3);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(nb, m), dim3(BLOCK), 0, ctx->stream, sb, n, bsum.p);
    hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1, m), dim3(1024), 0, ctx->stream, bsum.p, nb);
    hipLaunchKernelGGL(k_scan_tile_apply, dim3(nb, m), dim3(BLOCK), 0, ctx->stream, sb, n, bsum.p);
    HIP_CHECK(hipGetLastError());
    if (totals) {
        int64_t* tot = bsum.p + m * nb;
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(64), 0, ctx->stream, sb, m, n, tot);
        HIP_CHECK(hipGetLastError());
        std::memcpy(totals, ctx->readback(tot, m * sizeof(int64_t)), m * sizeof(int64_t));
    } else {
        // keep bsum alive until the kernels ran
        ctx->sync();
    }
}

int64_t scan_exclusive_i32_to_i64(dec_ctx* ctx, const int32_t* in, int64_t* out, int64_t n, bool want_total) {
    int64_t total = -1;
    scan_exclusive_multi(ctx, 1, &in, &out, n, want_total ? &total : nullptr);
    return total;
}

void copy_i64_to_i32(dec_ctx* ctx, const int64_t* in, int32_t* out, int64_t n) {
    hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for(n)), dim3(BLOCK), 0, ctx->stream, in, out, n);
    HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------- C ABI
std::string& free_error() {
    thread_local std::string msg;
    return msg;
}

extern "C" {

const char* dec_status_string(int status) {
    switch (status) {
        case DEC_OK: return "ok";
        case DEC_EINVAL: return "invalid argument";
        case DEC_ENOMEM: return "out of device memory";
        case DEC_EHIP: return "HIP runtime error";
        case DEC_ENOTCONV: return "not converged within max_iters";
        case DEC_EBREAKDOWN: return "CG breakdown";
        case DEC_ETOPO: return "invalid mesh topology";
        case DEC_EBUDGET: return "over the HBM budget";
        case DEC_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

const char* dec_last_error(const dec_ctx* ctx) {
    if (ctx) return ctx->last_error.c_str();
    return free_error().empty() ? "no context" : free_error().c_str();
}

int dec_create(dec_ctx** out, int device, void* stream, dec_alloc_fn alloc, dec_free_fn free_fn, void* user) {
    if (!out) return DEC_EINVAL;
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) return DEC_EINVAL;
    dec_ctx* c = new dec_ctx();
    try {
        int ndev = 0;
        HIP_CHECK(hipGetDeviceCount(&ndev));
        DEC_REQUIRE(device >= 0 && device < ndev, DEC_EINVAL, "device index out of range");
        c->device = device;
        c->stream = static_cast<hipStream_t>(stream);
        c->alloc = alloc;
        c->free_fn = free_fn;
        c->user = user;
        c->set_device();
        hipDeviceProp_t prop;
        HIP_CHECK(hipGetDeviceProperties(&prop, device));
        c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        // the staging area of scalar read-backs, so that no later read-back of up to 4 KiB allocates
        HIP_CHECK(hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault));
        c->pinned_bytes = 4096;
        noalloc_setup(device);
    } catch (const DecError& e) {
        int code = e.code;
        if (c->pinned) (void)hipHostFree(c->pinned);
        delete c;
        return code;
    }
    *out = c;
    return DEC_OK;
}

int dec_destroy(dec_ctx* ctx) {
    if (!ctx) return DEC_EINVAL;
    if (ctx->live_children > 0) {
        ctx->last_error = "context still owns meshes or servers";
        return DEC_ESTATE;
    }
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return DEC_OK;
}

}  // extern "C"
