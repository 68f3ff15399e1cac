// Integer deposit from explicit lists without any device allocation: the staged input lists
// and the int64 edge and node sums live in one file-scope device array (kStaticScratchBytes on
// each GPU the library runs on, held until the process ends). Host code never passes the
// array's name to a kernel or a copy: it uses the address hipGetSymbolAddress gives for the
// current device, looked up once per device when a context is created on it.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "qh_internal.h"

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

__global__ void k_zero_i64(int64_t *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

size_t qh_static_scratch_bytes() { return kStaticScratchBytes; }

// Address of this device's copy of the array; the device must be current.
int qh_static_scratch_init(qh_ctx *c) {
    if (c->device < 0 || c->device >= kMaxDevices) return qh_fail(c, QH_EINVAL, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[c->device]) return QH_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return qh_fail(c, QH_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[c->device] = ptr;
    return QH_OK;
}

// Bytes of the array a call with these list sizes needs on this mesh: the edge and node sums,
// then the lists (tet, 4 + 4 coordinates and charge number per piece; tet, 4 coordinates and
// charge number per point).
size_t qh_static_deposit_bytes(int64_t ne, int64_t nn, int64_t n_seg, int64_t n_pt) {
    const size_t sums = (size_t)(ne + nn) * sizeof(int64_t);
    return sums + (size_t)(10 * n_seg + 6 * n_pt) * sizeof(int32_t);
}

int qh_static_deposit(qh_ctx *c, int64_t n_seg, const int32_t *seg_tet, const int32_t *lam0, const int32_t *lam1,
                      const int32_t *seg_z, int64_t n_pt, const int32_t *pt_tet, const int32_t *pt_lam,
                      const int32_t *pt_z, int64_t *g_out, int64_t *q_out) {
    void *base;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch[c->device];
    }
    if (!base) return qh_fail(c, QH_ESTATE, "static scratch not set up on this device");
    const HostMesh &m = c->hm;
    int64_t *gd = static_cast<int64_t *>(base), *qd = gd + m.Ne;
    int32_t *st = reinterpret_cast<int32_t *>(qd + m.Nn);
    int32_t *l0 = st + n_seg, *l1 = l0 + 4 * n_seg, *sz = l1 + 4 * n_seg;
    int32_t *pt = sz + n_seg, *pl = pt + n_pt, *pz = pl + 4 * n_pt;
    hipError_t e = hipSuccess;
    auto cp = [&](int32_t *dst, const int32_t *src, int64_t k) {
        if (k > 0 && e == hipSuccess) e = hipMemcpyAsync(dst, src, sizeof(int32_t) * k, hipMemcpyHostToDevice, c->stream);
    };
    cp(st, seg_tet, n_seg); cp(l0, lam0, 4 * n_seg); cp(l1, lam1, 4 * n_seg); cp(sz, seg_z, n_seg);
    cp(pt, pt_tet, n_pt); cp(pl, pt_lam, 4 * n_pt); cp(pz, pt_z, n_pt);
    // the sums start at zero (a fill kernel: the array keeps the previous call's contents)
    const int64_t nsum = m.Ne + m.Nn;
    if (e == hipSuccess && nsum > 0) {
        hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)std::min<int64_t>((nsum + 255) / 256, 4096)), dim3(256), 0,
                           c->stream, gd, nsum);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_deposit_lists(c, n_seg, st, l0, l1, sz, n_pt, pt, pl, pz, gd, qd);
    if (e == hipSuccess && g_out) e = hipMemcpyAsync(g_out, gd, sizeof(int64_t) * m.Ne, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && q_out) e = hipMemcpyAsync(q_out, qd, sizeof(int64_t) * m.Nn, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return qh_fail(c, QH_EHIP, std::string("deposit: ") + hipGetErrorString(e));
    return QH_OK;
}
