// Gather-scatter setup on the device (the gs_setup of the NekRS paper,
// Sec. 3.2): from the global pointers g of every local copy build
//   mult[l]  number of copies of l's global node (1 for pointer 0),
//   perm     local indices of copies of nodes with 2+ copies, sorted by
//            (pointer, local index)  -- a stable radix sort of (g, l) pairs,
//   offs     start of each such node's run in perm (plus the total at the end),
//   W        counting weight 1/mult, 0 on Dirichlet copies (Sec. 3.4),
// and check that all copies of a node agree in coordinates and Dirichlet flag.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "sem_internal.h"

namespace semx {

__global__ void iota_kernel(int64_t n, int32_t *v)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) v[t] = (int32_t)t;
}

// per run: shared flag and the number of copies it contributes to perm
__global__ void run_flags_kernel(int64_t nruns, const int64_t *__restrict__ key,
                                 const int32_t *__restrict__ cnt, int32_t *__restrict__ flag,
                                 int32_t *__restrict__ ncopy)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns) return;
    const bool shared = key[r] != 0 && cnt[r] >= 2;
    flag[r] = shared ? 1 : 0;
    ncopy[r] = shared ? cnt[r] : 0;
}

__global__ void run_fill_kernel(int64_t nruns, const int64_t *__restrict__ key,
                                const int32_t *__restrict__ cnt, const int32_t *__restrict__ start,
                                const int32_t *__restrict__ segidx,
                                const int32_t *__restrict__ copyoff,
                                const int32_t *__restrict__ sorted_idx,
                                int32_t *__restrict__ perm, int32_t *__restrict__ offs,
                                int32_t *__restrict__ mult, const double *__restrict__ x,
                                const double *__restrict__ y, const double *__restrict__ z,
                                const uint8_t *__restrict__ dir, double tol, int *bad)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns) return;
    const int c = cnt[r], s0 = start[r];
    if (key[r] == 0) {
        for (int t = 0; t < c; ++t) mult[sorted_idx[s0 + t]] = 1;
        return;
    }
    for (int t = 0; t < c; ++t) mult[sorted_idx[s0 + t]] = c;
    if (c < 2) return;
    const int so = segidx[r], co = copyoff[r];
    offs[so] = co;
    const int l0 = sorted_idx[s0];
    for (int t = 0; t < c; ++t) {
        const int l = sorted_idx[s0 + t];
        perm[co + t] = l;
        if (x) {
            const double dx = fabs(x[l] - x[l0]), dy = fabs(y[l] - y[l0]), dz = fabs(z[l] - z[l0]);
            const double sc = 1.0 + fabs(x[l0]) + fabs(y[l0]) + fabs(z[l0]);
            if (dx > tol * sc || dy > tol * sc || dz > tol * sc) atomicOr(bad, 2);
        }
        if (dir && dir[l] != dir[l0]) atomicOr(bad, 4);
    }
}

__global__ void weights_kernel(int64_t nL, const int32_t *__restrict__ mult,
                               const uint8_t *__restrict__ dir, double *__restrict__ W,
                               float *__restrict__ W32)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nL) return;
    const double w = (dir && dir[l]) ? 0.0 : 1.0 / (double)mult[l];
    W[l] = w;
    if (W32) W32[l] = (float)w;
}

namespace {
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};
}  // namespace

int build_maps(Level &L, const int64_t *gid, const uint8_t *dir, const double *x, const double *y,
               const double *z, int *bad, hipStream_t s)
{
    const int64_t nL = L.nL;
    const int n = (int)nL;
    // highest set bit of the largest pointer bounds the radix passes
    int end_bit = 64;
    {
        DevBuf maxb, tmpb;
        size_t tb = 0;
        SEM_HIP(hipMalloc(&maxb.p, sizeof(int64_t)));
        SEM_HIP(hipcub::DeviceReduce::Max(nullptr, tb, gid, (int64_t *)maxb.p, n, s));
        SEM_HIP(hipMalloc(&tmpb.p, tb));
        SEM_HIP(hipcub::DeviceReduce::Max(tmpb.p, tb, gid, (int64_t *)maxb.p, n, s));
        int64_t gmax = 0;
        SEM_HIP(hipMemcpyAsync(&gmax, maxb.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SEM_HIP(hipStreamSynchronize(s));
        end_bit = 1;
        while (end_bit < 63 && (gmax >> end_bit) != 0) ++end_bit;
    }
    DevBuf kout, vin, vout, uniq, cnt, nr, start, flag, ncopy, segidx, copyoff, mult, tmp;
    SEM_HIP(hipMalloc(&kout.p, sizeof(int64_t) * nL));
    SEM_HIP(hipMalloc(&vin.p, sizeof(int32_t) * nL));
    SEM_HIP(hipMalloc(&vout.p, sizeof(int32_t) * nL));
    SEM_HIP(hipMalloc(&uniq.p, sizeof(int64_t) * nL));
    SEM_HIP(hipMalloc(&cnt.p, sizeof(int32_t) * nL));
    SEM_HIP(hipMalloc(&nr.p, sizeof(int64_t)));
    SEM_HIP(hipMalloc(&mult.p, sizeof(int32_t) * nL));
    const int bs = 256;
    const unsigned nbL = (unsigned)((nL + bs - 1) / bs);
    hipLaunchKernelGGL(iota_kernel, dim3(nbL), dim3(bs), 0, s, nL, (int32_t *)vin.p);
    SEM_HIP(hipGetLastError());

    size_t tb_sort = 0, tb_rle = 0, tb_scan = 0;
    SEM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb_sort, gid, (int64_t *)kout.p,
                                               (int32_t *)vin.p, (int32_t *)vout.p, n, 0, end_bit, s));
    SEM_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, tb_rle, (int64_t *)kout.p,
                                                  (int64_t *)uniq.p, (int32_t *)cnt.p,
                                                  (int64_t *)nr.p, n, s));
    SEM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb_scan, (int32_t *)cnt.p, (int32_t *)vin.p,
                                             n, s));
    const size_t tb = std::max(tb_sort, std::max(tb_rle, tb_scan));
    SEM_HIP(hipMalloc(&tmp.p, tb));
    size_t t1 = tb;
    SEM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, t1, gid, (int64_t *)kout.p, (int32_t *)vin.p,
                                               (int32_t *)vout.p, n, 0, end_bit, s));
    SEM_HIP(hipMemsetAsync(nr.p, 0, sizeof(int64_t), s));
    t1 = tb;
    SEM_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp.p, t1, (int64_t *)kout.p, (int64_t *)uniq.p,
                                                  (int32_t *)cnt.p, (int64_t *)nr.p, n, s));
    int64_t nruns = 0;
    SEM_HIP(hipMemcpyAsync(&nruns, nr.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    if (nruns < 1 || nruns > nL) {
        set_error("gs setup: run-length encoding returned %lld runs for %lld copies",
                  (long long)nruns, (long long)nL);
        return SEM_EHIP;
    }

    SEM_HIP(hipMalloc(&start.p, sizeof(int32_t) * (nruns + 1)));
    SEM_HIP(hipMalloc(&flag.p, sizeof(int32_t) * (nruns + 1)));
    SEM_HIP(hipMalloc(&ncopy.p, sizeof(int32_t) * (nruns + 1)));
    SEM_HIP(hipMalloc(&segidx.p, sizeof(int32_t) * (nruns + 1)));
    SEM_HIP(hipMalloc(&copyoff.p, sizeof(int32_t) * (nruns + 1)));
    const unsigned nbR = (unsigned)((nruns + bs - 1) / bs);
    t1 = tb;
    SEM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, t1, (int32_t *)cnt.p, (int32_t *)start.p,
                                             (int)nruns, s));
    hipLaunchKernelGGL(run_flags_kernel, dim3(nbR), dim3(bs), 0, s, nruns, (const int64_t *)uniq.p,
                       (const int32_t *)cnt.p, (int32_t *)flag.p, (int32_t *)ncopy.p);
    SEM_HIP(hipGetLastError());
    // scan nruns+1 entries so the last one holds the totals (pad with 0)
    SEM_HIP(hipMemsetAsync((int32_t *)flag.p + nruns, 0, sizeof(int32_t), s));
    SEM_HIP(hipMemsetAsync((int32_t *)ncopy.p + nruns, 0, sizeof(int32_t), s));
    t1 = tb;
    SEM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, t1, (int32_t *)flag.p, (int32_t *)segidx.p,
                                             (int)nruns + 1, s));
    t1 = tb;
    SEM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, t1, (int32_t *)ncopy.p, (int32_t *)copyoff.p,
                                             (int)nruns + 1, s));
    int32_t tot[2] = {0, 0};
    SEM_HIP(hipMemcpyAsync(&tot[0], (int32_t *)segidx.p + nruns, sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    SEM_HIP(hipMemcpyAsync(&tot[1], (int32_t *)copyoff.p + nruns, sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    L.nseg = tot[0];
    L.ncopies = tot[1];
    // unique nodes: distinct nonzero pointers + each pointer-0 copy
    {
        int64_t k0 = 0;
        int32_t c0 = 0;
        SEM_HIP(hipMemcpy(&k0, uniq.p, sizeof(int64_t), hipMemcpyDeviceToHost));
        SEM_HIP(hipMemcpy(&c0, cnt.p, sizeof(int32_t), hipMemcpyDeviceToHost));
        L.n_unique = (k0 == 0) ? (nruns - 1 + c0) : nruns;
    }
    SEM_HIP(hipMalloc(&L.perm, sizeof(int32_t) * (L.ncopies > 0 ? L.ncopies : 1)));
    SEM_HIP(hipMalloc(&L.offs, sizeof(int32_t) * (L.nseg + 1)));
    hipLaunchKernelGGL(run_fill_kernel, dim3(nbR), dim3(bs), 0, s, nruns, (const int64_t *)uniq.p,
                       (const int32_t *)cnt.p, (const int32_t *)start.p,
                       (const int32_t *)segidx.p, (const int32_t *)copyoff.p,
                       (const int32_t *)vout.p, L.perm, L.offs, (int32_t *)mult.p, x, y, z, dir,
                       1e-12, bad);
    SEM_HIP(hipGetLastError());
    const int32_t last = (int32_t)L.ncopies;
    SEM_HIP(hipMemcpyAsync(L.offs + L.nseg, &last, sizeof(int32_t), hipMemcpyHostToDevice, s));
    SEM_HIP(hipMalloc(&L.W, sizeof(double) * nL));
    SEM_HIP(hipMalloc(&L.W32, sizeof(float) * nL));
    hipLaunchKernelGGL(weights_kernel, dim3(nbL), dim3(bs), 0, s, nL, (const int32_t *)mult.p, dir,
                       L.W, L.W32);
    SEM_HIP(hipGetLastError());
    SEM_HIP(hipStreamSynchronize(s));
    return build_gs_chunks(L, s);
}

// Pack whole segments, in canonical order, into chunks of at most 64 copies
// (one wavefront each), and write each chunk's copy list padded to 64 lanes:
// chunk_perm[c][l] = copy l of the chunk, with kGsSegStart set where it
// starts a segment, -1 past the chunk's end.  Segments with more than 64
// copies go to an overflow list handled one thread per segment.  On the host:
// O(shared copies), setup only.
int build_gs_chunks(Level &L, hipStream_t s)
{
    if (L.nL >= (int64_t)kGsSegStart) {  // copy indices share their word with the flag
        set_error("setup: %lld local points exceed the gather-scatter limit of 2^30", (long long)L.nL);
        return SEM_EINVAL;
    }
    std::vector<int32_t> offs(L.nseg + 1);
    if (L.nseg > 0)
        SEM_HIP(hipMemcpy(offs.data(), L.offs, sizeof(int32_t) * (L.nseg + 1), hipMemcpyDeviceToHost));
    else
        offs[0] = 0;
    std::vector<int32_t> perm(L.ncopies);
    if (L.ncopies > 0)
        SEM_HIP(hipMemcpy(perm.data(), L.perm, sizeof(int32_t) * L.ncopies, hipMemcpyDeviceToHost));
    std::vector<int32_t> cp;  // padded chunk lists
    std::vector<int32_t> over;
    int32_t used = 64;  // lanes filled in the open chunk (64: none open)
    for (int64_t q = 0; q < L.nseg; ++q) {
        const int32_t a = offs[q], len = offs[q + 1] - offs[q];
        if (len > 64) {
            over.push_back((int32_t)q);
            continue;
        }
        if (used + len > 64) {  // open a new chunk
            cp.resize(cp.size() + 64, -1);
            used = 0;
        }
        int32_t *lanes = cp.data() + cp.size() - 64;
        for (int32_t o = 0; o < len; ++o) lanes[used + o] = perm[a + o] | (o == 0 ? kGsSegStart : 0);
        used += len;
    }
    const int64_t nch = (int64_t)cp.size() / 64;
    L.nchunks = nch;
    L.nover = (int64_t)over.size();
    if (nch > 0) {
        SEM_HIP(hipMalloc(&L.chunk_perm, sizeof(int32_t) * cp.size()));
        SEM_HIP(hipMemcpy(L.chunk_perm, cp.data(), sizeof(int32_t) * cp.size(), hipMemcpyHostToDevice));
    }
    if (L.nover > 0) {
        SEM_HIP(hipMalloc(&L.over, sizeof(int32_t) * L.nover));
        SEM_HIP(hipMemcpy(L.over, over.data(), sizeof(int32_t) * L.nover, hipMemcpyHostToDevice));
    }
    (void)s;
    return SEM_OK;
}

}  // namespace semx
