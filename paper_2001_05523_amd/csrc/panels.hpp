// Panel descriptors shared by every step of the H^2 product.
//
// Every step of the product is a set of small dense matrix-vector products
// whose matrices are stored as "row panels": for an output group g (a
// cluster), a dense row-major matrix of nrows x ncols whose columns are the
// concatenation of input segments x[seg_in .. seg_in + seg_len).
//
//   nearfield   group = row leaf t,     segments = nearfield column leaves s
//   coupling    group = row cluster t,  segments = x-hat of farfield columns s
//   leaf basis  group = leaf t,         one segment = x restricted to t   (V_t^T)
//   transfer    group = parent t,       segments = x-hat of the children  ([E_c0^T | E_c1^T])
//
// The transposed product of the same storage is described by "column panels":
// for an output segment (a cluster), the list of row-panel blocks that have
// it as an input segment, each with its column offset, row stride and input.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "h2b_internal.hpp"

namespace h2b {

// ------------------------------------------------------- device memory

// Device memory comes from the allocator installed with h2b_set_allocator
// (e.g. the caller's caching allocator), else from hipMalloc.  Each block
// remembers the allocator that produced it and returns to it.
struct DeviceAllocator {
    h2b_alloc_fn alloc = nullptr;  // NULL: hipMalloc / hipFree
    h2b_free_fn free = nullptr;
    void *ctx = nullptr;
};
DeviceAllocator current_allocator();
void set_allocator(const DeviceAllocator &a);
// Stream passed to the allocator for allocations made by the calling thread
// (the stream of the library call in progress).
hipStream_t alloc_stream();
struct AllocStreamScope {
    hipStream_t saved;
    explicit AllocStreamScope(hipStream_t st);
    ~AllocStreamScope();
};

struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DeviceAllocator a{};
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    DevMem(DevMem &&o) noexcept : p(o.p), bytes(o.bytes), a(o.a) { o.p = nullptr; o.bytes = 0; }
    DevMem &operator=(DevMem &&o) noexcept
    {
        release();
        p = o.p;
        bytes = o.bytes;
        a = o.a;
        o.p = nullptr;
        o.bytes = 0;
        return *this;
    }
    ~DevMem() { release(); }
    void release()
    {
        if (p) {
            if (a.free) {
                // work queued on any stream may still use the block; hipFree
                // waits for the device, and so does the return to the caller's
                // allocator, which may hand the block out again at once
                (void)hipDeviceSynchronize();
                a.free(p, alloc_stream(), a.ctx);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t n)
    {
        release();
        if (n == 0) n = 256;
        a = current_allocator();
        if (a.alloc) {
            p = a.alloc(n, alloc_stream(), a.ctx);
            if (!p) fail(H2B_ENOMEM, "the installed allocator returned NULL for " + std::to_string(n) + " bytes");
            if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
                a.free(p, alloc_stream(), a.ctx);
                p = nullptr;
                fail(H2B_EINVAL, "the installed allocator returned memory that is not 256-byte aligned");
            }
        } else if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(H2B_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
        }
        bytes = n;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

inline void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) fail(H2B_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Packs several host arrays into one device allocation (256-byte aligned).
struct Packer {
    std::vector<char> host;
    std::vector<std::pair<size_t, void **>> fixups;
    template <typename T> void add(const std::vector<T> &v, T **dst)
    {
        size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + v.size() * sizeof(T) + 8);
        if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
        fixups.push_back({off, reinterpret_cast<void **>(dst)});
    }
    void upload(DevMem &mem, hipStream_t st)
    {
        mem.alloc(host.size());
        hip_check(hipMemcpyAsync(mem.p, host.data(), host.size(), hipMemcpyHostToDevice, st),
                  "descriptor upload");
        hip_check(hipStreamSynchronize(st), "descriptor upload");
        for (auto &f : fixups) *f.second = static_cast<char *>(mem.p) + f.first;
    }
};

// -------------------------------------------------------------- panels

struct RowPanelDev {
    const int64_t *val_off;
    const int32_t *nrows, *ncols, *out_begin, *seg_ptr, *seg_in, *seg_len;
    const int32_t *seg_c0;         // column of each segment inside its group's panel
    const int32_t *tag, *seg_tag;  // cluster ids of groups and segments (assembly only)
};

struct ColPanelDev {
    const int32_t *out_begin, *out_len, *blk_ptr;
    const int64_t *b_val_off;
    const int32_t *b_stride, *b_c0, *b_nrows, *b_in;
};

struct RowPanels {
    std::vector<int64_t> val_off;
    std::vector<int32_t> nrows, ncols, out_begin, seg_ptr{0}, seg_in, seg_len;
    std::vector<int32_t> seg_c0;     // column of each segment inside its group's panel
    std::vector<int32_t> group_tag;  // cluster id of each group
    std::vector<int32_t> seg_tag;    // cluster id of each segment
    int64_t total = 0;               // number of stored values
    int max_ncols = 0, max_nrows = 0;
    RowPanelDev dev{};
    DevMem mem;

    int ngroups() const { return (int)nrows.size(); }
    // Appends a group; segments are appended with add_segment afterwards.
    void begin_group(int tag, int out, int rows)
    {
        group_tag.push_back(tag);
        out_begin.push_back(out);
        nrows.push_back(rows);
        ncols.push_back(0);
        val_off.push_back(0);
    }
    void add_segment(int in, int len, int tag)
    {
        seg_tag.push_back(tag);
        seg_in.push_back(in);
        seg_len.push_back(len);
        seg_c0.push_back(ncols.back());
        ncols.back() += len;
    }
    void end_group()
    {
        seg_ptr.push_back((int32_t)seg_in.size());
        val_off.back() = total;
        total += (int64_t)nrows.back() * ncols.back();
        max_ncols = std::max(max_ncols, ncols.back());
        max_nrows = std::max(max_nrows, nrows.back());
    }
    void upload(hipStream_t st)
    {
        Packer pk;
        pk.add(val_off, const_cast<int64_t **>(&dev.val_off));
        pk.add(nrows, const_cast<int32_t **>(&dev.nrows));
        pk.add(ncols, const_cast<int32_t **>(&dev.ncols));
        pk.add(out_begin, const_cast<int32_t **>(&dev.out_begin));
        pk.add(seg_ptr, const_cast<int32_t **>(&dev.seg_ptr));
        pk.add(seg_in, const_cast<int32_t **>(&dev.seg_in));
        pk.add(seg_len, const_cast<int32_t **>(&dev.seg_len));
        pk.add(seg_c0, const_cast<int32_t **>(&dev.seg_c0));
        pk.add(group_tag, const_cast<int32_t **>(&dev.tag));
        pk.add(seg_tag, const_cast<int32_t **>(&dev.seg_tag));
        pk.upload(mem, st);
    }
};

struct ColPanels {
    std::vector<int32_t> out_begin, out_len, blk_ptr{0};
    std::vector<int64_t> b_val_off;
    std::vector<int32_t> b_stride, b_c0, b_nrows, b_in;
    std::vector<int32_t> out_tag, b_tag;  // cluster ids of output groups and blocks (host only)
    int max_out = 0;
    ColPanelDev dev{};
    DevMem mem;

    int ngroups() const { return (int)out_len.size(); }
    void upload(hipStream_t st)
    {
        Packer pk;
        pk.add(out_begin, const_cast<int32_t **>(&dev.out_begin));
        pk.add(out_len, const_cast<int32_t **>(&dev.out_len));
        pk.add(blk_ptr, const_cast<int32_t **>(&dev.blk_ptr));
        pk.add(b_val_off, const_cast<int64_t **>(&dev.b_val_off));
        pk.add(b_stride, const_cast<int32_t **>(&dev.b_stride));
        pk.add(b_c0, const_cast<int32_t **>(&dev.b_c0));
        pk.add(b_nrows, const_cast<int32_t **>(&dev.b_nrows));
        pk.add(b_in, const_cast<int32_t **>(&dev.b_in));
        pk.upload(mem, st);
    }
};

// Column panels of the transposed product of groups [g0, g1) of rp: the output
// groups are the distinct input segments, in increasing order of their start.
void transpose_panels(const RowPanels &rp, int g0, int g1, ColPanels &cp);
// Row panels of the transposed matrix described by cp (= transpose_panels of
// some rp): one group per output group of cp, one segment per block, in cp's
// order, so that value (i, j) of block b of rp lands at (j, i) of segment b.
void regroup_transposed(const ColPanels &cp, RowPanels &out);

}  // namespace h2b
