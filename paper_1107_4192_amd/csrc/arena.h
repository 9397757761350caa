// Device memory arena: one hipMalloc up front, then best-fit sub-allocation with
// coalescing on release. The serving loop gives every admitted job's plan its
// buffers from one arena sized to the HBM budget, so admission is exact and a
// finished job returns its memory without a device-wide free.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <unordered_map>

namespace kfmeg {

class DeviceArena {
public:
    static constexpr size_t kAlign = 256;

    hipError_t init(size_t bytes) {
        size_ = bytes / kAlign * kAlign;
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, size_);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            size_ = 0;
            return e;
        }
        base_ = static_cast<char*>(p);
        free_.clear();
        free_[0] = size_;
        return hipSuccess;
    }

    ~DeviceArena() {
        if (base_) (void)hipFree(base_);
    }

    // Best fit; nullptr when no free block is large enough.
    void* alloc(size_t bytes) {
        if (bytes == 0) bytes = 1;
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        std::lock_guard<std::mutex> lk(mu_);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return nullptr;
        const size_t off = best->first, len = best->second;
        free_.erase(best);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        in_use_ += bytes;
        if (in_use_ > peak_) peak_ = in_use_;
        return base_ + off;
    }

    void release(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        const size_t off = static_cast<size_t>(static_cast<char*>(p) - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        in_use_ -= len;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {   // merge with the following block
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {                                // merge with the preceding block
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }

    bool owns(const void* p) const {
        const char* c = static_cast<const char*>(p);
        return base_ && c >= base_ && c < base_ + size_;
    }
    size_t capacity() const { return size_; }
    size_t in_use() {
        std::lock_guard<std::mutex> lk(mu_);
        return in_use_;
    }
    size_t peak() {
        std::lock_guard<std::mutex> lk(mu_);
        return peak_;
    }
    size_t largest_free() {
        std::lock_guard<std::mutex> lk(mu_);
        size_t m = 0;
        for (auto& kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

private:
    char* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;            // offset -> length
    std::unordered_map<size_t, size_t> used_;  // offset -> length
    std::mutex mu_;
    size_t in_use_ = 0, peak_ = 0;
};

}  // namespace kfmeg
