// Ownership rules of libsymba's context memory that graph capture relies on,
// as plain C++ with no HIP dependency (unit-tested on the host).
//
// A call captured into a HIP graph records pointers: its kernels' arguments
// and the source and destination of every copy.  A replay must find those
// bytes unchanged, whatever eager calls ran on the context in between.  So:
//   * descriptors uploaded under capture are placed in a capture arena that
//     is only ever appended to: no two captured calls share bytes, and no
//     byte is rewritten or freed before the context is destroyed;
//   * the partial-sum buffer is never freed while a captured call may use it:
//     once a capture has referenced it, growing it retires it (kept until the
//     context is destroyed) instead of freeing it, and growing it under
//     capture is refused (nothing may be allocated then).
#pragma once

#include <cstddef>

namespace symba {

// Append-only allocator over a fixed capacity: every allocation gets bytes
// that no earlier allocation had, aligned to `align` (a power of two).
class BumpArena {
public:
    explicit BumpArena(size_t capacity = 0) : cap_(capacity), used_(0) {}
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    // Offset of a fresh block of `bytes` bytes, or false when it does not fit.
    bool alloc(size_t bytes, size_t align, size_t &offset) {
        if (align == 0 || (align & (align - 1)) != 0) return false;
        const size_t start = (used_ + align - 1) & ~(align - 1);
        if (start < used_ || start > cap_ || bytes > cap_ - start) return false;
        offset = start;
        used_ = start + bytes;
        return true;
    }

private:
    size_t cap_, used_;
};

// What to do with the partial-sum buffer before a call that needs `need`
// bytes, given its current size, whether a captured call has referenced it,
// and whether this call is being captured.
struct PartialAction {
    enum Kind { Keep, Grow, Refuse } kind;
    size_t new_bytes;  // Grow: the size to allocate
    bool retire_old;   // Grow: keep the old buffer alive until destroy (a capture references it)
};

inline PartialAction plan_partial(size_t current, size_t need, bool referenced_by_capture, bool capturing) {
    if (need <= current) return {PartialAction::Keep, current, false};
    if (capturing) return {PartialAction::Refuse, current, false};
    // grow geometrically, so that a run of growing calls retires at most
    // about as many bytes as it finally holds
    size_t grown = current + current / 2;
    if (grown < need) grown = need;
    return {PartialAction::Grow, grown, referenced_by_capture && current > 0};
}

}  // namespace symba
