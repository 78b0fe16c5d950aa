// tree.hpp -- the pairwise tree of FP64 partial sums that fixes the order of
// every real-valued readout sum (cut, Eq. 1, Eq. 2 and Eq. 6 energies).
//
// The tree over a sequence v_0, v_1, ... pads it with zeros to a power of
// two and adds adjacent pairs level by level, the lower-indexed partial on
// the left.  TreeAcc builds the same tree incrementally, one value at a time
// in sequence order (a binary counter: slot L holds a completed subtree of
// 2^L values waiting for its right sibling), so a thread can fold in block
// sums as it produces them; finish() pairs every waiting subtree with the
// zero padding on its right, which leaves it unchanged.  No partial sum is
// ever -0 (sums start from +0 and x + (-x) rounds to +0), so adding the
// padding zeros is exact.
#pragma once
#include <hip/hip_runtime.h>

namespace oim {

template <int Levels>
struct TreeAccN {
    static constexpr int kLevels = Levels;  // up to 2^Levels values
    double* slot;                           // kLevels doubles (LDS or global), owned by the caller
    unsigned long long full = 0;            // bit L set: slot[L] holds a subtree

    __device__ explicit TreeAccN(double* storage) : slot(storage) {}

    __device__ void push(double v) {
        int L = 0;
        while (full & (1ull << L)) {
            v = slot[L] + v;
            full &= ~(1ull << L);
            ++L;
        }
        slot[L] = v;
        full |= 1ull << L;
    }

    __device__ double finish() const {
        bool any = false;
        double carry = 0.0;
        for (int L = 0; L < kLevels; ++L) {
            if (!(full & (1ull << L))) continue;
            carry = any ? slot[L] + carry : slot[L];
            any = true;
        }
        return carry;
    }
};

using TreeAcc = TreeAccN<32>;

}  // namespace oim
