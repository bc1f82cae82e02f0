// Pair-list views and per-pair Phase-A buffers shared by the collision rules.
#pragma once
#include "common.hpp"

namespace dsmc {

enum { RULE_DIR = 0, RULE_CHI = 1 };

struct PairsView {
    const int32_t* off;
    const int32_t* cnt;
    const int32_t* i;
    const int32_t* j;
    const int32_t* cell;
    int64_t cap;
    static PairsView of(const dsmc_pairs& p)
    {
        return PairsView{p.off, p.cnt, p.i, p.j, p.cell, p.cap};
    }
    // Accepted pairs in total (the list is dense and cell-major), never more
    // than the capacity.
    __device__ __forceinline__ int64_t total(int32_t n_cells) const
    {
        const int64_t t = (int64_t)off[n_cells - 1] + cnt[n_cells - 1];
        return t < cap ? t : cap;
    }
};

// Per-pair Phase-A results, SoA with stride cap+1:
//   RULE_DIR: (a, b, c) = unit direction u
//   RULE_CHI: (a, b) = (cos chi, sin chi), (c, d, e) = xi
template <typename T> struct PairBuf {
    static constexpr int kFields = 6;
    T *a, *b, *c, *d, *e, *f;
    static PairBuf of(void* base, int64_t cap)
    {
        T* p = static_cast<T*>(base);
        const int64_t s = cap + 1;
        return PairBuf{p, p + s, p + 2 * s, p + 3 * s, p + 4 * s, p + 5 * s};
    }
};

int phase_b(int rule, int dtype, int32_t n_cells, const int32_t* cell_start, dsmc_vec3 v,
            const dsmc_pairs& pairs, void* dirs, int64_t cap, int32_t schedule, hipStream_t s);

int check_pairs(const char* who, int32_t n_cells, dsmc_vec3 v, const dsmc_pairs& pairs,
                int32_t dtype, void* ws, size_t ws_bytes);

}  // namespace dsmc
