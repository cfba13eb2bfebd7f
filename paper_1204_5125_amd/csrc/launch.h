// Kernel steps as argument structs, launched either at once on a stream or
// recorded for a batched launch.
//
// A step is a struct A holding every argument of one dispatch, with
//   __device__ void operator()(int bx, int nbx) const
// run by each work-group (bx = its index among the nbx work-groups of this
// dispatch).  k_one runs one instance; k_many runs `count` instances of the
// same shape in one dispatch: grid (nbx, count), instance blockIdx.y reads
// its own argument struct.  Instances of one grid size have identical launch
// sequences (the hierarchy's shape depends only on the grid), so recording the
// sequence of each and zipping them gives the batched sequence.
#pragma once

#include <cstring>
#include <vector>

#include "common.h"

namespace glk {

// Both kernels inline the step body.  Left to itself the compiler inlines
// it into k_one but may call it out of line from k_many, with more
// registers and, where it contracts multiply-adds differently in the two
// copies, other rounding: a batch would then not equal the single solves.
template <class A, int BS>
__global__ __launch_bounds__(BS) void k_one(A a)
{
    [[clang::always_inline]] a(blockIdx.x, gridDim.x);
}

template <class A, int BS>
__global__ __launch_bounds__(BS) void k_many(const A *__restrict__ a)
{
    [[clang::always_inline]] a[blockIdx.y](blockIdx.x, gridDim.x);
}

// one recorded dispatch
struct Step {
    void (*many)(const void *dev_args, int nbx, int count, int lds, hipStream_t s);
    int nbx;
    int bs;
    int lds;  // dynamic LDS bytes
    std::vector<unsigned char> args;
};

template <class A, int BS>
void launch_many(const void *dev_args, int nbx, int count, int lds, hipStream_t s)
{
    k_many<A, BS><<<dim3(nbx, count), BS, lds, s>>>(static_cast<const A *>(dev_args));
}

struct Launch {
    hipStream_t s = nullptr;
    std::vector<Step> *rec = nullptr;  // non-null: record instead of launching

    template <class A, int BS = kBlock>
    void run(int nbx, const A &a, int lds = 0) const
    {
        if (nbx <= 0) return;
        if (rec) {
            Step st;
            st.many = &launch_many<A, BS>;
            st.nbx = nbx;
            st.bs = BS;
            st.lds = lds;
            st.args.resize(sizeof(A));
            std::memcpy(st.args.data(), &a, sizeof(A));
            rec->push_back(std::move(st));
            return;
        }
        k_one<A, BS><<<nbx, BS, lds, s>>>(a);
        GLK_CHECK_LAUNCH();
    }
};

// Event-bracketed launch of one selected kernel class (profiling); recording
// passes straight through.
template <class F>
void prof_launch(int id, double bytes, const Launch &L, F &&launch, int count = 1)
{
    if (L.rec) {
        launch();
        return;
    }
    prof_launch(id, bytes, L.s, launch, count);
}

}  // namespace glk
