// The second tile variant of the right-hand-side kernel (Tile<N, 1>): the
// three launches of the FP64 step and the two of the precision form that
// differ from them (FP32 R1), compiled apart from kernels.hip so that the
// two sets of instantiations build in parallel.
#include "rhs_kernel.h"

namespace numa {

namespace {

template <typename F>
hipError_t for_order(int N, F &&f)
{
    switch (N) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t rhs_launch_alt(numa_ctx *c, const RhsParams &p, int epi, bool mixed)
{
    return for_order(c->N, [&](auto n) -> hipError_t {
        constexpr int NN = decltype(n)::value;
        if (epi == EPI_R)
            return mixed ? rhs_launch_t<NN, 1, EPI_R, false, true>(c, p) : rhs_launch_t<NN, 1, EPI_R, false, false>(c, p);
        if (epi == EPI_TWO)
            return mixed ? rhs_launch_t<NN, 1, EPI_TWO, true, true>(c, p) : rhs_launch_t<NN, 1, EPI_TWO, true, false>(c, p);
        return rhs_launch_t<NN, 1, EPI_FINAL, false, false>(c, p);
    });
}

hipError_t rhs_prepare_alt(const numa_ctx *c, int zc, bool mixed)
{
    return for_order(c->N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        return mixed ? rhs_prepare_step<NN, 1, true>(c, zc) : rhs_prepare_step<NN, 1, false>(c, zc);
    });
}

size_t rhs_lds_alt(int N, int zc, int nez)
{
    size_t b = 0;
    (void)for_order(N, [&](auto n) {
        b = rhs_lds_bytes<decltype(n)::value, 1>(zc, nez);
        return hipSuccess;
    });
    return b;
}

bool rhs_alt_differs(int N)
{
    bool d = false;
    (void)for_order(N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        d = Tile<NN, 1>::TX != Tile<NN, 0>::TX || Tile<NN, 1>::TY != Tile<NN, 0>::TY;
        return hipSuccess;
    });
    return d;
}

}  // namespace numa
