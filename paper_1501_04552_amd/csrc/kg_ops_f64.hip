// kg_ops_f64.hip -- kernel launchers of the FP64 path for every grid size.
#include "kg_plan.hpp"

namespace kg {

namespace {

template <int W>
std::unique_ptr<Ops> make(int n)
{
    switch (n) {
    case 8: return std::make_unique<OpsImpl<double, 8, W>>();
    case 16: return std::make_unique<OpsImpl<double, 16, W>>();
    case 24: return std::make_unique<OpsImpl<double, 24, W>>();
    case 32: return std::make_unique<OpsImpl<double, 32, W>>();
    case 48: return std::make_unique<OpsImpl<double, 48, W>>();
    case 64: return std::make_unique<OpsImpl<double, 64, W>>();
    case 96: return std::make_unique<OpsImpl<double, 96, W>>();
    case 128: return std::make_unique<OpsImpl<double, 128, W>>();
    case 192: return std::make_unique<OpsImpl<double, 192, W>>();
    case 256: return std::make_unique<OpsImpl<double, 256, W>>();
    case 384: return std::make_unique<OpsImpl<double, 384, W>>();
    case 512: return std::make_unique<OpsImpl<double, 512, W>>();
    default: return nullptr;
    }
}

}  // namespace

std::unique_ptr<Ops> make_ops_f64(int n, int W)
{
    return W == 4 ? make<4>(n) : make<8>(n);
}

}  // namespace kg
