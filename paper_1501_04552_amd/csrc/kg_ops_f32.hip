// kg_ops_f32.hip -- kernel launchers of the FP32 path for every grid size.
#include "kg_plan.hpp"

namespace kg {

namespace {

template <int W>
std::unique_ptr<Ops> make(int n)
{
    switch (n) {
    case 8: return std::make_unique<OpsImpl<float, 8, W>>();
    case 16: return std::make_unique<OpsImpl<float, 16, W>>();
    case 24: return std::make_unique<OpsImpl<float, 24, W>>();
    case 32: return std::make_unique<OpsImpl<float, 32, W>>();
    case 48: return std::make_unique<OpsImpl<float, 48, W>>();
    case 64: return std::make_unique<OpsImpl<float, 64, W>>();
    case 96: return std::make_unique<OpsImpl<float, 96, W>>();
    case 128: return std::make_unique<OpsImpl<float, 128, W>>();
    case 192: return std::make_unique<OpsImpl<float, 192, W>>();
    case 256: return std::make_unique<OpsImpl<float, 256, W>>();
    case 384: return std::make_unique<OpsImpl<float, 384, W>>();
    case 512: return std::make_unique<OpsImpl<float, 512, W>>();
    default: return nullptr;
    }
}

}  // namespace

std::unique_ptr<Ops> make_ops_f32(int n, int W)
{
    return W == 8 ? make<8>(n) : make<16>(n);
}

}  // namespace kg
