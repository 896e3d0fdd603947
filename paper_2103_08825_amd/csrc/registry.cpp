// registry.cpp -- process-wide table of compiled fused-kernel launchers.
#include "registry.hpp"

#include <map>
#include <mutex>
#include <tuple>

namespace stn {
namespace {

using Key = std::tuple<int, int, int, int, int, int, int>;

std::mutex &reg_mutex() {
    static std::mutex m;
    return m;
}
struct Entry {
    SweepLauncher fn;
    OccupancyFn occ;
};
std::map<Key, Entry> &reg_map() {
    static std::map<Key, Entry> m;
    return m;
}
Key tup(const KernelKey &k) { return Key(k.dtype, k.dim, k.r, k.box, k.variant, k.k, k.mode); }

}  // namespace

void register_launcher(const KernelKey &key, SweepLauncher fn, OccupancyFn occ) {
    std::lock_guard<std::mutex> g(reg_mutex());
    reg_map()[tup(key)] = Entry{fn, occ};
}

SweepLauncher find_launcher(const KernelKey &key) {
    std::lock_guard<std::mutex> g(reg_mutex());
    auto it = reg_map().find(tup(key));
    return it == reg_map().end() ? nullptr : it->second.fn;
}

int resident_blocks(const KernelKey &key) {
    OccupancyFn occ = nullptr;
    {
        std::lock_guard<std::mutex> g(reg_mutex());
        auto it = reg_map().find(tup(key));
        if (it != reg_map().end()) occ = it->second.occ;
    }
    if (!occ) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus * occ();
}

int registered_max_k(int dtype, int dim, int r, int box, int variant, int mode) {
    std::lock_guard<std::mutex> g(reg_mutex());
    int best = 0;
    for (const auto &kv : reg_map()) {
        const Key &k = kv.first;
        if (std::get<0>(k) == dtype && std::get<1>(k) == dim && std::get<2>(k) == r &&
            std::get<3>(k) == box && std::get<4>(k) == variant && std::get<6>(k) == mode &&
            std::get<5>(k) > best)
            best = std::get<5>(k);
    }
    return best;
}

int registered_keys(KernelKey *out, int cap) {
    std::lock_guard<std::mutex> g(reg_mutex());
    int n = 0;
    for (const auto &kv : reg_map()) {
        if (out && n < cap) {
            const Key &k = kv.first;
            out[n] = KernelKey{std::get<0>(k), std::get<1>(k), std::get<2>(k),
                               std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k)};
        }
        ++n;
    }
    return n;
}

}  // namespace stn
