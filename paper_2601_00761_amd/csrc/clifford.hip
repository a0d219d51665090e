// Random brick-wall Clifford circuits for preconditioning (Clifford preconditioning
// section): the two-qubit Clifford group modulo phase, and the gate list of n_layers
// brick-wall layers with each gate drawn uniformly from it.  Host code only; the
// gates are applied by the dense two-qubit gate kernel.
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "philox.h"

namespace pw {
namespace {

using C = std::complex<double>;
using M4 = std::array<C, 16>;  // row-major, local index b_{q0} + 2 b_{q1}

M4 mul(const M4& a, const M4& b) {
    M4 r{};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            C s = 0;
            for (int k = 0; k < 4; ++k) s += a[4 * i + k] * b[4 * k + j];
            r[4 * i + j] = s;
        }
    return r;
}

// Representative of the phase class: the first entry of magnitude > 1e-9 made real
// positive.  Key: entries on a 2^-24 grid.
M4 canonical(const M4& a) {
    C ph = 1;
    for (const C& v : a)
        if (std::abs(v) > 1e-9) {
            ph = std::conj(v) / std::abs(v);
            break;
        }
    M4 r;
    for (int i = 0; i < 16; ++i) r[i] = a[i] * ph;
    return r;
}

std::array<long long, 32> key_of(const M4& a) {
    std::array<long long, 32> k;
    for (int i = 0; i < 16; ++i) {
        k[2 * i] = std::llround(a[i].real() * 16777216.0);
        k[2 * i + 1] = std::llround(a[i].imag() * 16777216.0);
    }
    return k;
}

// Generators on (q0, q1): H and S on either qubit, CNOT either way.
std::vector<M4> generators() {
    const double h = 1.0 / std::sqrt(2.0);
    const C H[4] = {h, h, h, -h};
    const C S[4] = {1, 0, 0, C(0, 1)};
    std::vector<M4> g;
    for (int q = 0; q < 2; ++q)
        for (const C* u : {H, S}) {
            M4 m{};
            for (int o = 0; o < 4; ++o)
                for (int i = 0; i < 4; ++i) {
                    const int ob = (o >> q) & 1, ib = (i >> q) & 1;
                    const bool other_same = ((o >> (1 - q)) & 1) == ((i >> (1 - q)) & 1);
                    m[4 * o + i] = other_same ? u[2 * ob + ib] : C(0);
                }
            g.push_back(m);
        }
    for (int ctl = 0; ctl < 2; ++ctl) {
        M4 m{};
        for (int i = 0; i < 4; ++i) {
            const int o = ((i >> ctl) & 1) ? (i ^ (1 << (1 - ctl))) : i;
            m[4 * o + i] = 1;
        }
        g.push_back(m);
    }
    return g;
}

struct Table {
    std::vector<M4> mats;
};

const Table& table() {
    static Table t;
    static std::once_flag once;
    std::call_once(once, [] {
        const std::vector<M4> gen = generators();
        std::map<std::array<long long, 32>, int> seen;
        M4 id{};
        for (int i = 0; i < 4; ++i) id[5 * i] = 1;
        t.mats.push_back(id);
        seen[key_of(id)] = 0;
        for (size_t head = 0; head < t.mats.size(); ++head)
            for (const M4& g : gen) {
                const M4 m = canonical(mul(g, t.mats[head]));
                const auto k = key_of(m);
                if (seen.count(k)) continue;
                seen[k] = (int)t.mats.size();
                t.mats.push_back(m);
            }
    });
    return t;
}

}  // namespace

int clifford2_count() { return (int)table().mats.size(); }

void clifford2_matrix(int i, double* m32) {
    const M4& m = table().mats[(size_t)i];
    for (int k = 0; k < 16; ++k) {
        m32[2 * k] = m[k].real();
        m32[2 * k + 1] = m[k].imag();
    }
}

// Layer l pairs (i, i+1) for i = l mod 2, l mod 2 + 2, ...; periodic for even n (odd
// layers include (n-1, 0), every layer has n/2 gates), open for odd n.  Gate g of the
// list takes table index floor(W 11520 / 2^64), W the first 64-bit word of
// Philox4x32-10 with counter (g, 0, stream "CLIF") and key seed.
void brickwall_clifford(int n, int n_layers, uint64_t seed, std::vector<int>& q, std::vector<int>& idx,
                        std::vector<int>* layer_start) {
    q.clear();
    idx.clear();
    if (layer_start) layer_start->clear();
    const uint64_t order = (uint64_t)clifford2_count();
    uint64_t g = 0;
    for (int l = 0; l < n_layers; ++l) {
        const int start = l & 1;
        std::vector<std::pair<int, int>> pairs;
        if (n % 2 == 0) {
            for (int i = start; i < start + n; i += 2) pairs.push_back({i % n, (i + 1) % n});
        } else {
            for (int i = start; i + 1 < n; i += 2) pairs.push_back({i, i + 1});
        }
        if (layer_start) layer_start->push_back((int)idx.size());
        for (const auto& p : pairs) {
            uint64_t W0, W1;
            philox_words(seed, g++, 0u, STREAM_CLIF, W0, W1);
            q.push_back(p.first);
            q.push_back(p.second);
            idx.push_back((int)(((unsigned __int128)W0 * order) >> 64));
        }
    }
}

}  // namespace pw
