// Search-difficulty analysis of a measured tune space (section V.B): the
// fitness flow graph (FFG) and the proportion of PageRank centrality.
//
// Nodes are the measured configurations.  Two configurations are neighbours
// when they differ in exactly one tunable.  The FFG has a directed edge from
// a configuration to every neighbour with strictly better fitness (lower time
// or energy); a random walk on it mimics a randomised first-improvement local
// search, and local minima (no better neighbour) are where it stops.  With
// PageRank on the FFG (damping d, teleportation to a uniform node, the rank of
// nodes without out-edges redistributed uniformly), the proportion of
// centrality for a factor p is the PageRank mass of the minima whose fitness is
// within p * f_opt divided by the mass of all minima.
#include <cmath>
#include <unordered_map>
#include <vector>

#include "gt_internal.hpp"

using namespace gt;

namespace {

uint64_t key_of(const gt_conv_config &c, int skip) {
    const int32_t v[6] = {c.block_size_x, c.block_size_y, c.tile_size_x, c.tile_size_y, c.use_lds_padding, c.read_path};
    uint64_t h = 1469598103934665603ull ^ (uint64_t)skip;
    for (int k = 0; k < 6; ++k) {
        if (k == skip) continue;
        h = (h ^ (uint64_t)(uint32_t)v[k]) * 1099511628211ull;
        h = (h ^ (uint64_t)k) * 1099511628211ull;
    }
    return h;
}

bool same_except(const gt_conv_config &a, const gt_conv_config &b, int skip) {
    const int32_t va[6] = {a.block_size_x, a.block_size_y, a.tile_size_x, a.tile_size_y, a.use_lds_padding, a.read_path};
    const int32_t vb[6] = {b.block_size_x, b.block_size_y, b.tile_size_x, b.tile_size_y, b.use_lds_padding, b.read_path};
    for (int k = 0; k < 6; ++k)
        if (k != skip && va[k] != vb[k]) return false;
    return va[skip] != vb[skip];
}

}  // namespace

extern "C" int gt_ffg_centrality(const gt_conv_config *cfgs, const double *fitness, size_t n, double damping,
                                 const double *p_values, size_t n_p, double *pagerank, int32_t *is_minimum,
                                 double *proportion) {
    clear_error();
    if (!cfgs || !fitness || !n || !(damping >= 0 && damping < 1) || (n_p && (!p_values || !proportion)))
        return set_error(GT_E_INVAL, "gt_ffg_centrality: bad argument");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(fitness[i])) return set_error(GT_E_INVAL, "gt_ffg_centrality: fitness %zu not finite", i);
    // neighbour lists: bucket configurations by all fields but one
    std::vector<std::vector<int32_t>> better(n);
    for (int skip = 0; skip < 6; ++skip) {
        std::unordered_map<uint64_t, std::vector<int32_t>> groups;
        for (size_t i = 0; i < n; ++i) groups[key_of(cfgs[i], skip)].push_back((int32_t)i);
        for (auto &g : groups) {
            const std::vector<int32_t> &m = g.second;
            for (size_t a = 0; a < m.size(); ++a)
                for (size_t b = 0; b < m.size(); ++b) {
                    const int32_t u = m[a], v = m[b];
                    if (u != v && same_except(cfgs[u], cfgs[v], skip) && fitness[v] < fitness[u])
                        better[u].push_back(v);
                }
        }
    }
    // PageRank by power iteration
    std::vector<double> pr(n, 1.0 / n), nx(n);
    for (int it = 0; it < 10000; ++it) {
        double dangling = 0;
        for (size_t u = 0; u < n; ++u)
            if (better[u].empty()) dangling += pr[u];
        const double base = (1.0 - damping) / n + damping * dangling / n;
        for (size_t v = 0; v < n; ++v) nx[v] = base;
        for (size_t u = 0; u < n; ++u)
            if (!better[u].empty()) {
                const double share = damping * pr[u] / better[u].size();
                for (int32_t v : better[u]) nx[v] += share;
            }
        double diff = 0;
        for (size_t v = 0; v < n; ++v) diff += std::fabs(nx[v] - pr[v]);
        pr.swap(nx);
        if (diff < 1e-15) break;
    }
    double f_opt = fitness[0];
    for (size_t i = 1; i < n; ++i) f_opt = std::min(f_opt, fitness[i]);
    double mass_min = 0;
    for (size_t i = 0; i < n; ++i) {
        if (pagerank) pagerank[i] = pr[i];
        if (is_minimum) is_minimum[i] = better[i].empty() ? 1 : 0;
        if (better[i].empty()) mass_min += pr[i];
    }
    for (size_t k = 0; k < n_p; ++k) {
        double good = 0;
        for (size_t i = 0; i < n; ++i)
            if (better[i].empty() && fitness[i] <= p_values[k] * f_opt) good += pr[i];
        proportion[k] = mass_min > 0 ? good / mass_min : NAN;
    }
    return GT_OK;
}
