// Host-side reaction network: parsing, validation and the derived tables the
// device kernels read.  No HIP calls here except in DeviceNet::upload.
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

namespace abdf {

constexpr int kTwoBody = 0;
constexpr int kCosmicRay = 1;
constexpr int kPhoto = 2;
constexpr int kCrPhoton = 3;   // photoreaction by cosmic-ray-induced photons
constexpr int kRhsSegment = 32;   // right-hand-side entries summed by one lane before the species' lanes combine
constexpr int kRhsResidentGroups = 16;   // lane groups the streaming right-hand side holds in registers
constexpr int kRhsResidentLen = 40;      // the longest lane it holds

// Device copies of the network tables (one per HIP device).
struct DeviceNet {
    int device = -1;
    int S = 0, R = 0, NP = 0;
    double albedo = 0.0;           // dust albedo of the cosmic-ray-induced photon rate
    // per reaction
    int32_t *rx_ab = nullptr;      // reactant a in low 16 bits, b in high 16 bits (0xffff: none)
    int32_t *rx_type = nullptr;
    double *alpha = nullptr, *beta = nullptr, *gamma = nullptr;
    // right-hand side f_i = sum_r nu_ir rate_r in the layout of a wave: species
    // i's nonzero entries (reactions ascending) are split over m_i =
    // min(64, ceil(n_i / segment)) consecutive lanes of one group of 64
    // lanes (at least one lane per species); entry j of the lanes of group g
    // sits at sg_ent[sg_base[g] + 64 j + lane], so a wave's loads of entry j
    // are adjacent.  A lane sums its entries in order, then the lanes of a
    // species are added pairwise (lane 2t takes lane 2t+1, then 4t takes
    // 4t+2, ...) and the species' first lane holds f_i.
    // Lanes hold up to kRhsSegment entries, or up to kRhsResidentLen when that
    // brings the groups down to kRhsResidentGroups.
    int32_t n_sgroup = 0;
    int32_t sg_maxlen = 0;         // longest lane of any group
    int32_t *sg_base = nullptr;    // [n_sgroup] first entry of the group
    int32_t *sg_len = nullptr;     // [n_sgroup] longest lane | pairwise steps (ceil log2 of the widest species) << 24
    int32_t *sg_lane = nullptr;    // [64 n_sgroup] entries of the lane
    int32_t *sg_red = nullptr;     // [64 n_sgroup] species << 14 | lane within the species << 7 | m_i; -1 unused
    int32_t *sg_ent = nullptr;     // packed entries reaction << 3 | (nu + 4); 4 (coefficient 0) in the padding
    // Jacobian: nonzeros of J grouped by row, each with its list of terms
    int32_t *jrow_ptr = nullptr;   // [S+1]
    int32_t *jcol = nullptr;       // [nnzJ]
    int32_t *jrow = nullptr;       // [nnzJ] row of each nonzero
    int32_t *jterm_ptr = nullptr;  // [nnzJ+1]
    int32_t *jt_rx_other = nullptr;  // reaction << 16 | (other species + 1), 0 in the low half = none
    double *jt_coef = nullptr;     // [nterm] nu_ir * multiplicity
    int32_t nnzJ = 0, nterm = 0;
    // reaction-major stoichiometry: the species of reaction r with nu != 0
    int32_t *rnu_ptr = nullptr;    // [R+1]
    int32_t *rnu_ent = nullptr;    // species << 3 | (nu + 4)
    // d rate_r / d x_j grouped by species j: reaction << 16 | (other reactant + 1), multiplicity
    int32_t *dcol_ptr = nullptr;   // [S+1]
    int32_t *dcol_ent = nullptr;
    double *dcol_coef = nullptr;
    // dense map (i, j) -> index of the Jacobian nonzero, -1 where J_ij = 0 structurally [NP][NP]
    int32_t *jidx = nullptr;
    // the same map in 64-column words: bit c of jmask[i][b] is set when J has a
    // nonzero at (i, 64 b + c); jbase[i][b] is the index of the row's first
    // nonzero at or after column 64 b (nonzeros are numbered row by row, columns
    // ascending), so the index of (i, j) is jbase + the set bits below j
    int32_t nbw = 0;               // words per row, ceil(NP / 64)
    uint64_t *jmask = nullptr;     // [NP][nbw]
    int32_t *jbase = nullptr;      // [NP][nbw]
};

struct HostNetwork {
    std::string name;
    double albedo = 0.0;                  // dust grain albedo (optional "albedo" line), in [0, 1)
    std::vector<std::string> elements;
    std::vector<std::string> species;
    std::vector<int32_t> charge;          // [S]
    std::vector<int32_t> comp;            // [S * E]
    std::vector<int32_t> rtype;           // [R]
    std::vector<int32_t> react;           // [R * 2], -1 padded
    std::vector<int32_t> prod;            // [R * 3], -1 padded
    std::vector<double> alpha, beta, gamma;

    // derived (built by finalize())
    int S = 0, R = 0, E = 0, NP = 0;
    std::vector<int32_t> sg_base, sg_len, sg_lane, sg_red, sg_ent;
    std::vector<int32_t> jrow_ptr, jcol, jrow, jterm_ptr, jt_rx_other;
    std::vector<double> jt_coef;
    std::vector<int32_t> rnu_ptr, rnu_ent, dcol_ptr, dcol_ent, jidx, jbase;
    std::vector<uint64_t> jmask;
    std::vector<double> dcol_coef;

    // per-device uploads, created on first use
    mutable std::mutex mu;
    mutable std::vector<DeviceNet *> dev;
    // one solver workspace per device kept between calls (the largest returned)
    struct Block { void *ptr = nullptr; size_t bytes = 0; };
    mutable std::vector<Block> spare;

    ~HostNetwork();
    // Parses the text format; on failure returns an abdf_status code and sets err.
    int parse(const char *text, size_t len, std::string &err);
    // Builds the gather tables; called by parse.
    void finalize();
    // Device tables for the current HIP device (uploaded once); nullptr + err on failure.
    const DeviceNet *device_tables(std::string &err) const;
    // The tables of device devid if already uploaded, else nullptr (uploads nothing).
    const DeviceNet *device_tables_present(int devid) const;
    // A cached workspace of at least `bytes` on device devid (removed from the
    // cache; its size in *got), or nullptr (a smaller cached one is freed).
    void *take_workspace(int devid, size_t bytes, size_t *got) const;
    // Returns a workspace to the cache, which keeps the larger of it and the
    // one it holds and frees the other.
    void keep_workspace(int devid, void *ptr, size_t bytes) const;
    // Bytes cached on device devid.
    size_t cached_workspace_bytes(int devid) const;
};

}  // namespace abdf
