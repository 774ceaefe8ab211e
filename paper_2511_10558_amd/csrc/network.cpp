// Network text parser, integer conservation check and gather-table builder.
//
// The tables restate the mass-action model of the paper (Sec. 2): the
// stoichiometric (incidence) matrix nu_ir = (count of i among products) -
// (count of i among reactants), the right-hand side f_i = sum_r nu_ir rate_r
// and its Jacobian J_ij = sum_r nu_ir d rate_r / d x_j.
#include "network.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <sstream>

#include "../../include/astrobdf.h"

namespace abdf {

namespace {

// Orders the entries of each lane of a group (the lane's sum runs in this
// order) so that the rates the lanes read at the same step fall in different
// LDS banks where the entries allow.  Lanes are taken sixteen at a time (at
// 128 bytes a clock, a 64-lane read of doubles is served sixteen lanes at a
// time) and a rate's bank is its index mod 16 (two of 32 four-byte banks per
// double).  Step by step, a maximum matching
// of the lanes still holding entries to distinct banks (lanes with the most
// entries left first, banks with the most entries left tried first) picks
// one entry per lane; a lane left unmatched takes the entry whose bank is
// least used at that step.
void order_for_banks(std::vector<std::vector<int32_t>> &lanes) {
    constexpr int Q = 16, NB = 16;
    auto bank = [](int32_t e) { return (e >> 3) % NB; };
    for (size_t q0 = 0; q0 < lanes.size(); q0 += Q) {
        std::vector<std::vector<int32_t>> rem(lanes.begin() + long(q0), lanes.begin() + long(q0 + Q)), out(Q);
        size_t L = 0;
        for (auto &v : rem) L = std::max(L, v.size());
        for (size_t j = 0; j < L; ++j) {
            int deg[NB] = {}, match_b[NB], match_l[Q], mult[NB] = {};
            std::fill(match_b, match_b + NB, -1);
            std::fill(match_l, match_l + Q, -1);
            for (auto &v : rem)
                for (int32_t e : v) ++deg[bank(e)];
            std::vector<int> act;
            for (int l = 0; l < Q; ++l)
                if (!rem[size_t(l)].empty()) act.push_back(l);
            std::vector<int> by_need = act;
            std::stable_sort(by_need.begin(), by_need.end(),
                             [&](int a, int b) { return rem[size_t(a)].size() > rem[size_t(b)].size(); });
            // augmenting paths (Kuhn); a lane's banks tried most loaded first
            auto options = [&](int l) {
                std::vector<int> o;
                bool has[NB] = {};
                for (int32_t e : rem[size_t(l)]) has[bank(e)] = true;
                for (int b = 0; b < NB; ++b)
                    if (has[b]) o.push_back(b);
                std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return deg[a] > deg[b]; });
                return o;
            };
            std::vector<std::vector<int>> opts(Q);
            for (int l : act) opts[size_t(l)] = options(l);
            std::vector<char> seen(NB);
            std::function<bool(int)> augment = [&](int l) {
                for (int b : opts[size_t(l)]) {
                    if (seen[size_t(b)]) continue;
                    seen[size_t(b)] = 1;
                    if (match_b[b] < 0 || augment(match_b[b])) {
                        match_b[b] = l;
                        match_l[l] = b;
                        return true;
                    }
                }
                return false;
            };
            for (int l : by_need) {
                std::fill(seen.begin(), seen.end(), 0);
                augment(l);
            }
            for (int l : act) {
                std::vector<int32_t> &v = rem[size_t(l)];
                size_t pick = 0;
                if (match_l[l] >= 0) {
                    while (bank(v[pick]) != match_l[l]) ++pick;
                } else {
                    for (size_t t = 1; t < v.size(); ++t) {
                        const int bt = bank(v[t]), bp = bank(v[pick]);
                        if (mult[bt] < mult[bp] || (mult[bt] == mult[bp] && deg[bt] > deg[bp])) pick = t;
                    }
                }
                ++mult[bank(v[pick])];
                out[size_t(l)].push_back(v[pick]);
                v.erase(v.begin() + long(pick));
            }
        }
        for (int l = 0; l < Q; ++l) lanes[q0 + size_t(l)] = out[size_t(l)];
    }
}

}  // namespace

namespace {

struct Tok {
    std::istringstream in;
    explicit Tok(const std::string &s) : in(s) {}
    template <typename T>
    bool get(T &v) { return static_cast<bool>(in >> v); }
};

bool expect_word(Tok &t, const char *w) {
    std::string s;
    return t.get(s) && s == w;
}

}  // namespace

HostNetwork::~HostNetwork() {
    for (size_t i = 0; i < spare.size(); ++i) {
        if (!spare[i].ptr) continue;
        int prev = 0;
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(int(i)) == hipSuccess) {
            (void)hipFree(spare[i].ptr);
            (void)hipSetDevice(prev);
        }
    }
    for (DeviceNet *d : dev) {
        if (!d) continue;
        int prev = 0;
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(d->device) == hipSuccess) {
            void *ptrs[] = {d->rx_ab, d->rx_type, d->alpha, d->beta, d->gamma, d->sg_base, d->sg_len,
                            d->sg_lane, d->sg_red, d->sg_ent, d->jrow_ptr, d->jcol, d->jrow, d->jterm_ptr, d->jt_rx_other, d->jt_coef,
                            d->rnu_ptr, d->rnu_ent, d->dcol_ptr, d->dcol_ent, d->dcol_coef, d->jidx,
                            d->jmask, d->jbase};
            for (void *p : ptrs)
                if (p) (void)hipFree(p);
            (void)hipSetDevice(prev);
        }
        delete d;
    }
}

int HostNetwork::parse(const char *text, size_t len, std::string &err) {
    Tok t(std::string(text, len));
    int version = 0;
    if (!expect_word(t, "astrobdf-network") || !t.get(version) || version != 1) {
        err = "not an astrobdf-network version 1 text";
        return ABDF_E_PARSE;
    }
    if (!expect_word(t, "name") || !t.get(name)) { err = "missing name"; return ABDF_E_PARSE; }
    std::string word;
    if (!t.get(word)) { err = "bad elements line"; return ABDF_E_PARSE; }
    if (word == "albedo") {
        if (!t.get(albedo) || !(albedo >= 0.0 && albedo < 1.0)) { err = "albedo must be in [0, 1)"; return ABDF_E_PARSE; }
        if (!t.get(word)) { err = "bad elements line"; return ABDF_E_PARSE; }
    }
    if (word != "elements" || !t.get(E) || E < 1 || E > 32) { err = "bad elements line"; return ABDF_E_PARSE; }
    elements.resize(E);
    for (int e = 0; e < E; ++e)
        if (!t.get(elements[e])) { err = "bad elements line"; return ABDF_E_PARSE; }
    if (!expect_word(t, "species") || !t.get(S) || S < 1 || S > 32000) { err = "bad species count"; return ABDF_E_PARSE; }
    species.resize(S);
    charge.resize(S);
    comp.resize(size_t(S) * E);
    for (int i = 0; i < S; ++i) {
        int idx = -1;
        if (!t.get(idx) || idx != i || !t.get(species[i]) || !t.get(charge[i])) {
            err = "bad species record " + std::to_string(i);
            return ABDF_E_PARSE;
        }
        for (int e = 0; e < E; ++e)
            if (!t.get(comp[size_t(i) * E + e]) || comp[size_t(i) * E + e] < 0) {
                err = "bad species record " + std::to_string(i);
                return ABDF_E_PARSE;
            }
    }
    if (!expect_word(t, "reactions") || !t.get(R) || R < 1 || R > (1 << 24)) { err = "bad reaction count"; return ABDF_E_PARSE; }
    rtype.resize(R);
    react.assign(size_t(R) * 2, -1);
    prod.assign(size_t(R) * 3, -1);
    alpha.resize(R);
    beta.resize(R);
    gamma.resize(R);
    for (int r = 0; r < R; ++r) {
        int idx = -1, nr = 0, np = 0;
        int32_t a[2], p[3];
        bool ok = t.get(idx) && idx == r && t.get(rtype[r]) && t.get(nr) && t.get(a[0]) && t.get(a[1]) &&
                  t.get(np) && t.get(p[0]) && t.get(p[1]) && t.get(p[2]) && t.get(alpha[r]) &&
                  t.get(beta[r]) && t.get(gamma[r]);
        if (!ok || nr < 1 || nr > 2 || np < 1 || np > 3 || rtype[r] < 0 || rtype[r] > 3) {
            err = "bad reaction record " + std::to_string(r);
            return ABDF_E_PARSE;
        }
        if ((rtype[r] != kTwoBody && nr != 1) || (rtype[r] == kTwoBody && nr != 2)) {
            err = "reaction " + std::to_string(r) + ": two-body needs 2 reactants, cosmic-ray/photo 1";
            return ABDF_E_PARSE;
        }
        for (int j = 0; j < 2; ++j) {
            bool used = j < nr;
            if ((used && (a[j] < 0 || a[j] >= S)) || (!used && a[j] != -1)) {
                err = "reaction " + std::to_string(r) + ": reactant index out of range";
                return ABDF_E_PARSE;
            }
            react[size_t(r) * 2 + j] = a[j];
        }
        for (int j = 0; j < 3; ++j) {
            bool used = j < np;
            if ((used && (p[j] < 0 || p[j] >= S)) || (!used && p[j] != -1)) {
                err = "reaction " + std::to_string(r) + ": product index out of range";
                return ABDF_E_PARSE;
            }
            prod[size_t(r) * 3 + j] = p[j];
        }
        // integer conservation of every element and the charge
        for (int e = 0; e <= E; ++e) {
            long long lhs = 0, rhs = 0;
            for (int j = 0; j < nr; ++j) lhs += e < E ? comp[size_t(a[j]) * E + e] : charge[a[j]];
            for (int j = 0; j < np; ++j) rhs += e < E ? comp[size_t(p[j]) * E + e] : charge[p[j]];
            if (lhs != rhs) {
                err = "reaction " + std::to_string(r) + " does not conserve " +
                      (e < E ? "element " + elements[e] : std::string("charge"));
                return ABDF_E_NONCONSERVING;
            }
        }
        if (!std::isfinite(alpha[r]) || !std::isfinite(beta[r]) || !std::isfinite(gamma[r])) {
            err = "reaction " + std::to_string(r) + ": non-finite parameter";
            return ABDF_E_PARSE;
        }
    }
    if (!expect_word(t, "end")) { err = "missing end"; return ABDF_E_PARSE; }
    finalize();
    return ABDF_OK;
}

void HostNetwork::finalize() {
    NP = (S + 15) / 16 * 16;
    // nu as a sparse map per species: (reaction, coefficient)
    std::vector<std::map<int, int>> nu(S);
    for (int r = 0; r < R; ++r) {
        for (int j = 0; j < 3; ++j)
            if (prod[size_t(r) * 3 + j] >= 0) nu[prod[size_t(r) * 3 + j]][r] += 1;
        for (int j = 0; j < 2; ++j)
            if (react[size_t(r) * 2 + j] >= 0) nu[react[size_t(r) * 2 + j]][r] -= 1;
    }
    // right-hand side: each species' nonzero entries, reactions ascending,
    // packed as reaction << 3 | (nu + 4)
    std::vector<std::vector<int32_t>> ent(S);
    for (int i = 0; i < S; ++i)
        for (auto &kv : nu[i])
            if (kv.second != 0) ent[size_t(i)].push_back((kv.first << 3) | (kv.second + 4));
    {
        // wave layout (DeviceNet::sg_ent): species i takes m_i consecutive
        // lanes of one group, its entries split as evenly as they go
        const size_t nS = static_cast<size_t>(S);
        std::vector<int> m(nS), len(nS), order(nS), used;
        std::vector<std::vector<int>> members;
        auto pack = [&](int seg) {
            for (int i = 0; i < S; ++i) {
                const int ni = int(ent[size_t(i)].size());
                m[size_t(i)] = std::max(1, std::min(64, (ni + seg - 1) / seg));
                len[size_t(i)] = (ni + m[size_t(i)] - 1) / m[size_t(i)];
                order[size_t(i)] = i;
            }
            // longest lanes first, each species into the first group with
            // room: a group's loop runs as long as its first species' lanes
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                return len[size_t(a)] != len[size_t(b)] ? len[size_t(a)] > len[size_t(b)] : m[size_t(a)] > m[size_t(b)];
            });
            used.clear();
            members.clear();
            for (int i : order) {
                size_t g = 0;
                while (g < used.size() && used[g] + m[size_t(i)] > 64) ++g;
                if (g == used.size()) {
                    used.push_back(0);
                    members.emplace_back();
                }
                members[g].push_back(i);
                used[g] += m[size_t(i)];
            }
        };
        // lanes of kRhsSegment entries, or longer ones (up to kRhsResidentLen)
        // where that brings the groups down to kRhsResidentGroups, the most the
        // streaming right-hand side keeps in registers
        for (int seg = kRhsSegment;; seg += 2) {
            pack(seg);
            if (used.size() <= size_t(kRhsResidentGroups)) break;
            if (seg + 2 > kRhsResidentLen) {
                pack(kRhsSegment);
                break;
            }
        }
        const size_t ng = used.size();
        sg_base.assign(ng, 0);
        sg_len.assign(ng, 0);
        sg_lane.assign(ng * 64, 0);
        sg_red.assign(ng * 64, -1);
        sg_ent.clear();
        for (size_t g = 0; g < ng; ++g) {
            int L = 0, mm = 1, steps = 0;
            for (int i : members[g]) {
                L = std::max(L, len[size_t(i)]);
                mm = std::max(mm, m[size_t(i)]);
            }
            while ((1 << steps) < mm) ++steps;
            sg_base[g] = int32_t(sg_ent.size());
            sg_len[g] = L | (steps << 24);
            sg_ent.resize(sg_ent.size() + size_t(L) * 64, 4);
            std::vector<std::vector<int32_t>> lanes(64);
            int lane = 0;
            for (int i : members[g]) {
                const std::vector<int32_t> &e = ent[size_t(i)];
                const int ni = int(e.size()), mi = m[size_t(i)], base = ni / mi, extra = ni % mi;
                size_t next = 0;
                for (int q = 0; q < mi; ++q, ++lane) {
                    const int lq = base + (q < extra ? 1 : 0);
                    sg_lane[g * 64 + size_t(lane)] = lq;
                    sg_red[g * 64 + size_t(lane)] = (i << 14) | (q << 7) | mi;
                    lanes[size_t(lane)].assign(e.begin() + long(next), e.begin() + long(next + size_t(lq)));
                    next += size_t(lq);
                }
            }
            order_for_banks(lanes);
            for (size_t l = 0; l < 64; ++l)
                for (size_t j = 0; j < lanes[l].size(); ++j) sg_ent[size_t(sg_base[g]) + j * 64 + l] = lanes[l][j];
        }
    }

    // Jacobian terms: d rate_r / d x_j of a mass-action rate
    struct Term { int j, r, other; double coef; };
    std::vector<std::vector<Term>> rows(S);
    rnu_ptr.assign(R + 1, 0);
    rnu_ent.clear();
    std::vector<std::vector<Term>> dcols(S);
    for (int r = 0; r < R; ++r) {
        int a = react[size_t(r) * 2], b = react[size_t(r) * 2 + 1];
        Term d[2];
        int nd = 0;
        if (b < 0) d[nd++] = {a, r, -1, 1.0};
        else if (a == b) d[nd++] = {a, r, a, 2.0};
        else { d[nd++] = {a, r, b, 1.0}; d[nd++] = {b, r, a, 1.0}; }
        for (int q = 0; q < nd; ++q) dcols[d[q].j].push_back(d[q]);
        std::map<int, int> nur;
        for (int j = 0; j < 3; ++j)
            if (prod[size_t(r) * 3 + j] >= 0) nur[prod[size_t(r) * 3 + j]] += 1;
        for (int j = 0; j < 2; ++j)
            if (react[size_t(r) * 2 + j] >= 0) nur[react[size_t(r) * 2 + j]] -= 1;
        rnu_ptr[r] = int32_t(rnu_ent.size());
        for (auto &kv : nur)
            if (kv.second != 0) rnu_ent.push_back((kv.first << 3) | (kv.second + 4));
        for (auto &kv : nur) {
            if (kv.second == 0) continue;
            for (int q = 0; q < nd; ++q)
                rows[kv.first].push_back({d[q].j, r, d[q].other, kv.second * d[q].coef});
        }
    }
    jrow_ptr.assign(S + 1, 0);
    jcol.clear();
    jrow.clear();
    jterm_ptr.clear();
    jt_rx_other.clear();
    jt_coef.clear();
    for (int i = 0; i < S; ++i) {
        auto &v = rows[i];
        std::stable_sort(v.begin(), v.end(), [](const Term &x, const Term &y) {
            return x.j != y.j ? x.j < y.j : x.r < y.r;
        });
        jrow_ptr[i] = int32_t(jcol.size());
        int last = -1;
        for (auto &tm : v) {
            if (tm.j != last) {
                jcol.push_back(tm.j);
                jrow.push_back(i);
                jterm_ptr.push_back(int32_t(jt_coef.size()));
                last = tm.j;
            }
            jt_rx_other.push_back((tm.r << 16) | (tm.other + 1));
            jt_coef.push_back(tm.coef);
        }
    }
    jrow_ptr[S] = int32_t(jcol.size());
    jterm_ptr.push_back(int32_t(jt_coef.size()));
    rnu_ptr[R] = int32_t(rnu_ent.size());
    dcol_ptr.assign(S + 1, 0);
    dcol_ent.clear();
    dcol_coef.clear();
    for (int j = 0; j < S; ++j) {
        dcol_ptr[j] = int32_t(dcol_ent.size());
        for (auto &tm : dcols[j]) {
            dcol_ent.push_back((tm.r << 16) | (tm.other + 1));
            dcol_coef.push_back(tm.coef);
        }
    }
    dcol_ptr[S] = int32_t(dcol_ent.size());
    jidx.assign(size_t(NP) * NP, -1);
    for (size_t e = 0; e < jcol.size(); ++e) jidx[size_t(jrow[e]) * NP + jcol[e]] = int32_t(e);
    const int nbw = (NP + 63) / 64;
    jmask.assign(size_t(NP) * nbw, 0);
    jbase.assign(size_t(NP) * nbw, 0);
    for (int i = 0; i < NP; ++i) {
        int32_t next = i < S ? jrow_ptr[i] : 0;
        for (int b = 0; b < nbw; ++b) {
            jbase[size_t(i) * nbw + b] = next;
            uint64_t m = 0;
            for (int c = 0; c < 64 && 64 * b + c < NP; ++c)
                if (jidx[size_t(i) * NP + 64 * b + c] >= 0) {
                    // the numbering the word encodes is the map's
                    if (jidx[size_t(i) * NP + 64 * b + c] != next) std::abort();
                    m |= uint64_t(1) << c;
                    ++next;
                }
            jmask[size_t(i) * nbw + b] = m;
        }
    }
}

namespace {
template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src) {
    size_t n = std::max<size_t>(src.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), n);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}
}  // namespace

const DeviceNet *HostNetwork::device_tables_present(int devid) const {
    std::lock_guard<std::mutex> lock(mu);
    return devid >= 0 && devid < int(dev.size()) ? dev[devid] : nullptr;
}

void *HostNetwork::take_workspace(int devid, size_t bytes, size_t *got) const {
    void *drop = nullptr, *p = nullptr;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (devid < 0 || devid >= int(spare.size()) || !spare[devid].ptr) return nullptr;
        if (spare[devid].bytes >= bytes) {
            p = spare[devid].ptr;
            *got = spare[devid].bytes;
        } else {
            drop = spare[devid].ptr;   // too small: released, so that a larger one can be allocated
        }
        spare[devid] = Block{};
    }
    if (drop) (void)hipFree(drop);
    return p;
}

void HostNetwork::keep_workspace(int devid, void *ptr, size_t bytes) const {
    void *drop = nullptr;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (devid < 0) {
            drop = ptr;
        } else {
            if (int(spare.size()) <= devid) spare.resize(devid + 1);
            Block &b = spare[devid];
            if (bytes > b.bytes) {
                drop = b.ptr;
                b = Block{ptr, bytes};
            } else {
                drop = ptr;
            }
        }
    }
    if (drop) (void)hipFree(drop);
}

size_t HostNetwork::cached_workspace_bytes(int devid) const {
    std::lock_guard<std::mutex> lock(mu);
    return devid >= 0 && devid < int(spare.size()) ? spare[devid].bytes : 0;
}

const DeviceNet *HostNetwork::device_tables(std::string &err) const {
    int devid = 0;
    if (hipGetDevice(&devid) != hipSuccess) {
        err = "no HIP device";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (int(dev.size()) <= devid) dev.resize(devid + 1, nullptr);
    if (dev[devid]) return dev[devid];
    if (R >= (1 << 15) || S >= 0xffff) {
        err = "network too large for the packed device tables";
        return nullptr;
    }
    auto *d = new DeviceNet();
    d->device = devid;
    d->S = S;
    d->R = R;
    d->NP = NP;
    std::vector<int32_t> ab(R);
    for (int r = 0; r < R; ++r) {
        int a = react[size_t(r) * 2], b = react[size_t(r) * 2 + 1];
        ab[r] = (a & 0xffff) | ((b < 0 ? 0xffff : b) << 16);
    }
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(upload(&d->rx_ab, ab));
    chk(upload(&d->rx_type, rtype));
    d->albedo = albedo;
    chk(upload(&d->alpha, alpha));
    chk(upload(&d->beta, beta));
    chk(upload(&d->gamma, gamma));
    chk(upload(&d->sg_base, sg_base));
    chk(upload(&d->sg_len, sg_len));
    chk(upload(&d->sg_lane, sg_lane));
    chk(upload(&d->sg_red, sg_red));
    chk(upload(&d->sg_ent, sg_ent));
    chk(upload(&d->jrow_ptr, jrow_ptr));
    chk(upload(&d->jcol, jcol));
    chk(upload(&d->jrow, jrow));
    chk(upload(&d->jterm_ptr, jterm_ptr));
    chk(upload(&d->jt_rx_other, jt_rx_other));
    chk(upload(&d->jt_coef, jt_coef));
    chk(upload(&d->rnu_ptr, rnu_ptr));
    chk(upload(&d->rnu_ent, rnu_ent));
    chk(upload(&d->dcol_ptr, dcol_ptr));
    chk(upload(&d->dcol_ent, dcol_ent));
    chk(upload(&d->dcol_coef, dcol_coef));
    chk(upload(&d->jidx, jidx));
    chk(upload(&d->jmask, jmask));
    chk(upload(&d->jbase, jbase));
    d->nbw = (NP + 63) / 64;
    d->n_sgroup = int32_t(sg_base.size());
    d->sg_maxlen = 0;
    for (int32_t w : sg_len) d->sg_maxlen = std::max(d->sg_maxlen, w & 0xffffff);
    d->nnzJ = int32_t(jcol.size());
    d->nterm = int32_t(jt_coef.size());
    if (e != hipSuccess) {
        err = std::string("uploading network tables: ") + hipGetErrorString(e);
        return nullptr;  // the partial upload is leaked rather than reused
    }
    dev[devid] = d;
    return d;
}

}  // namespace abdf
