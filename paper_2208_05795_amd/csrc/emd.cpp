// Cycle / EMD spectrum of a QC code (Section II, Table II), computed on the
// base matrix: a walk that alternates block columns and block rows through
// nonzero circulants, column j -(row i)-> column j', moves the offset c of a
// variable to (c - s_ij + s_ij') mod z, and closes on the starting variable
// exactly when its alternating exponent sum is 0 mod z (Fossorier's condition).
// The walk keeps the lifted offsets only to reject lifts that revisit a node
// (which are not simple cycles) and to measure each cycle's EMD: the number of
// (cycle variable, check) incidences whose check meets the cycle in exactly one
// variable.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

using namespace tsg;

namespace {

struct Walker {
    const ts_code *c;
    int z, mb, nb, max_len, emd_max;
    std::vector<int32_t> S;           // shifts [mb][nb], -1 = zero block
    std::vector<std::vector<int>> rows_of, cols_of;   // nonzero blocks per column / row
    std::vector<int> vj, vc, ci, cr;  // cycle variables (column, offset), checks (row, offset)
    std::vector<uint8_t> used_v, used_c;
    int64_t *out;

    int shift(int i, int j) const { return S[(size_t)i * nb + j]; }

    // EMD of the cycle held in vj/vc (l variables)
    int emd(int l) const {
        int e = 0;
        for (int a = 0; a < l; ++a)
            for (int i : rows_of[vj[a]]) {
                const int r = ((vc[a] - shift(i, vj[a])) % z + z) % z;
                int hits = 0;
                for (int b = 0; b < l; ++b) {
                    const int s = shift(i, vj[b]);
                    if (s >= 0 && (r + s) % z == vc[b]) ++hits;
                }
                if (hits == 1) ++e;
            }
        return e;
    }

    // at variable vj[l-1], vc[l-1] with l variables and l-1 checks on the path
    void from_variable(int l) {
        if (2 * l > max_len) return;
        const int j = vj[l - 1], c = vc[l - 1];
        for (int i : rows_of[j]) {
            const int r = ((c - shift(i, j)) % z + z) % z;
            const size_t cid = (size_t)i * z + r;
            if (used_c[cid]) continue;
            used_c[cid] = 1;
            ci.push_back(i);
            cr.push_back(r);
            from_check(l);
            ci.pop_back();
            cr.pop_back();
            used_c[cid] = 0;
        }
    }

    // at check ci.back(), cr.back() after l variables
    void from_check(int l) {
        const int i = ci.back(), r = cr.back(), jprev = vj[l - 1];
        for (int j : cols_of[i]) {
            if (j == jprev) continue;   // the edge just taken
            const int c = (r + shift(i, j)) % z;
            if (j == vj[0] && c == vc[0]) {
                if (l >= 2) {
                    // each undirected cycle through the start once: first check below last
                    const size_t first = (size_t)ci[0] * z + cr[0], last = (size_t)i * z + r;
                    if (first < last) {
                        const int e = std::min(emd(l), emd_max);
                        out[(size_t)l * (emd_max + 1) + e]++;
                    }
                }
                continue;
            }
            const size_t vid = (size_t)j * z + c;
            if (used_v[vid] || 2 * (l + 1) > max_len) continue;
            used_v[vid] = 1;
            vj.push_back(j);
            vc.push_back(c);
            from_variable(l + 1);
            vj.pop_back();
            vc.pop_back();
            used_v[vid] = 0;
        }
    }
};

}  // namespace

extern "C" int ts_cycle_emd(ts_ctx *ctx, const ts_code *code, int32_t max_len, int32_t emd_max,
                            int64_t *out) {
    clear_error();
    if (!ctx || !code || !out) { set_error("null argument"); return TS_E_INVAL; }
    if (code->ctx != ctx) { set_error("code belongs to another context"); return TS_E_STATE; }
    if (code->z <= 0) { set_error("the cycle spectrum needs a code in QC form"); return TS_E_INVAL; }
    if (max_len < 4 || max_len > 16 || (max_len & 1) || emd_max < 0 || emd_max > 4096) {
        set_error("max_len must be even in 4..16, emd_max in 0..4096");
        return TS_E_INVAL;
    }
    Walker w;
    w.c = code;
    w.z = code->z;
    w.mb = code->mb;
    w.nb = code->nb;
    w.max_len = max_len;
    w.emd_max = emd_max;
    w.out = out;
    // recover the exponent matrix from the expanded code: row i*z of block row
    // i meets column j*z + s in block (i, j)
    w.S.assign((size_t)w.mb * w.nb, -1);
    for (int i = 0; i < w.mb; ++i)
        for (int64_t e = code->row_ptr[(size_t)i * w.z]; e < code->row_ptr[(size_t)i * w.z + 1]; ++e) {
            const int v = code->col[e];
            w.S[(size_t)i * w.nb + v / w.z] = v % w.z;
        }
    w.rows_of.assign(w.nb, {});
    w.cols_of.assign(w.mb, {});
    for (int i = 0; i < w.mb; ++i)
        for (int j = 0; j < w.nb; ++j)
            if (w.shift(i, j) >= 0) {
                w.rows_of[j].push_back(i);
                w.cols_of[i].push_back(j);
            }
    std::memset(out, 0, sizeof(int64_t) * (size_t)(max_len / 2 + 1) * (emd_max + 1));
    w.used_v.assign((size_t)code->n, 0);
    w.used_c.assign((size_t)code->m, 0);
    for (int j0 = 0; j0 < w.nb; ++j0) {
        w.vj.assign(1, j0);
        w.vc.assign(1, 0);
        w.ci.clear();
        w.cr.clear();
        w.used_v[(size_t)j0 * w.z] = 1;
        w.from_variable(1);
        w.used_v[(size_t)j0 * w.z] = 0;
    }
    return TS_OK;
}
