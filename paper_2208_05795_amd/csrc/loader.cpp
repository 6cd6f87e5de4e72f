// Code loading: validation, QC expansion, adjacency, girth, device upload, and
// the impulse pattern families.
//
// QC expansion (Section II, eq. 1-3): the circulant P^s has the one of row r in
// column (r+s) mod z; block (i,j) with exponent s joins check i*z+r to variable
// j*z+(r+s) mod z, and exponent -1 is the zero block.
#include <algorithm>
#include <climits>
#include <array>
#include <cstring>
#include <queue>

#include "internal.h"

namespace tsg {

namespace {

// Shortest cycle of the Tanner graph: breadth-first search from every variable
// with the parent node recorded; a non-tree edge (x,y) closes a cycle of length
// d(x) + d(y) + 1 through the root's tree, and the minimum over all roots is
// the girth.
int girth_bfs(const ts_code *c) {
    const int nv = c->n, nn = c->n + c->m;
    std::vector<int> dist(nn, -1), parent(nn, -1), touched;
    std::vector<int> q;
    q.reserve(nn);
    touched.reserve(nn);
    int best = 0;
    for (int root = 0; root < nv; ++root) {
        for (int x : touched) dist[x] = -1;
        touched.clear();
        q.clear();
        dist[root] = 0;
        parent[root] = -1;
        touched.push_back(root);
        q.push_back(root);
        for (size_t h = 0; h < q.size(); ++h) {
            const int x = q[h];
            if (best && 2 * dist[x] + 1 >= best) break;
            const bool is_var = x < nv;
            const int64_t lo = is_var ? c->vptr[x] : c->row_ptr[x - nv];
            const int64_t hi = is_var ? c->vptr[x + 1] : c->row_ptr[x - nv + 1];
            for (int64_t k = lo; k < hi; ++k) {
                const int y = is_var ? nv + c->vchk[k] : c->col[k];
                if (y == parent[x]) continue;
                if (dist[y] < 0) {
                    dist[y] = dist[x] + 1;
                    parent[y] = x;
                    touched.push_back(y);
                    q.push_back(y);
                } else {
                    const int len = dist[x] + dist[y] + 1;
                    if (!best || len < best) best = len;
                }
            }
        }
    }
    return best;
}

}  // namespace

int build_code(const ts_code_desc *d, ts_code *c) {
    if (!d) { set_error("null code description"); return TS_E_INVAL; }
    if (d->kind == TS_CODE_QC) {
        if (d->mb <= 0 || d->nb <= 0 || d->z <= 0 || !d->shifts) {
            set_error("QC code needs mb, nb, z > 0 and shifts");
            return TS_E_INVAL;
        }
        const int64_t n = (int64_t)d->nb * d->z, m = (int64_t)d->mb * d->z;
        if (n > (1 << 24) || m > (1 << 24)) { set_error("code too large"); return TS_E_INVAL; }
        if ((int64_t)d->mb * d->nb > (1 << 24)) { set_error("base matrix too large"); return TS_E_INVAL; }
        for (int i = 0; i < d->mb * d->nb; ++i)
            if (d->shifts[i] < -1 || d->shifts[i] >= d->z) {
                set_error("shift %d at %d outside [-1, z)", d->shifts[i], i);
                return TS_E_INVAL;
            }
        c->n = (int)n;
        c->m = (int)m;
        c->z = d->z;
        c->mb = d->mb;
        c->nb = d->nb;
        c->row_ptr.assign((size_t)m + 1, 0);
        c->col.clear();
        for (int i = 0; i < d->mb; ++i)
            for (int r = 0; r < d->z; ++r) {
                const size_t start = c->col.size();
                for (int j = 0; j < d->nb; ++j) {
                    const int s = d->shifts[i * d->nb + j];
                    if (s >= 0) c->col.push_back(j * d->z + (r + s) % d->z);
                }
                std::sort(c->col.begin() + start, c->col.end());
                c->row_ptr[(size_t)i * d->z + r + 1] = (int64_t)c->col.size();
            }
    } else if (d->kind == TS_CODE_CSR) {
        if (d->n <= 0 || d->m <= 0 || !d->row_ptr || (d->nnz > 0 && !d->col_idx)) {
            set_error("CSR code needs n, m > 0 and arrays");
            return TS_E_INVAL;
        }
        if (d->n > (1 << 24) || d->m > (1 << 24)) { set_error("code too large"); return TS_E_INVAL; }
        if (d->row_ptr[0] != 0 || d->row_ptr[d->m] != d->nnz) {
            set_error("row_ptr must start at 0 and end at nnz");
            return TS_E_INVAL;
        }
        c->n = d->n;
        c->m = d->m;
        c->z = 0;
        c->row_ptr.assign(d->row_ptr, d->row_ptr + d->m + 1);
        c->col.assign(d->col_idx, d->col_idx + d->nnz);
        for (int r = 0; r < d->m; ++r) {
            if (c->row_ptr[r + 1] < c->row_ptr[r]) { set_error("row_ptr not monotone"); return TS_E_INVAL; }
            std::sort(c->col.begin() + c->row_ptr[r], c->col.begin() + c->row_ptr[r + 1]);
        }
        for (int64_t k = 0; k < d->nnz; ++k)
            if (c->col[k] < 0 || c->col[k] >= d->n) {
                set_error("column %d out of range", c->col[k]);
                return TS_E_INVAL;
            }
    } else {
        set_error("unknown code kind %d", d->kind);
        return TS_E_INVAL;
    }
    c->e = (int64_t)c->col.size();
    if (c->e >= (int64_t)1 << 30) { set_error("too many edges"); return TS_E_INVAL; }
    c->dc_max = 0;
    for (int r = 0; r < c->m; ++r) {
        const int deg = (int)(c->row_ptr[r + 1] - c->row_ptr[r]);
        if (deg < 2) { set_error("check %d has degree %d (< 2)", r, deg); return TS_E_INVAL; }
        for (int64_t k = c->row_ptr[r] + 1; k < c->row_ptr[r + 1]; ++k)
            if (c->col[k] == c->col[k - 1]) { set_error("duplicate edge in check %d", r); return TS_E_INVAL; }
        c->dc_max = std::max(c->dc_max, deg);
    }
    // variable side: counting sort of the edges by variable
    c->vptr.assign((size_t)c->n + 1, 0);
    for (int32_t v : c->col) c->vptr[v + 1]++;
    for (int v = 0; v < c->n; ++v) c->vptr[v + 1] += c->vptr[v];
    c->vchk.assign((size_t)c->e, 0);
    c->vedge.assign((size_t)c->e, 0);
    std::vector<int64_t> pos(c->vptr.begin(), c->vptr.end() - 1);
    for (int r = 0; r < c->m; ++r)
        for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; ++k) {
            const int v = c->col[k];
            c->vchk[pos[v]] = r;
            c->vedge[pos[v]] = (int32_t)k;
            pos[v]++;
        }
    c->dv_max = 0;
    for (int v = 0; v < c->n; ++v) {
        const int deg = (int)(c->vptr[v + 1] - c->vptr[v]);
        if (deg == 0) { set_error("variable %d has no check", v); return TS_E_INVAL; }
        c->dv_max = std::max(c->dv_max, deg);
    }
    c->girth = girth_bfs(c);
    return TS_OK;
}

namespace {

// Order of each check's edges in the device neighbour tables: slot j of check
// r holds edge ord[row_ptr[r] + j].  The lanes of a wavefront own 64
// consecutive checks, and the APP gather (and atomic add) of slot j touches
// one LDS word per lane; words in one bank serialise.  The order within a
// check is free for the decoders (min-sum does not depend on it; the
// sum-product sums follow it in every layout alike), so a local search swaps
// two edges of a check while that lowers the sum over slots of the squared
// bank loads, counted over 64 banks per wavefront and over 32 banks per
// half-wavefront.
std::vector<int64_t> edge_order(const ts_code *c) {
    std::vector<int64_t> ord((size_t)c->e);
    for (int64_t k = 0; k < c->e; ++k) ord[k] = k;
    // a QC code keeps its natural order: consecutive rows of a circulant already
    // gather consecutive words, and the streamed layout derives its indices
    // from the block structure
    if (c->z > 0) return ord;
    const int dmax = c->dc_max;
    std::vector<int> c64((size_t)dmax * 64), c32((size_t)2 * dmax * 32);
    for (int g0 = 0; g0 < c->m; g0 += 64) {
        const int g1 = std::min(c->m, g0 + 64);
        std::fill(c64.begin(), c64.end(), 0);
        std::fill(c32.begin(), c32.end(), 0);
        for (int r = g0; r < g1; ++r) {
            const int h = (r - g0) >> 5;
            for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; ++k) {
                const int j = (int)(k - c->row_ptr[r]), v = c->col[ord[k]];
                c64[(size_t)j * 64 + (v & 63)]++;
                c32[((size_t)h * dmax + j) * 32 + (v & 31)]++;
            }
        }
        for (int pass = 0; pass < 8; ++pass) {
            bool moved = false;
            for (int r = g0; r < g1; ++r) {
                const int h = (r - g0) >> 5, d = (int)(c->row_ptr[r + 1] - c->row_ptr[r]);
                int64_t *o = ord.data() + c->row_ptr[r];
                for (int j1 = 0; j1 < d; ++j1)
                    for (int j2 = j1 + 1; j2 < d; ++j2) {
                        const int a = c->col[o[j1]], b = c->col[o[j2]];
                        int *p1 = &c64[(size_t)j1 * 64], *p2 = &c64[(size_t)j2 * 64];
                        int *q1 = &c32[((size_t)h * dmax + j1) * 32], *q2 = &c32[((size_t)h * dmax + j2) * 32];
                        const int a6 = a & 63, b6 = b & 63, a5 = a & 31, b5 = b & 31;
                        int delta = 0;
                        if (a6 != b6) delta += 2 * (p1[b6] - p1[a6] + p2[a6] - p2[b6]) + 4;
                        if (a5 != b5) delta += 2 * (q1[b5] - q1[a5] + q2[a5] - q2[b5]) + 4;
                        if (delta >= 0) continue;
                        p1[a6]--, p1[b6]++, p2[b6]--, p2[a6]++;
                        q1[a5]--, q1[b5]++, q2[b5]--, q2[a5]++;
                        std::swap(o[j1], o[j2]);
                        moved = true;
                    }
            }
            if (!moved) break;
        }
    }
    return ord;
}

}  // namespace

int upload_code(ts_exec &ex, ts_code *c) {
    DevCode &d = c->dev;
    d.n = c->n;
    d.m = c->m;
    d.e = (int)c->e;
    d.dv_max = c->dv_max;
    d.dc_max = c->dc_max;
    d.z = c->z;
    // padded tables: cn_tab[j][check] = j-th variable of the check, vn_tab[d][var] =
    // edge of the var's d-th check; both with a column stride rounded to 64
    d.dc_pad = c->dc_max;
    d.m_tab = (c->m + 63) / 64 * 64;
    d.dv_pad = c->dv_max;
    d.n_tab = (c->n + 63) / 64 * 64;
    std::vector<int32_t> rp32(c->row_ptr.begin(), c->row_ptr.end());
    std::vector<int32_t> vp32(c->vptr.begin(), c->vptr.end());
    std::vector<int32_t> cn((size_t)d.dc_pad * d.m_tab, -1), vn((size_t)d.dv_pad * d.n_tab, -1);
    const std::vector<int64_t> ord = edge_order(c);
    for (int r = 0; r < c->m; ++r)
        for (int64_t k = c->row_ptr[r]; k < c->row_ptr[r + 1]; ++k)
            cn[(size_t)(k - c->row_ptr[r]) * d.m_tab + r] = c->col[ord[k]];
    for (int v = 0; v < c->n; ++v)
        for (int64_t k = c->vptr[v]; k < c->vptr[v + 1]; ++k)
            vn[(size_t)(k - c->vptr[v]) * d.n_tab + v] = c->vedge[k];
    // streamed layout: checks sorted (stably) by degree, each degree padded to
    // its class; class q stores slot j of its checks contiguously
    std::vector<int32_t> order(c->m);
    for (int r = 0; r < c->m; ++r) order[r] = r;
    auto deg = [&](int r) { return (int)(c->row_ptr[r + 1] - c->row_ptr[r]); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return deg(x) < deg(y); });
    const bool skip24 = c->dc_max > 24;
    auto class_of = [skip24](int dg) {
        for (int q = 0; q < kGMaxCls; ++q)
            if (kGClasses[q] >= dg && !(skip24 && kGClasses[q] == 24)) return q;
        return -1;
    };
    d.g_ncls = 0;
    std::vector<int32_t> gcn, gvs((size_t)d.dv_pad * d.n_tab, -1);
    if (c->dc_max <= kGClasses[kGMaxCls - 1]) {
        std::vector<int32_t> edge_slot(c->e, -1);
        int p = 0, off = 0;
        while (p < c->m) {
            const int q = class_of(deg(order[p]));
            int p1 = p;
            while (p1 < c->m && class_of(deg(order[p1])) == q) ++p1;
            const int cnt = p1 - p, stride = (cnt + 63) / 64 * 64, dcq = kGClasses[q];
            const int k = d.g_ncls++;
            d.g_dc[k] = dcq;
            d.g_c0[k] = p;
            d.g_stride[k] = stride;
            d.g_off[k] = off;
            gcn.resize((size_t)off + (size_t)dcq * stride, c->n);
            for (int i = p; i < p1; ++i) {
                const int r = order[i];
                for (int64_t e = c->row_ptr[r]; e < c->row_ptr[r + 1]; ++e) {
                    const int j = (int)(e - c->row_ptr[r]);
                    const int slot = off + j * stride + (i - p);
                    gcn[slot] = c->col[ord[e]];
                    edge_slot[ord[e]] = slot;
                }
            }
            off += dcq * stride;
            p = p1;
        }
        d.g_c0[d.g_ncls] = c->m;
        d.g_off[d.g_ncls] = off;
        for (int v = 0; v < c->n; ++v)
            for (int64_t k = c->vptr[v]; k < c->vptr[v + 1]; ++k)
                gvs[(size_t)(k - c->vptr[v]) * d.n_tab + v] = edge_slot[c->vedge[k]];
    }
    if (gcn.empty()) gcn.push_back(c->n);
    // QC code: the streamed indices from per-circulant tables (block row i,
    // neighbour slot j -> (j z, shift); block column j, k-th check -> (slot base,
    // shift)), switched on only once every computed index equals the table
    // entry it replaces
    d.q_ok = 0;
    std::vector<int32_t> qtab, qrow;
    if (c->z > 0 && d.g_ncls > 0 && c->z < (1 << 16) && c->mb < (1 << 15)) {
        const int z = c->z, mb = c->mb, nb = c->nb;
        std::vector<int> S((size_t)mb * nb, -1);   // shifts, read off row 0 of each block row
        for (int i = 0; i < mb; ++i)
            for (int64_t e = c->row_ptr[(size_t)i * z]; e < c->row_ptr[(size_t)i * z + 1]; ++e)
                S[(size_t)i * nb + c->col[e] / z] = c->col[e] % z;
        const int qdc = d.g_dc[d.g_ncls - 1], qdv = d.dv_pad;
        std::vector<int> pos_of((size_t)c->m);
        for (int p = 0; p < c->m; ++p) pos_of[order[p]] = p;
        const size_t vb = 2 * (size_t)mb * qdc;
        qtab.assign(vb + 2 * (size_t)nb * qdv, -1);
        bool ok = true;
        for (int i = 0; i < mb; ++i) {
            int jj = 0;
            for (int j = 0; j < nb; ++j)
                if (S[(size_t)i * nb + j] >= 0) {
                    if (jj >= qdc) { ok = false; break; }
                    qtab[2 * ((size_t)i * qdc + jj)] = j * z;
                    qtab[2 * ((size_t)i * qdc + jj) + 1] = S[(size_t)i * nb + j];
                    ++jj;
                }
        }
        for (int j = 0; j < nb && ok; ++j) {
            int kk = 0;
            for (int i = 0; i < mb; ++i) {
                if (S[(size_t)i * nb + j] < 0) continue;
                if (kk >= qdv) { ok = false; break; }
                int jp = 0;   // slot of column j among the nonzero blocks of row i
                for (int j2 = 0; j2 < j; ++j2) jp += S[(size_t)i * nb + j2] >= 0;
                const int P0 = pos_of[(size_t)i * z];
                int q = 0;
                while (q + 1 < d.g_ncls && P0 >= d.g_c0[q + 1]) ++q;
                qtab[vb + 2 * ((size_t)j * qdv + kk)] = d.g_off[q] + jp * d.g_stride[q] + (P0 - d.g_c0[q]);
                qtab[vb + 2 * ((size_t)j * qdv + kk) + 1] = S[(size_t)i * nb + j];
                ++kk;
            }
        }
        qrow.resize((size_t)c->m);
        for (int p = 0; p < c->m; ++p) qrow[p] = ((order[p] / z) << 16) | (order[p] % z);
        for (int q = 0; q < d.g_ncls && ok; ++q)
            for (int p = d.g_c0[q]; p < d.g_c0[q + 1] && ok; ++p) {
                const int i = qrow[p] >> 16, r = qrow[p] & 0xffff;
                for (int j = 0; j < d.g_dc[q] && ok; ++j) {
                    const int v = qc_neighbour(&qtab[2 * ((size_t)i * qdc + j)], r, z, c->n);
                    ok = v == gcn[(size_t)d.g_off[q] + (size_t)j * d.g_stride[q] + (p - d.g_c0[q])];
                }
            }
        for (int v = 0; v < c->n && ok; ++v) {
            const int jc = v / z, cc = v % z;
            for (int k = 0; k < qdv && ok; ++k)
                ok = qc_slot(&qtab[vb + 2 * ((size_t)jc * qdv + k)], cc, z) == gvs[(size_t)k * d.n_tab + v];
        }
        // the tables must not cost a code its streamed frame at any iteration count
        const int qb = (int)(qtab.size() * 4);
        const size_t lim = ex.ctx ? ex.ctx->lds_per_block : 0;
        const bool fits = kHdrLds + lds_layout_g(c->n, kMaxIter, qb).total <= lim ||
                          kHdrLds + lds_layout_g(c->n, kMaxIter, 0).total > lim;
        if (ok && fits && qb <= kQTabMaxBytes) {
            d.q_ok = 1;
            d.q_dc = qdc;
            d.q_dv = qdv;
            d.q_bytes = (int)(qtab.size() * 4);
            d.q_var_off = (int)vb;
            d.q_inv_z = 1.0f / (float)z;
        }
    }
    if (qtab.empty()) qtab.push_back(-1);
    if (qrow.empty()) qrow.push_back(0);
    // layered schedule: block rows of a QC code; otherwise each check, in index
    // order, goes to the lowest layer none of whose checks shares a variable
    std::vector<int32_t> lay((size_t)std::max(c->m, 1), 0);
    d.n_layers = 0;
    if (c->z > 0) {
        for (int r = 0; r < c->m; ++r) lay[r] = r / c->z;
        d.n_layers = c->mb;
    } else {
        std::vector<uint64_t> busy((size_t)c->n, 0);   // bit L: variable has a check in layer L
        bool ok = true;
        for (int r = 0; r < c->m && ok; ++r) {
            uint64_t taken = 0;
            for (int64_t e = c->row_ptr[r]; e < c->row_ptr[r + 1]; ++e) taken |= busy[c->col[e]];
            if (~taken == 0) { ok = false; break; }
            const int L = __builtin_ctzll(~taken);
            lay[r] = L;
            for (int64_t e = c->row_ptr[r]; e < c->row_ptr[r + 1]; ++e) busy[c->col[e]] |= 1ull << L;
            d.n_layers = std::max(d.n_layers, L + 1);
        }
        if (!ok) d.n_layers = 0;   // more than 64 layers: the layered decoder is not offered
    }
    // layer-major check order: a wavefront's lanes then hold checks of one layer,
    // so each layer's update runs on few wavefronts instead of all of them
    std::vector<int32_t> lorder(c->m);
    for (int r = 0; r < c->m; ++r) lorder[r] = r;
    std::stable_sort(lorder.begin(), lorder.end(), [&](int x, int y) { return lay[x] < lay[y]; });
    std::vector<int32_t> lay_pos((size_t)std::max(c->m, 1), 0), cnl((size_t)d.dc_pad * d.m_tab, -1);
    for (int p = 0; p < c->m; ++p) {
        lay_pos[p] = lay[lorder[p]];
        for (int j = 0; j < d.dc_pad; ++j) cnl[(size_t)j * d.m_tab + p] = cn[(size_t)j * d.m_tab + lorder[p]];
    }
    struct Up { const void *src; size_t bytes; const int **dst; } ups[] = {
        {rp32.data(), rp32.size() * 4, &d.row_ptr}, {c->col.data(), c->col.size() * 4, &d.col},
        {vp32.data(), vp32.size() * 4, &d.vptr},    {c->vchk.data(), c->vchk.size() * 4, &d.vchk},
        {c->vedge.data(), c->vedge.size() * 4, &d.vedge}, {cn.data(), cn.size() * 4, &d.cn_tab},
        {vn.data(), vn.size() * 4, &d.vn_tab}, {gcn.data(), gcn.size() * 4, &d.g_cn},
        {gvs.data(), gvs.size() * 4, &d.g_vslot}, {lay_pos.data(), lay_pos.size() * 4, &d.lay_of},
        {cnl.data(), cnl.size() * 4, &d.cn_lay},
        {qtab.data(), qtab.size() * 4, &d.q_tab}, {qrow.data(), qrow.size() * 4, &d.q_rowpos},
    };
    for (auto &u : ups) {
        void *p = ex.dalloc(u.bytes ? u.bytes : 4);
        if (!p) { set_error("device allocation of %zu bytes failed", u.bytes); return TS_E_NOMEM; }
        c->dev_allocs.push_back(p);
        TSG_HIP(hipMemcpyAsync(p, u.src, u.bytes, hipMemcpyHostToDevice, ex.stream));
        *u.dst = (const int *)p;
    }
    TSG_HIP(hipStreamSynchronize(ex.stream));
    return TS_OK;
}

namespace {

// Canonical form of a variable set under the QC shift v = jz + c -> jz + (c+t)
// mod z: the lexicographically smallest sorted image.  Its first element is an
// image of an element of the lowest block column at offset 0, so only the shifts
// that map such an element to offset 0 can produce it.
void canon_set(const int32_t *p, int k, int z, std::vector<int32_t> &best, std::vector<int32_t> &tmp) {
    int jmin = INT32_MAX;
    for (int i = 0; i < k; ++i) jmin = std::min(jmin, p[i] / z);
    best.assign(p, p + k);
    std::sort(best.begin(), best.end());
    bool have = false;
    for (int i = 0; i < k; ++i) {
        if (p[i] / z != jmin) continue;
        const int t = (z - p[i] % z) % z;
        tmp.resize(k);
        for (int q = 0; q < k; ++q) tmp[q] = (p[q] / z) * z + (p[q] % z + t) % z;
        std::sort(tmp.begin(), tmp.end());
        if (!have || tmp < best) {
            best = tmp;
            have = true;
        }
    }
}

}  // namespace

// Impulse pattern families drawn from the depth-3 impulse tree of Section III
// (VN1-CN1-VN2-CN2-VN3): single roots, pairs of variables at Tanner distance 2
// or 4, and the variable sets of tree paths v1-c-v2-c'-v3 with c != c'.  With
// TS_PAT_QC_ORBITS only the patterns equal to their canonical QC form.
int64_t make_patterns(const ts_code *c, int kind, int32_t *out, int64_t cap) {
    if (kind & TS_PAT_QC_ORBITS) {
        const int base = kind & 0xff;
        if (c->z <= 0 || base < 1 || base > 3 || (kind & ~(0xff | TS_PAT_QC_ORBITS))) return -1;
        const int64_t n = make_patterns(c, base, nullptr, 0);
        std::vector<int32_t> all((size_t)n * base);
        make_patterns(c, base, all.data(), n);
        std::vector<int32_t> best, tmp;
        int64_t cnt = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int32_t *p = all.data() + i * base;   // sorted ascending
            canon_set(p, base, c->z, best, tmp);
            if (!std::equal(best.begin(), best.end(), p)) continue;
            if (cnt < cap) std::memcpy(out + cnt * base, p, base * 4);
            ++cnt;
        }
        return cnt;
    }
    const int n = c->n;
    auto checks_of = [&](int v, auto &&f) {
        for (int64_t p = c->vptr[v]; p < c->vptr[v + 1]; ++p) f(c->vchk[p]);
    };
    auto vars_of = [&](int ch, auto &&f) {
        for (int64_t q = c->row_ptr[ch]; q < c->row_ptr[ch + 1]; ++q) f(c->col[q]);
    };
    int64_t cnt = 0;
    if (kind == TS_PAT_SINGLES) {
        for (int v = 0; v < n; ++v) {
            if (cnt < cap) out[cnt] = v;
            ++cnt;
        }
        return cnt;
    }
    if (kind == TS_PAT_PAIRS) {
        std::vector<int> stamp(n, -1), ring1;
        std::vector<int> near;
        for (int u = 0; u < n; ++u) {
            ring1.clear();
            near.clear();
            stamp[u] = u;
            checks_of(u, [&](int ch) {
                vars_of(ch, [&](int w) {
                    if (stamp[w] != u) { stamp[w] = u; ring1.push_back(w); near.push_back(w); }
                });
            });
            for (int w : ring1)
                checks_of(w, [&](int ch) {
                    vars_of(ch, [&](int x) {
                        if (stamp[x] != u) { stamp[x] = u; near.push_back(x); }
                    });
                });
            std::sort(near.begin(), near.end());
            for (int v : near)
                if (v > u) {
                    if (cnt < cap) { out[2 * cnt] = u; out[2 * cnt + 1] = v; }
                    ++cnt;
                }
        }
        return cnt;
    }
    if (kind == TS_PAT_TRIPLES) {
        std::vector<std::array<int32_t, 3>> all;
        for (int v1 = 0; v1 < n; ++v1)
            checks_of(v1, [&](int ch) {
                vars_of(ch, [&](int v2) {
                    if (v2 == v1) return;
                    checks_of(v2, [&](int ch2) {
                        if (ch2 == ch) return;
                        vars_of(ch2, [&](int v3) {
                            if (v3 == v1 || v3 == v2) return;
                            std::array<int32_t, 3> t{v1, v2, v3};
                            std::sort(t.begin(), t.end());
                            all.push_back(t);
                        });
                    });
                });
            });
        std::sort(all.begin(), all.end());
        all.erase(std::unique(all.begin(), all.end()), all.end());
        for (auto &t : all) {
            if (cnt < cap) std::memcpy(out + 3 * cnt, t.data(), 12);
            ++cnt;
        }
        return cnt;
    }
    return -1;
}

}  // namespace tsg
