// graph.cpp -- graph ingestion (Eq. 2-3: couplings J, biases h).
//
// Two phases so that a server can prepare graphs on worker threads while
// its scheduler keeps the device busy:
//   host_graph_from_edges / host_graph_from_csr  (CPU only)
//       validate, build the symmetric CSR with rows sorted by column, the
//       statistics (W_total, mean(s_i), bounds) and the packed edge
//       encodings the kernels read;
//   upload_graph  (device)
//       copy the arrays to the context's device.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "engine.hpp"
#include "psa.h"

namespace psa {

namespace {

// Sort each row by column; reject diagonal entries and repeated columns.
psa_status canonical_rows(int32_t n, const std::vector<int64_t> &row_ptr,
                          std::vector<int32_t> &col, std::vector<int32_t> &val) {
    std::vector<std::pair<int32_t, int32_t>> tmp;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t b = row_ptr[i], e = row_ptr[i + 1];
        tmp.clear();
        for (int64_t p = b; p < e; ++p) tmp.emplace_back(col[p], val[p]);
        std::sort(tmp.begin(), tmp.end());
        for (size_t k = 0; k < tmp.size(); ++k) {
            if (tmp[k].first == i) {
                set_error("graph: self loop at p-bit " + std::to_string(i));
                return PSA_EINVAL;
            }
            if (k > 0 && tmp[k].first == tmp[k - 1].first) {
                set_error("graph: repeated pair (" + std::to_string(i) + ", " +
                          std::to_string(tmp[k].first) + ")");
                return PSA_EINVAL;
            }
            col[b + static_cast<int64_t>(k)] = tmp[k].first;
            val[b + static_cast<int64_t>(k)] = tmp[k].second;
        }
    }
    return PSA_OK;
}

// Statistics, bounds, padding and packed encodings of a canonical CSR.
psa_status finish_host_graph(int32_t n, const std::vector<int64_t> &row_ptr,
                             std::vector<int32_t> &&col, std::vector<int32_t> &&val,
                             const int32_t *h, HostGraph *out) {
    const int64_t nnz = row_ptr[n];
    if (nnz >= (int64_t{1} << 31)) {
        set_error("graph: more than 2^31 - 1 stored couplings");
        return PSA_EUNSUPPORTED;
    }
    psa_graph_info info{};
    info.n = n;
    info.nnz = nnz;
    info.edges = nnz / 2;
    int64_t w2 = 0;
    int64_t max_field = 0;
    int32_t max_deg = 0;
    bool unit = true;
    double sum_s = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t s1 = 0, s2 = 0, absrow = h ? std::llabs(static_cast<int64_t>(h[i])) : 0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const int64_t J = val[p];
            s1 += J;
            s2 += J * J;
            absrow += std::llabs(J);
            if (J != 1 && J != -1) unit = false;
        }
        w2 += s1;
        max_field = std::max(max_field, absrow);
        max_deg = std::max<int32_t>(max_deg, static_cast<int32_t>(row_ptr[i + 1] - row_ptr[i]));
        // s_i = sqrt((n-1) Var(J_i,:)), population variance over the n
        // entries of the dense row: Var = (n s2 - s1^2) / n^2.
        const int64_t num = static_cast<int64_t>(n) * s2 - s1 * s1;
        const double var =
            static_cast<double>(num) / (static_cast<double>(n) * static_cast<double>(n));
        sum_s += sqrt(static_cast<double>(n - 1) * var);
    }
    if (max_field >= (int64_t{1} << 24)) {
        set_error("graph: max_i |h_i| + sum_j |J_ij| must be < 2^24");
        return PSA_EINVAL;
    }
    info.w_total = -(w2 / 2);
    info.max_abs_field = static_cast<int32_t>(max_field);
    info.max_degree = max_deg;
    info.unit_weights = (unit && nnz > 0) ? 1 : 0;
    info.mean_s = sum_s / static_cast<double>(n);

    HostGraph g;
    g.info = info;
    g.n = n;
    g.n4 = (n + 3) / 4 * 4;
    g.nnz = nnz;
    g.w2 = w2;
    g.max_degree = max_deg;
    // row_ptr padded to n4 + 4 entries (empty padding rows), h padded to n4
    g.rp32.assign(static_cast<size_t>(g.n4) + 4, static_cast<int32_t>(nnz));
    for (int32_t i = 0; i <= n; ++i) g.rp32[i] = static_cast<int32_t>(row_ptr[i]);
    g.h.assign(static_cast<size_t>(g.n4), 0);
    if (h)
        for (int32_t i = 0; i < n; ++i) g.h[i] = h[i];
    bool fits16 = true;
    for (int64_t p = 0; p < nnz; ++p)
        if (val[p] < -32768 || val[p] > 32767) fits16 = false;
    if (n <= 65536 && fits16) {
        g.pk32.resize(static_cast<size_t>(nnz));
        for (int64_t p = 0; p < nnz; ++p)
            g.pk32[p] = static_cast<uint32_t>(col[p]) | (static_cast<uint32_t>(val[p]) << 16);
    }
    // 16-bit edge arrays are padded with zeros to a multiple of 8 entries:
    // kernels that stream rows from global memory load them 8 at a time
    const size_t nnz8 = static_cast<size_t>((nnz + 7) / 8 * 8);
    if (n <= 32768 && info.unit_weights) {
        g.pk16.assign(nnz8, 0);
        for (int64_t p = 0; p < nnz; ++p)
            g.pk16[p] = static_cast<uint16_t>((static_cast<uint32_t>(col[p]) << 1) |
                                              (val[p] < 0 ? 1u : 0u));
    }
    if (2 * static_cast<int64_t>(g.n4) <= 65536 && info.unit_weights) {
        g.ux16.assign(nnz8, 0);
        for (int64_t p = 0; p < nnz; ++p)
            g.ux16[p] = static_cast<uint16_t>(col[p] + (val[p] < 0 ? g.n4 : 0));
    }
    if (n <= 32768 && info.unit_weights && max_deg <= 255) {
        // per-task ELL: task m pads its four rows to the longest of them
        const int32_t tasks = g.n4 / 4;
        g.eptr.assign(static_cast<size_t>(tasks) + 1, 0);
        for (int32_t m = 0; m < tasks; ++m) {
            int32_t d = 0;
            for (int32_t p = 0; p < 4; ++p) d = std::max(d, g.rp32[4 * m + p + 1] - g.rp32[4 * m + p]);
            g.eptr[m + 1] = g.eptr[m] + d;
        }
        // an entry is the neighbour's word index with the coupling's sign in
        // bit 31 (shifted out when the index becomes a byte address); past a
        // row's end, the zero word n4
        const uint32_t zero = static_cast<uint32_t>(g.n4);
        g.ell.assign(4 * static_cast<size_t>(g.eptr[tasks]), zero);
        for (int32_t m = 0; m < tasks; ++m)
            for (int32_t p = 0; p < 4; ++p) {
                const int32_t i = 4 * m + p;
                for (int32_t e = g.rp32[i]; e < g.rp32[i + 1]; ++e)
                    g.ell[4 * (static_cast<size_t>(g.eptr[m]) + (e - g.rp32[i])) + p] =
                        static_cast<uint32_t>(col[e]) | (val[e] < 0 ? 0x80000000u : 0u);
            }
    }
    g.col = std::move(col);
    g.val = std::move(val);
    *out = std::move(g);
    return PSA_OK;
}

// Allocate and fill a device copy of src; the bytes are added to *acct.
template <typename T>
psa_status upload(T **dst, const std::vector<T> &src, size_t *acct) {
    *dst = nullptr;
    if (src.empty()) return PSA_OK;
    if (hipMalloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T)) != hipSuccess) {
        *dst = nullptr;
        set_error("graph upload: device allocation failed");
        return PSA_ENOMEM;
    }
    *acct += src.size() * sizeof(T);
    const hipError_t e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error(std::string("graph upload: ") + hipGetErrorString(e));
        return PSA_EHIP;
    }
    return PSA_OK;
}

}  // namespace

void graph_release(psa_graph *g) {
    if (!g) return;
    for (void *p : {static_cast<void *>(g->d_row_ptr), static_cast<void *>(g->d_col),
                    static_cast<void *>(g->d_val), static_cast<void *>(g->d_h),
                    static_cast<void *>(g->d_pk32), static_cast<void *>(g->d_pk16),
                    static_cast<void *>(g->d_ux16), static_cast<void *>(g->d_dense),
                    static_cast<void *>(g->d_ell), static_cast<void *>(g->d_eptr)})
        if (p) (void)hipFree(p);
    psa_ctx *ctx = g->retained ? g->ctx : nullptr;
    delete g;
    if (ctx) ctx_release(ctx);
}

void graph_unref(psa_graph *g) {
    if (!g) return;
    if (g->refs.fetch_sub(1) != 1) return;
    if (g->ctx) {
        (void)hipSetDevice(g->ctx->device);
        (void)hipStreamSynchronize(g->ctx->stream);
        if (g->ctx->stream2) (void)hipStreamSynchronize(g->ctx->stream2);
    }
    graph_release(g);
}

psa_status ensure_dense_matrix(psa_graph *g) {
    if (g->d_dense) return PSA_OK;
    const int32_t n = g->info.n;
    // one shared value -> 1-bit fields; one shared magnitude -> 2-bit fields;
    // otherwise int8 entries
    // (a stored zero coupling takes the int8 encoding, which keeps it zero)
    int32_t mag = 0, val0 = 0;
    bool one_mag = true, one_val = true, first = true;
    for (int32_t v : g->val_host) {
        if (v == 0) {
            one_mag = one_val = false;
            continue;
        }
        const int32_t a = v < 0 ? -v : v;
        if (first) mag = a, val0 = v, first = false;
        one_mag = one_mag && a == mag;
        one_val = one_val && v == val0;
    }
    const int32_t np = one_mag ? (n + 255) / 256 * 256 : (n + 127) / 128 * 128;
    psa_status st;
    if (one_val && !g->val_host.empty()) {
        // 1-bit fields (J = val0 * f), tiled for the step kernel: for each
        // 64-row tile and 256-column chunk, 2 KB in the order the 64 lanes of
        // a wave load them (two 16-byte loads per lane, each load 1 KB
        // contiguous).  Lane l, half H, word j holds row 64 rt + 16 j + l % 16
        // and, of k-step H of the chunk, columns 32 (l / 16) + 0..31: column
        // 32 g + 8 d + q (d = 0..3, q = 0..7) in bit 4q + d, so that operand
        // dword d is (w >> d) & 0x11111111 moved to bit 4q + 1 (fp4 1.0).
        const int32_t nchunks = np / 256;
        std::vector<uint32_t> words(static_cast<size_t>(np) * np / 32, 0u);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = g->row_ptr_host[i]; p < g->row_ptr_host[i + 1]; ++p) {
                const int32_t k = g->col_host[p];
                const int32_t rt = i >> 6, rb = (i >> 4) & 3, lr = i & 15;
                const int32_t c = k >> 8, ks = (k >> 7) & 1, grp = (k >> 5) & 3;
                const int32_t d = (k >> 3) & 3, q = k & 7;
                const int32_t lane = grp * 16 + lr;
                const size_t at = ((((static_cast<size_t>(rt) * nchunks + c) * 2 + ks) * 64 + lane) * 4) + rb;
                words[at] |= 1u << (4 * q + d);
            }
        uint32_t *dev = nullptr;
        if ((st = upload(&dev, words, &g->dense_bytes)) != PSA_OK) return st;
        g->d_dense = dev;
        g->dense_enc = kDenseB1;
        g->dense_scale = val0;
    } else if (one_mag) {
        // 2-bit fields that two masks turn into fp4 operands, tiled for the
        // step kernel: for each 64-row tile and 256-column chunk, 4 KB in the
        // order the 64 lanes of a wave load them (four 16-byte loads per
        // lane, each load 1 KB contiguous).  Lane l, quarter Q, word j holds
        // row 64 rt + 16 (2 (Q % 2) + j / 2) + l % 16 and, of k-step Q / 2
        // of the chunk, columns 32 (l / 16) + 16 (j % 2) + 0..15: column
        // 32 g + 8 d + q (d = 0..3, q = 0..7) of the k-step has its nonzero
        // bit at 4q + 1 (d even) or 4q (d odd) and its sign bit two above.
        const int32_t nchunks = np / 256;
        std::vector<uint32_t> words(static_cast<size_t>(np) * np / 16, 0u);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = g->row_ptr_host[i]; p < g->row_ptr_host[i + 1]; ++p) {
                const int32_t k = g->col_host[p];
                const int32_t rt = i >> 6, rb = (i >> 4) & 3, lr = i & 15;
                const int32_t c = k >> 8, ks = (k >> 7) & 1, grp = (k >> 5) & 3;
                const int32_t d = (k >> 3) & 3, q = k & 7;
                const int32_t quarter = ks * 2 + (rb >> 1), j = (rb & 1) * 2 + (d >> 1), lane = grp * 16 + lr;
                const size_t at = ((((static_cast<size_t>(rt) * nchunks + c) * 4 + quarter) * 64 + lane) * 4) + j;
                const int32_t nz = 4 * q + ((d & 1) ? 0 : 1);
                words[at] |= 1u << nz;
                if (g->val_host[p] < 0) words[at] |= 1u << (nz + 2);
            }
        uint32_t *dev = nullptr;
        if ((st = upload(&dev, words, &g->dense_bytes)) != PSA_OK) return st;
        g->d_dense = dev;
        g->dense_enc = kDenseT2;
        g->dense_scale = mag == 0 ? 1 : mag;
    } else {
        if (mag > 127 || std::any_of(g->val_host.begin(), g->val_host.end(),
                                     [](int32_t v) { return v < -127 || v > 127; })) {
            set_error("dense path: a coupling does not fit int8");
            return PSA_EUNSUPPORTED;
        }
        std::vector<int8_t> dense(static_cast<size_t>(np) * np, 0);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = g->row_ptr_host[i]; p < g->row_ptr_host[i + 1]; ++p)
                dense[static_cast<size_t>(i) * np + g->col_host[p]] = static_cast<int8_t>(g->val_host[p]);
        int8_t *dev = nullptr;
        if ((st = upload(&dev, dense, &g->dense_bytes)) != PSA_OK) return st;
        g->d_dense = dev;
        g->dense_enc = kDenseI8;
        g->dense_scale = 1;
    }
    g->np = np;
    return PSA_OK;
}

void release_dense_matrix(psa_graph *g) {
    if (!g->d_dense) return;
    if (g->ctx) {
        (void)hipSetDevice(g->ctx->device);
        (void)hipStreamSynchronize(g->ctx->stream);
        if (g->ctx->stream2) (void)hipStreamSynchronize(g->ctx->stream2);
    }
    (void)hipFree(g->d_dense);
    g->d_dense = nullptr;
    g->dense_bytes = 0;
}

psa_status host_graph_from_edges(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                                 const int32_t *val, const int32_t *h, uint32_t flags,
                                 HostGraph *out) {
    if (!out || n < 1 || m < 0 || (m > 0 && (!u || !v || !val)) ||
        (flags & ~PSA_GRAPH_MAXCUT) != 0) {
        set_error("psa_graph_from_edges: invalid arguments");
        return PSA_EINVAL;
    }
    const bool maxcut = (flags & PSA_GRAPH_MAXCUT) != 0;
    std::vector<int64_t> row_ptr(static_cast<size_t>(n) + 1, 0);
    for (int64_t e = 0; e < m; ++e) {
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) {
            set_error("psa_graph_from_edges: edge " + std::to_string(e) + " out of range");
            return PSA_EINVAL;
        }
        if (u[e] == v[e]) {
            set_error("psa_graph_from_edges: self loop at edge " + std::to_string(e));
            return PSA_EINVAL;
        }
        if (val[e] == std::numeric_limits<int32_t>::min()) {
            set_error("psa_graph_from_edges: edge value out of range");
            return PSA_EINVAL;
        }
        ++row_ptr[u[e] + 1];
        ++row_ptr[v[e] + 1];
    }
    for (int32_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    std::vector<int32_t> col(static_cast<size_t>(row_ptr[n])), vv(static_cast<size_t>(row_ptr[n]));
    std::vector<int64_t> fill(row_ptr.begin(), row_ptr.end() - 1);
    for (int64_t e = 0; e < m; ++e) {
        const int32_t J = maxcut ? -val[e] : val[e];
        col[fill[u[e]]] = v[e];
        vv[fill[u[e]]++] = J;
        col[fill[v[e]]] = u[e];
        vv[fill[v[e]]++] = J;
    }
    psa_status st = canonical_rows(n, row_ptr, col, vv);
    if (st != PSA_OK) return st;
    return finish_host_graph(n, row_ptr, std::move(col), std::move(vv), h, out);
}

psa_status host_graph_from_csr(int32_t n, const int64_t *row_ptr, const int32_t *col,
                               const int32_t *val, const int32_t *h, uint32_t flags,
                               HostGraph *out) {
    if (!out || n < 1 || !row_ptr || (flags & ~PSA_GRAPH_MAXCUT) != 0) {
        set_error("psa_graph_from_csr: invalid arguments");
        return PSA_EINVAL;
    }
    if (row_ptr[0] != 0) {
        set_error("psa_graph_from_csr: row_ptr[0] must be 0");
        return PSA_EINVAL;
    }
    for (int32_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) {
            set_error("psa_graph_from_csr: row_ptr is not non-decreasing");
            return PSA_EINVAL;
        }
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && (!col || !val)) {
        set_error("psa_graph_from_csr: col/val NULL");
        return PSA_EINVAL;
    }
    const bool maxcut = (flags & PSA_GRAPH_MAXCUT) != 0;
    std::vector<int64_t> rp(row_ptr, row_ptr + n + 1);
    std::vector<int32_t> cc(static_cast<size_t>(nnz)), vv(static_cast<size_t>(nnz));
    for (int64_t p = 0; p < nnz; ++p) {
        if (col[p] < 0 || col[p] >= n || val[p] == std::numeric_limits<int32_t>::min()) {
            set_error("psa_graph_from_csr: entry " + std::to_string(p) + " out of range");
            return PSA_EINVAL;
        }
        cc[p] = col[p];
        vv[p] = maxcut ? -val[p] : val[p];
    }
    psa_status st = canonical_rows(n, rp, cc, vv);
    if (st != PSA_OK) return st;
    // symmetry: J_ij == J_ji for every stored entry
    for (int32_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int32_t j = cc[p];
            auto b = cc.begin() + rp[j], e = cc.begin() + rp[j + 1];
            auto it = std::lower_bound(b, e, i);
            if (it == e || *it != i || vv[it - cc.begin()] != vv[p]) {
                set_error("psa_graph_from_csr: CSR is not symmetric at (" + std::to_string(i) +
                          ", " + std::to_string(j) + ")");
                return PSA_EINVAL;
            }
        }
    return finish_host_graph(n, rp, std::move(cc), std::move(vv), h, out);
}

psa_status upload_graph(psa_ctx *ctx, HostGraph &&hg, psa_graph **out) {
    if (hipSetDevice(ctx->device) != hipSuccess) {
        set_error("graph upload: hipSetDevice failed");
        return PSA_EHIP;
    }
    std::unique_ptr<psa_graph, void (*)(psa_graph *)> g(new psa_graph(), graph_release);
    g->ctx = ctx;
    ctx_retain(ctx);
    g->retained = true;
    g->info = hg.info;
    psa_status st;
    if ((st = upload(&g->d_row_ptr, hg.rp32, &g->dev_bytes)) != PSA_OK) return st;
    if ((st = upload(&g->d_col, hg.col, &g->dev_bytes)) != PSA_OK) return st;
    if ((st = upload(&g->d_val, hg.val, &g->dev_bytes)) != PSA_OK) return st;
    if ((st = upload(&g->d_h, hg.h, &g->dev_bytes)) != PSA_OK) return st;
    if ((st = upload(&g->d_pk32, hg.pk32, &g->dev_bytes)) != PSA_OK) return st;
    if ((st = upload(&g->d_pk16, hg.pk16, &g->dev_bytes)) != PSA_OK) return st;
    if ((st = upload(&g->d_ux16, hg.ux16, &g->dev_bytes)) != PSA_OK) return st;
    if ((st = upload(&g->d_ell, hg.ell, &g->dev_bytes)) != PSA_OK) return st;
    if ((st = upload(&g->d_eptr, hg.eptr, &g->dev_bytes)) != PSA_OK) return st;
    g->dev.n = hg.n;
    g->dev.n4 = hg.n4;
    g->dev.nnz = hg.nnz;
    g->dev.max_degree = hg.max_degree;
    g->dev.row_ptr = g->d_row_ptr;
    g->dev.col = g->d_col;
    g->dev.val = g->d_val;
    g->dev.h = g->d_h;
    g->dev.pk32 = g->d_pk32;
    g->dev.pk16 = g->d_pk16;
    g->dev.ux16 = g->d_ux16;
    g->dev.ell = g->d_ell;
    g->dev.eptr = g->d_eptr;
    g->dev.w2 = hg.w2;
    g->row_ptr_host = std::move(hg.rp32);
    g->h_host = std::move(hg.h);
    g->col_host = std::move(hg.col);
    g->val_host = std::move(hg.val);
    *out = g.release();
    return PSA_OK;
}

}  // namespace psa
