// Assembly of the coarsest level's operator on its free unique nodes into
// CSR (host code; plain C++, no device calls).  The assembled matrix is
// sum_e P_e^T A_e P_e restricted to the free nodes (Sec. 2.3, the direct
// stiffness summation Q^T A_L Q, with R dropping Dirichlet nodes), where P_e
// maps element e's local points to unique free nodes.
//
//   E, np     elements and points per element
//   nf        free unique nodes (node ids 0 .. nf-1)
//   uid       [E*np] node id of each local point, -1 on Dirichlet points
//   Ae        [E][np][np] element matrices, Ae[(e*np + q)*np + p] = (A_e)_{qp}
//   row, col, val   the CSR (columns ascending within a row, no duplicates)
//   dinv      1 / diagonal of each row
//
// Each row's columns are the free nodes that share an element with it.  The
// values are summed in a fixed order (element, then row point, then column
// point), so the result does not depend on anything but the inputs.  Returns
// -1 on success, else the first row whose diagonal is not positive.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

namespace semx {

inline int64_t assemble_free_csr(int64_t E, int np, int64_t nf, const int32_t *uid, const double *Ae,
                                 std::vector<int32_t> &row, std::vector<int32_t> &col,
                                 std::vector<double> &val, std::vector<double> &dinv)
{
    row.assign((size_t)nf + 1, 0);
    col.clear();
    {
        // each row's column list with duplicates, then sorted and made unique
        std::vector<int64_t> cnt((size_t)nf + 1, 0);
        for (int64_t e = 0; e < E; ++e) {
            int nfe = 0;
            for (int q = 0; q < np; ++q) nfe += uid[e * np + q] >= 0;
            for (int q = 0; q < np; ++q) {
                const int32_t rq = uid[e * np + q];
                if (rq >= 0) cnt[(size_t)rq + 1] += nfe;
            }
        }
        for (int64_t r = 0; r < nf; ++r) cnt[(size_t)r + 1] += cnt[(size_t)r];
        std::vector<int32_t> all((size_t)cnt[(size_t)nf]);
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int q = 0; q < np; ++q) {
                const int32_t rq = uid[e * np + q];
                if (rq < 0) continue;
                for (int p = 0; p < np; ++p) {
                    const int32_t cp = uid[e * np + p];
                    if (cp >= 0) all[(size_t)fill[(size_t)rq]++] = cp;
                }
            }
        col.reserve(all.size());
        for (int64_t r = 0; r < nf; ++r) {
            auto b = all.begin() + cnt[(size_t)r], en = all.begin() + cnt[(size_t)r + 1];
            std::sort(b, en);
            en = std::unique(b, en);
            col.insert(col.end(), b, en);
            row[(size_t)r + 1] = (int32_t)col.size();
        }
    }
    val.assign(col.size(), 0.0);
    for (int64_t e = 0; e < E; ++e)
        for (int q = 0; q < np; ++q) {
            const int32_t rq = uid[e * np + q];
            if (rq < 0) continue;
            const int32_t *cb = col.data() + row[(size_t)rq], *ce = col.data() + row[(size_t)rq + 1];
            for (int p = 0; p < np; ++p) {
                const int32_t cp = uid[e * np + p];
                if (cp < 0) continue;
                val[(size_t)(std::lower_bound(cb, ce, cp) - col.data())] += Ae[(e * np + q) * np + p];
            }
        }
    dinv.assign((size_t)nf, 0.0);
    for (int64_t r = 0; r < nf; ++r) {
        const int32_t *cb = col.data() + row[(size_t)r], *ce = col.data() + row[(size_t)r + 1];
        const int32_t *d = std::lower_bound(cb, ce, (int32_t)r);
        const double diag = (d != ce && *d == r) ? val[(size_t)(d - col.data())] : 0.0;
        if (!(diag > 0.0)) return r;
        dinv[(size_t)r] = 1.0 / diag;
    }
    return -1;
}

}  // namespace semx
