"""Seeded sparse inputs: bag-of-words style count matrices given as COO entries.

Like the rest of ``smp_inputs`` this module holds no arithmetic of the method;
it only builds entries (row l, column i, value v) that both the GPU path and
the CPU oracle consume.

The paper's real datasets are sparse count/feature matrices (Section 4,
"Description of datasets"; Table 1): NIPS-BW (word-by-paper counts, 12,419
words, 1,500 papers split into two sets of 750) and URL-reputation
(URL-by-feature, d = 792,145 or 1,603,985 URLs, two sets of n = 10,000
features). They are not available here. A topic model stands in for
them: it gives the skewed word (feature) frequencies, the power-law row and
column degrees and the approximately low-rank co-occurrence A^T B that make
those products interesting.

Generator (``topic_counts``), numpy's seeded PCG64 stream:
  * R topics; topic t's word weights are 1/2 a shared Zipf law over the
    vocabulary (rank^-s, ranks in a random order) plus 1/2 its own Zipf law
    over its own random order of the vocabulary;
  * each document has a length L ~ Poisson(tokens_per_doc) (at least 1) and
    topic weights theta ~ Dirichlet(concentration, ..., concentration);
  * its L tokens are split over the topics by a multinomial draw of theta,
    and each topic's tokens are drawn from that topic's word weights;
  * the entry (document, word) is the number of times the word was drawn, so
    every (document, word) pair occurs once, with a positive integer count.
The two sides of a product share the topics: for a word-by-document pair
(``orient="rows_are_words"``) A and B are two disjoint sets of documents
over one vocabulary (NIPS-BW); for a record-by-feature pair
(``orient="rows_are_docs"``) A and B are two disjoint halves of the feature
vocabulary, seen by the same records (URL-reputation).
"""

import numpy as np


def _zipf_weights(rng, n_vocab, s):
    w = 1.0 / np.arange(1, n_vocab + 1, dtype=np.float64) ** s
    return w[rng.permutation(n_vocab)]


def topic_counts(n_docs, n_vocab, R, tokens_per_doc, zipf_s, concentration, seed, chunk=200_000):
    """(doc, word, count) for n_docs documents over n_vocab words: int64,
    int64, float32 arrays sorted by (doc, word), each pair once."""
    rng = np.random.default_rng(int(seed))
    shared = _zipf_weights(rng, n_vocab, zipf_s)
    shared /= shared.sum()
    cdfs = []
    for _ in range(R):
        own = _zipf_weights(rng, n_vocab, zipf_s)
        phi = 0.5 * shared + 0.5 * own / own.sum()
        c = np.cumsum(phi)
        c /= c[-1]
        cdfs.append(c)
    docs, words, counts = [], [], []
    for d0 in range(0, n_docs, chunk):
        d1 = min(n_docs, d0 + chunk)
        nd = d1 - d0
        L = np.maximum(1, rng.poisson(tokens_per_doc, nd))
        theta = rng.dirichlet(np.full(R, concentration), nd)
        per_topic = rng.multinomial(L, theta)                 # (nd, R)
        keys = []
        for t in range(R):
            cnt = per_topic[:, t]
            tot = int(cnt.sum())
            if tot == 0:
                continue
            doc = np.repeat(np.arange(d0, d1, dtype=np.int64), cnt)
            word = np.searchsorted(cdfs[t], rng.random(tot), side="right").astype(np.int64)
            np.minimum(word, n_vocab - 1, out=word)
            keys.append(doc * n_vocab + word)
        k, c = np.unique(np.concatenate(keys), return_counts=True)
        docs.append(k // n_vocab)
        words.append(k % n_vocab)
        counts.append(c.astype(np.float32))
    return np.concatenate(docs), np.concatenate(words), np.concatenate(counts)


def sparse_pair(cfg, seed):
    """(A, B) for a sparse configuration, each as (rows, cols, vals) COO arrays
    (int64, int32, float32) of a d x n matrix in a seeded random order (the
    entries arrive in arbitrary order)."""
    d, n1, n2 = cfg["d"], cfg["n1"], cfg["n2"]
    rng = np.random.default_rng(int(seed) + 1)
    if cfg["orient"] == "rows_are_words":
        doc, word, cnt = topic_counts(n1 + n2, d, cfg["R"], cfg["tokens_per_doc"], cfg["zipf_s"],
                                      cfg["concentration"], seed)
        ina = doc < n1
        A = (word[ina], doc[ina].astype(np.int32), cnt[ina])
        B = (word[~ina], (doc[~ina] - n1).astype(np.int32), cnt[~ina])
    elif cfg["orient"] == "rows_are_docs":
        doc, feat, cnt = topic_counts(d, n1 + n2, cfg["R"], cfg["tokens_per_doc"], cfg["zipf_s"],
                                      cfg["concentration"], seed)
        ina = feat < n1
        A = (doc[ina], feat[ina].astype(np.int32), cnt[ina])
        B = (doc[~ina], (feat[~ina] - n1).astype(np.int32), cnt[~ina])
    else:
        raise ValueError(f"unknown orientation {cfg['orient']!r}")

    def shuffle(e):
        p = rng.permutation(len(e[0]))
        return tuple(np.ascontiguousarray(x[p]) for x in e)

    return shuffle(A), shuffle(B)


def densify(entries, d, n):
    """The d x n FP32 matrix that COO entries describe (tests only, small sizes)."""
    rows, cols, vals = entries
    X = np.zeros((d, n), dtype=np.float32)
    X[rows, cols] = vals
    return X


# Sparse workloads. m = None means 4 n r ln n with n = max(n1, n2).
SPARSE_CONFIGS = {
    # oracle-size parity case (word-by-document)
    "s1_small": dict(orient="rows_are_words", d=3000, n1=120, n2=150, R=5, tokens_per_doc=300, zipf_s=1.0,
                     concentration=0.3, k=64, r=5, T=10),
    # NIPS-BW shape: 12,419 words x 750 + 750 papers, ~1,270 tokens (~500 distinct words) per paper
    "s2_bow": dict(orient="rows_are_words", d=12_419, n1=750, n2=750, R=20, tokens_per_doc=1270, zipf_s=1.0,
                   concentration=0.2, k=400, r=10, T=10),
    # URL-malicious shape (Table 1): 792,145 records x two sets of 10,000 features, k = 2,000
    "s3_url": dict(orient="rows_are_docs", d=792_145, n1=10_000, n2=10_000, R=20, tokens_per_doc=60, zipf_s=1.1,
                   concentration=0.2, k=2000, r=10, T=10),
}
