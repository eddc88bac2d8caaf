"""Brute-force linear-scan model of the table semantics (pins the oracle on tiny inputs).

A plain Python list of [key, value] pairs searched front to back: a different
data structure and a different algorithm from the oracle's hash map, so a
mistake in either shows up as a disagreement.  Statuses: 0 OK, 1 DUPLICATE,
2 FULL, 3 INVALID_KEY, 4 NOT_FOUND.
"""

RESERVED = (0, 0xFFFFFFFF)


class BruteTable:
    def __init__(self, kind: int, capacity: int):
        self.kind, self.capacity, self.pairs = kind, capacity, []

    def _find(self, k):
        for idx, (pk, _) in enumerate(self.pairs):
            if pk == k:
                return idx
        return -1

    def insert(self, keys, values=None):
        out = []
        for i, k in enumerate(keys):
            k = int(k)
            if k in RESERVED:
                out.append(3)
                continue
            if self.kind == 1:  # multi-value: always a new pair
                if len(self.pairs) < self.capacity:
                    self.pairs.append([k, int(values[i])])
                    out.append(0)
                else:
                    out.append(2)
                continue
            idx = self._find(k)
            if idx >= 0:
                if self.kind == 0:
                    self.pairs[idx][1] = int(values[i])
                else:
                    self.pairs[idx][1] = (self.pairs[idx][1] + 1) % (1 << 32)
                out.append(1)
            elif len(self.pairs) < self.capacity:
                self.pairs.append([k, int(values[i]) if self.kind == 0 else 1])
                out.append(0)
            else:
                out.append(2)
        return out

    def retrieve(self, keys):
        vals, found = [], []
        for k in keys:
            k = int(k)
            hits = [v for pk, v in self.pairs if pk == k and k not in RESERVED]
            if self.kind == 1:
                vals.append(len(hits))
                found.append(1 if hits else 0)
            else:
                vals.append(hits[0] if hits else 0)
                found.append(1 if hits else 0)
        return vals, found

    def erase(self, keys):
        out = []
        for k in keys:
            k = int(k)
            if k in RESERVED:
                out.append(3)
                continue
            before = len(self.pairs)
            self.pairs = [p for p in self.pairs if p[0] != k]
            out.append(0 if len(self.pairs) < before else 4)
        return out

    def retrieve_all(self, keys):
        offsets, values = [0], []
        for k in keys:
            k = int(k)
            seg = sorted(v for pk, v in self.pairs if pk == k and k not in RESERVED)
            values.extend(seg)
            offsets.append(offsets[-1] + len(seg))
        return offsets, values

    def size(self):
        return len(self.pairs)

    def num_keys(self):
        seen = []
        for pk, _ in self.pairs:
            if pk not in seen:
                seen.append(pk)
        return len(seen)

    def contents(self):
        """Every stored (key, value) pair (one per key for single-value / counting), sorted."""
        return sorted((pk, v) for pk, v in self.pairs)
