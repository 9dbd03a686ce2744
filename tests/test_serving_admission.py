"""Host logic of admission by footprint (no GPU): slots are created only while the
budget allows, idle slots of the same class are reused, idle slots of other classes
are evicted least recently used first, and a request that cannot fit is refused."""
from paper_2601_01437_amd.serving import FootprintAdmission, Slot, estimate_system_bytes


class _Fake:
    def __init__(self, sizes):
        self.sizes = sizes        # key -> bytes of a new slot
        self.log = []

    def create(self, spec, room):
        b = self.sizes[spec]
        if b > room:
            return b
        self.log.append(("create", spec))
        return Slot(spec, system=None, theta=None, nbytes=b)

    def destroy(self, slot):
        self.log.append(("destroy", slot.key))


def test_budget_reuse_and_lru_eviction():
    f = _Fake({"a": 40, "b": 50, "c": 70, "d": 200})
    adm = FootprintAdmission(100, f.create, f.destroy)
    a1 = adm.acquire("a", "a", 40)
    b1 = adm.acquire("b", "b", 50)
    assert a1 is not None and b1 is not None and adm.used == 90
    # a second "a" slot does not fit while both are held
    assert adm.acquire("a", "a", 40) is None
    adm.release(a1, now=1.0)
    # the idle "a" slot is reused, not recreated
    assert adm.acquire("a", "a", 40) is a1 and adm.reused == 1
    adm.release(a1, now=2.0)
    adm.release(b1, now=3.0)
    # "c" needs 70: the least recently used idle slot ("a", then "b") is evicted
    c1 = adm.acquire("c", "c", 70)
    assert c1 is not None
    assert ("destroy", "a") in f.log and ("destroy", "b") in f.log
    assert f.log.index(("destroy", "a")) < f.log.index(("destroy", "b"))
    assert adm.used == 70 and adm.peak <= 100
    # a class whose estimate exceeds the budget is refused without evicting anything
    adm.release(c1, now=4.0)
    assert adm.acquire("d", "d", 200) is None
    assert adm.used == 70


def test_same_class_idle_slot_is_not_evicted_for_itself():
    f = _Fake({"a": 60})
    adm = FootprintAdmission(100, f.create, f.destroy)
    a1 = adm.acquire("a", "a", 60)
    a2 = adm.acquire("a", "a", 60)
    assert a1 is not None and a2 is None
    adm.release(a1, now=1.0)
    assert adm.acquire("a", "a", 60) is a1


def test_first_creation_learns_the_exact_size():
    # the estimate says 10 bytes, the slot needs 60: the first try reports 60,
    # room is made for 60 and the second try succeeds
    f = _Fake({"a": 50, "b": 60})
    adm = FootprintAdmission(100, f.create, f.destroy)
    a1 = adm.acquire("a", "a", 50)
    adm.release(a1, now=1.0)
    b1 = adm.acquire("b", "b", 10)
    assert b1 is not None and ("destroy", "a") in f.log
    assert adm.known["b"] == 60 and adm.used == 60


def test_estimate_grows_with_the_set():
    assert estimate_system_bytes(20, 10, 10, 1 << 20) > estimate_system_bytes(20, 10, 10, 1 << 14)
    # full spaces carry the string tables
    assert estimate_system_bytes(12, 6, 6, None) > 16 * 853776
